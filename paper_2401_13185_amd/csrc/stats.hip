// Column statistics of the validation blocks and of the training partitions.
//
//  * per validation block V_p (Algorithm 7 steps 10, 17, 19): the FP64 sums
//    and sums of squares of the pivot-shifted values and the raw minimum and
//    maximum (for an exact "column constant over T_p" test), combined in a
//    fixed order from the per-chunk partials of the pack pass, so results
//    are deterministic.  The shift c (one per column) keeps the sums of
//    squares of Lemma 12 small, so the variance form does not cancel on
//    columns with a large mean; every output is invariant to c.
//  * per training partition T_p: the downdates of Lemma 14 and Lemma 7, the
//    deviation by Lemma 12 with divisor |T_p| - ddof, and the zero -> 1 rule
//    of Algorithm 7 step 24 read as "column constant over T_p".
#include <cmath>

#include "internal.h"

namespace cvg {
namespace {

// fold layout: [4][P][W]
__global__ __launch_bounds__(256) void stats_reduce_kernel(const double* __restrict__ part,
                                                           int64_t n_chunks,
                                                           const int32_t* __restrict__ cbeg,
                                                           int32_t P, int64_t W,
                                                           double* __restrict__ fold) {
  const int64_t j = (int64_t)blockIdx.y * blockDim.x + threadIdx.x;
  const int32_t p = blockIdx.x;
  if (j >= W) return;
  const int64_t ps = n_chunks * W;
  double s = 0.0, q = 0.0, mn = INFINITY, mx = -INFINITY;
  for (int32_t c = cbeg[p]; c < cbeg[p + 1]; ++c) {
    s += part[0 * ps + (int64_t)c * W + j];
    q += part[1 * ps + (int64_t)c * W + j];
    mn = fmin(mn, part[2 * ps + (int64_t)c * W + j]);
    mx = fmax(mx, part[3 * ps + (int64_t)c * W + j]);
  }
  const int64_t fs = (int64_t)P * W;
  fold[0 * fs + (int64_t)p * W + j] = s;
  fold[1 * fs + (int64_t)p * W + j] = q;
  fold[2 * fs + (int64_t)p * W + j] = mn;
  fold[3 * fs + (int64_t)p * W + j] = mx;
}

// One thread per column; loops over folds in order (deterministic).
// scratch: [2][P][W] suffix minima / maxima of the fold extrema.
__global__ __launch_bounds__(256) void train_stats_kernel(
    const double* __restrict__ fold, const int64_t* __restrict__ offsets, int32_t P, int64_t N,
    int64_t W, int ddof, const double* __restrict__ pivot, double* __restrict__ scratch,
    double* __restrict__ tr_sum, double* __restrict__ tr_mean, double* __restrict__ tr_std,
    double* __restrict__ tr_mu, uint8_t* __restrict__ tr_const, int64_t* __restrict__ ntrain) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= W) return;
  const int64_t fs = (int64_t)P * W;
  const double* fsum = fold;
  const double* fsq = fold + fs;
  const double* fmn = fold + 2 * fs;
  const double* fmx = fold + 3 * fs;
  double* smn = scratch;
  double* smx = scratch + fs;
  // totals over all rows (Algorithm 7 step 4, shifted) and suffix extrema
  double S = 0.0, Q = 0.0;
  for (int32_t p = 0; p < P; ++p) {
    S += fsum[(int64_t)p * W + j];
    Q += fsq[(int64_t)p * W + j];
  }
  double run_mn = INFINITY, run_mx = -INFINITY;
  for (int32_t p = P - 1; p >= 0; --p) {
    smn[(int64_t)p * W + j] = run_mn;  // extrema over folds > p
    smx[(int64_t)p * W + j] = run_mx;
    run_mn = fmin(run_mn, fmn[(int64_t)p * W + j]);
    run_mx = fmax(run_mx, fmx[(int64_t)p * W + j]);
  }
  const double c = pivot[j];
  double pre_mn = INFINITY, pre_mx = -INFINITY;
  for (int32_t p = 0; p < P; ++p) {
    const int64_t e = (int64_t)p * W + j;
    const int64_t nv = offsets[p + 1] - offsets[p];
    const int64_t nt = N - nv;
    const double NT = (double)nt;
    const double sT = S - fsum[e];                 // Lemma 14
    const double qT = Q - fsq[e];
    const double mu = sT / NT;                     // training mean of shifted values
    const double tmn = fmin(pre_mn, smn[e]);
    const double tmx = fmax(pre_mx, smx[e]);
    const bool constant = tmn == tmx;
    double sd;
    if (nt - ddof < 1) {
      sd = NAN;                                    // not scalable (Definition 6)
    } else if (constant) {
      sd = 1.0;                                    // Algorithm 7 step 24
    } else {
      // Lemma 12 on shifted values: (|T| mu^2 + sum x^2 - 2 mu sum x) / (|T| - ddof)
      double var = (NT * mu * mu + qT - 2.0 * mu * sT) / (double)(nt - ddof);
      sd = sqrt(var > 0.0 ? var : 0.0);
      if (sd == 0.0) sd = 1.0;
    }
    tr_sum[e] = sT;
    tr_mean[e] = constant ? 0.0 : mu;
    tr_std[e] = sd;
    tr_mu[e] = constant ? tmn : c + mu;
    tr_const[e] = constant ? 1 : 0;
    if (j == 0) ntrain[p] = nt;
    pre_mn = fmin(pre_mn, fmn[e]);
    pre_mx = fmax(pre_mx, fmx[e]);
  }
}

__global__ void fold_stats_kernel(const double* __restrict__ tr_mu,
                                  const double* __restrict__ tr_std, int32_t p, int64_t K,
                                  int64_t M, double* mx, double* sx, double* my, double* sy) {
  const int64_t W = K + M;
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= W) return;
  const double m = tr_mu[(int64_t)p * W + j];
  const double s = tr_std[(int64_t)p * W + j];
  if (j < K) {
    if (mx) mx[j] = m;
    if (sx) sx[j] = s;
  } else {
    if (my) my[j - K] = m;
    if (sy) sy[j - K] = s;
  }
}

}  // namespace

void launch_stats_reduce(const double* part, int64_t n_chunks, const int32_t* chunk_begin,
                         int32_t P, int64_t W, double* fold, hipStream_t s) {
  dim3 grid((unsigned)P, (unsigned)((W + 255) / 256));
  stats_reduce_kernel<<<grid, 256, 0, s>>>(part, n_chunks, chunk_begin, P, W, fold);
  CVG_LAUNCH_CHECK();
}

void launch_train_stats(const double* fold, const int64_t* offsets, int32_t P, int64_t N,
                        int64_t W, int ddof, const double* pivot, double* scratch,
                        double* tr_sum, double* tr_mean, double* tr_std, double* tr_mu,
                        uint8_t* tr_const, int64_t* ntrain, hipStream_t s) {
  train_stats_kernel<<<(unsigned)((W + 255) / 256), 256, 0, s>>>(
      fold, offsets, P, N, W, ddof, pivot, scratch, tr_sum, tr_mean, tr_std, tr_mu, tr_const,
      ntrain);
  CVG_LAUNCH_CHECK();
}

void launch_fold_stats(const double* tr_mu, const double* tr_std, int32_t p, int64_t K,
                       int64_t M, double* mx, double* sx, double* my, double* sy, hipStream_t s) {
  fold_stats_kernel<<<(unsigned)((K + M + 255) / 256), 256, 0, s>>>(tr_mu, tr_std, p, K, M, mx,
                                                                     sx, my, sy);
  CVG_LAUNCH_CHECK();
}

}  // namespace cvg
