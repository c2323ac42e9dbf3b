// Column statistics of the validation blocks and of the training partitions.
//
//  * pivot: one shift c_j per column of Z = [X | Y] (the FP64 mean of the
//    first min(N, 256) rows, rounded to the input precision in the mixed
//    modes).  Every output is invariant to c: centred results do not depend
//    on a common shift, and uncentred ones are rebuilt exactly from the
//    shifted sums.  Shifting keeps the sums of squares of Lemma 12 small, so
//    the variance form does not cancel on columns with a large mean.
//  * per validation block V_p (Algorithm 7 steps 10, 17, 19): FP64 sums and
//    sums of squares of the shifted values, and the raw minimum and maximum
//    (used for an exact "column constant over T_p" test).  Rows are read in
//    fold-aligned chunks through the fold permutation; chunk partials are
//    combined in a fixed order, so results are deterministic.
//  * per training partition T_p: the downdates of Lemma 14 and Lemma 7, the
//    deviation by Lemma 12 with divisor |T_p| - ddof, and the zero -> 1 rule
//    of Algorithm 7 step 24 read as "column constant over T_p".
#include <cmath>

#include "internal.h"

namespace cvg {
namespace {

template <typename T>
__device__ inline double zval(const T* __restrict__ X, const T* __restrict__ Y, int64_t K,
                              int64_t M, int64_t row, int64_t j) {
  return j < K ? (double)X[row * K + j] : (double)Y[row * M + (j - K)];
}

template <typename T>
__global__ __launch_bounds__(256) void pivot_kernel(const T* __restrict__ X,
                                                    const T* __restrict__ Y, int64_t rows,
                                                    int64_t K, int64_t M, int round_f32,
                                                    double* __restrict__ pivot) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= K + M) return;
  double s = 0.0;
  for (int64_t r = 0; r < rows; ++r) s += zval(X, Y, K, M, r, j);
  double c = s / (double)rows;
  if (round_f32) c = (double)(float)c;
  pivot[j] = c;
}

constexpr int kStatCols = 256;
constexpr int kUnroll = 8;

// part layout: [4][n_chunks][W] = sum, sumsq, min, max
template <typename T>
__global__ __launch_bounds__(kStatCols) void colstats_kernel(
    const T* __restrict__ X, const T* __restrict__ Y, int64_t K, int64_t M,
    const int32_t* __restrict__ perm, const RowChunk* __restrict__ chunks, int64_t n_chunks,
    const double* __restrict__ pivot, double* __restrict__ part) {
  const int64_t W = K + M;
  const int64_t j = (int64_t)blockIdx.y * kStatCols + threadIdx.x;
  const int64_t c = blockIdx.x;
  if (j >= W) return;
  const RowChunk ch = chunks[c];
  const double piv = pivot[j];
  double s = 0.0, q = 0.0, mn = INFINITY, mx = -INFINITY;
  int64_t r = ch.r0;
  for (; r + kUnroll <= ch.r1; r += kUnroll) {
    double v[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) v[u] = zval(X, Y, K, M, (int64_t)perm[r + u], j);
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const double d = v[u] - piv;
      s += d;
      q = fma(d, d, q);
      mn = fmin(mn, v[u]);
      mx = fmax(mx, v[u]);
    }
  }
  for (; r < ch.r1; ++r) {
    const double x = zval(X, Y, K, M, (int64_t)perm[r], j);
    const double d = x - piv;
    s += d;
    q = fma(d, d, q);
    mn = fmin(mn, x);
    mx = fmax(mx, x);
  }
  const int64_t stride = n_chunks * W;
  part[0 * stride + c * W + j] = s;
  part[1 * stride + c * W + j] = q;
  part[2 * stride + c * W + j] = mn;
  part[3 * stride + c * W + j] = mx;
}

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

void launch_pivot(const void* X, const void* Y, cvgram_dtype dt, bool round_f32, int64_t N,
                  int64_t K, int64_t M, double* pivot, hipStream_t s) {
  const int64_t rows = N < 256 ? N : 256;
  const unsigned blocks = (unsigned)((K + M + 255) / 256);
  if (dt == CVGRAM_F64)
    pivot_kernel<double><<<blocks, 256, 0, s>>>((const double*)X, (const double*)Y, rows, K, M,
                                                round_f32 ? 1 : 0, pivot);
  else
    pivot_kernel<float><<<blocks, 256, 0, s>>>((const float*)X, (const float*)Y, rows, K, M,
                                               round_f32 ? 1 : 0, pivot);
  CVG_LAUNCH_CHECK();
}

void launch_colstats(const void* X, const void* Y, cvgram_dtype dt, int64_t K, int64_t M,
                     const int32_t* perm, const RowChunk* chunks, int64_t n_chunks,
                     const double* pivot, double* part, hipStream_t s) {
  dim3 grid((unsigned)n_chunks, (unsigned)((K + M + kStatCols - 1) / kStatCols));
  if (dt == CVGRAM_F64)
    colstats_kernel<double><<<grid, kStatCols, 0, s>>>((const double*)X, (const double*)Y, K, M,
                                                       perm, chunks, n_chunks, pivot, part);
  else
    colstats_kernel<float><<<grid, kStatCols, 0, s>>>((const float*)X, (const float*)Y, K, M,
                                                      perm, chunks, n_chunks, pivot, part);
  CVG_LAUNCH_CHECK();
}

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
