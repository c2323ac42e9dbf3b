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
#include <climits>
#include <cmath>

#include "internal.h"

namespace cvg {
namespace {

// fold layout: [4][P][W].  items: (prob, fold); grid.y = blocks of 64
// columns.  The 4 waves of a workgroup take every 4th chunk of the fold and
// are combined in wave order (deterministic).
__global__ __launch_bounds__(256) void stats_reduce_kernel(const ProbDesc* __restrict__ pds,
                                                           const Item* __restrict__ items) {
  __shared__ double sh[4][4][64];
  const Item it = items[blockIdx.x];
  const ProbDesc& pd = pds[it.prob];
  const int32_t p = it.a;
  const int64_t W = pd.W;
  if ((int64_t)blockIdx.y * 64 >= W) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t j = (int64_t)blockIdx.y * 64 + lane;
  const int64_t ps = pd.n_chunks * W;
  const CVG_GLOBAL double* part = gmem((const double*)pd.part);
  const CVG_GLOBAL int32_t* chunk_begin = gmem(pd.chunk_begin);
  double s = 0.0, q = 0.0, mn = INFINITY, mx = -INFINITY;
  if (j < W) {
    const int32_t c1 = chunk_begin[p + 1];
#pragma unroll 4
    for (int32_t c = chunk_begin[p] + w; c < c1; c += 4) {
      s += part[0 * ps + (int64_t)c * W + j];
      q += part[1 * ps + (int64_t)c * W + j];
      mn = fmin(mn, part[2 * ps + (int64_t)c * W + j]);
      mx = fmax(mx, part[3 * ps + (int64_t)c * W + j]);
    }
  }
  sh[0][w][lane] = s;
  sh[1][w][lane] = q;
  sh[2][w][lane] = mn;
  sh[3][w][lane] = mx;
  __syncthreads();
  if (w == 0 && j < W) {
    for (int k = 1; k < 4; ++k) {
      s += sh[0][k][lane];
      q += sh[1][k][lane];
      mn = fmin(mn, sh[2][k][lane]);
      mx = fmax(mx, sh[3][k][lane]);
    }
    const int64_t fs = (int64_t)pd.P * W;
    CVG_GLOBAL double* fold = gmem(pd.fold);
    fold[0 * fs + (int64_t)p * W + j] = s;
    fold[1 * fs + (int64_t)p * W + j] = q;
    fold[2 * fs + (int64_t)p * W + j] = mn;
    fold[3 * fs + (int64_t)p * W + j] = mx;
  }
}

// Fused-path problems (many small folds, no per-fold chunks): the same four
// per-fold quantities read directly from the fold's rows, X and Y gathered
// through the permutation and shifted by the pivot exactly as in the pack
// pass.  items: (prob, first fold, end fold); grid.y = blocks of 64 columns.
// Wave w takes folds f0 + w, f0 + w + 4, ... and sums each in row order.
template <typename T>
__global__ __launch_bounds__(256) void fold_sums_rows_kernel(const ProbDesc* __restrict__ pds,
                                                             const Item* __restrict__ items) {
  const Item it = items[blockIdx.x];
  const ProbDesc& pd = pds[it.prob];
  const int64_t W = pd.W, K = pd.K, M = pd.M;
  if ((int64_t)blockIdx.y * 64 >= W) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t j = (int64_t)blockIdx.y * 64 + lane;
  if (j >= W) return;
  const CVG_GLOBAL T* X = gmem((const T*)pd.X);
  const CVG_GLOBAL T* Y = gmem((const T*)pd.Y);
  const CVG_GLOBAL int32_t* perm = gmem(pd.perm);
  const CVG_GLOBAL int64_t* offsets = gmem(pd.offsets);
  CVG_GLOBAL double* fold = gmem(pd.fold);
  const int64_t fs = (int64_t)pd.P * W;
  const double c = gmem((const double*)pd.pivot)[j];
  for (int32_t p = it.a + w; p < it.b; p += 4) {
    double s = 0.0, q = 0.0, mn = INFINITY, mx = -INFINITY;
    const int64_t r1 = offsets[p + 1];
    for (int64_t r = offsets[p]; r < r1; ++r) {
      const int64_t row = perm[r];
      const double x = j < K ? (double)X[row * K + j] : (double)Y[row * M + (j - K)];
      const double d = x - c;
      s += d;
      q = fma(d, d, q);
      mn = fmin(mn, x);
      mx = fmax(mx, x);
    }
    fold[0 * fs + (int64_t)p * W + j] = s;
    fold[1 * fs + (int64_t)p * W + j] = q;
    fold[2 * fs + (int64_t)p * W + j] = mn;
    fold[3 * fs + (int64_t)p * W + j] = mx;
  }
}

// Column totals over all folds and, for the exact constant test, the
// smallest and largest value of each column with the fold holding it and
// the runner-up over the other folds: the extrema over T_p (all folds but p)
// are then available for every p in O(1).
// tot layout: [8][W] = S, Q, min1, argmin (as double), min2, max1, argmax, max2
struct Ext {
  double v1;
  int32_t f1;
  double v2;
};

__device__ inline Ext ext_min(Ext a, Ext b) {
  // smallest value, the lower fold winning ties; runner-up from another fold
  Ext r;
  const bool a_first = a.v1 < b.v1 || (a.v1 == b.v1 && a.f1 <= b.f1);
  r.v1 = a_first ? a.v1 : b.v1;
  r.f1 = a_first ? a.f1 : b.f1;
  r.v2 = fmin(fmin(a.v2, b.v2), a_first ? b.v1 : a.v1);
  return r;
}

__device__ inline Ext ext_max(Ext a, Ext b) {
  Ext r;
  const bool a_first = a.v1 > b.v1 || (a.v1 == b.v1 && a.f1 <= b.f1);
  r.v1 = a_first ? a.v1 : b.v1;
  r.f1 = a_first ? a.f1 : b.f1;
  r.v2 = fmax(fmax(a.v2, b.v2), a_first ? b.v1 : a.v1);
  return r;
}

// Two levels, both in a fixed order (deterministic).  Part: items (prob,
// block of 64 columns, range of kFoldRange folds); the 4 waves take folds
// w, w + 4, ... of the range and are combined in wave order into tot_part.
// Final: items (prob, block of 64 columns); the ranges are combined in
// range order into tot (64 threads, one column each).
__global__ __launch_bounds__(256) void fold_totals_part_kernel(const ProbDesc* __restrict__ pds,
                                                               const Item* __restrict__ items) {
  __shared__ double sS[4][64], sQ[4][64];
  __shared__ Ext sMn[4][64], sMx[4][64];
  const Item it = items[blockIdx.x];
  const ProbDesc& pd = pds[it.prob];
  const int64_t W = pd.W;
  const int32_t P = pd.P;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t j = (int64_t)it.a * 64 + lane;
  const int64_t fs = (int64_t)P * W;
  const int32_t f0 = it.b * kFoldRange;
  const int32_t f1 = f0 + kFoldRange < P ? f0 + kFoldRange : P;
  const CVG_GLOBAL double* fold = gmem((const double*)pd.fold);
  double S = 0.0, Q = 0.0;
  Ext mn{INFINITY, INT32_MAX, INFINITY}, mx{-INFINITY, INT32_MAX, -INFINITY};
  if (j < W) {
#pragma unroll 4
    for (int32_t p = f0 + w; p < f1; p += 4) {
      const int64_t e = (int64_t)p * W + j;
      S += fold[e];
      Q += fold[fs + e];
      mn = ext_min(mn, Ext{fold[2 * fs + e], p, INFINITY});
      mx = ext_max(mx, Ext{fold[3 * fs + e], p, -INFINITY});
    }
  }
  sS[w][lane] = S;
  sQ[w][lane] = Q;
  sMn[w][lane] = mn;
  sMx[w][lane] = mx;
  __syncthreads();
  if (w == 0 && j < W) {
    for (int k = 1; k < 4; ++k) {
      S += sS[k][lane];
      Q += sQ[k][lane];
      mn = ext_min(mn, sMn[k][lane]);
      mx = ext_max(mx, sMx[k][lane]);
    }
    CVG_GLOBAL double* tp = gmem(pd.tot_part) + (int64_t)it.b * 8 * W;
    tp[0 * W + j] = S;
    tp[1 * W + j] = Q;
    tp[2 * W + j] = mn.v1;
    tp[3 * W + j] = (double)mn.f1;
    tp[4 * W + j] = mn.v2;
    tp[5 * W + j] = mx.v1;
    tp[6 * W + j] = (double)mx.f1;
    tp[7 * W + j] = mx.v2;
  }
}

__global__ __launch_bounds__(64) void fold_totals_final_kernel(const ProbDesc* __restrict__ pds,
                                                                const Item* __restrict__ items) {
  const Item it = items[blockIdx.x];
  const ProbDesc& pd = pds[it.prob];
  const int64_t W = pd.W;
  const int64_t j = (int64_t)it.a * 64 + threadIdx.x;
  if (j >= W) return;
  const CVG_GLOBAL double* tp = gmem((const double*)pd.tot_part);
  double S = 0.0, Q = 0.0;
  Ext mn{INFINITY, INT32_MAX, INFINITY}, mx{-INFINITY, INT32_MAX, -INFINITY};
  for (int32_t r = 0; r < pd.n_franges; ++r) {
    const CVG_GLOBAL double* t = tp + (int64_t)r * 8 * W + j;
    S += t[0 * W];
    Q += t[1 * W];
    mn = ext_min(mn, Ext{t[2 * W], (int32_t)t[3 * W], t[4 * W]});
    mx = ext_max(mx, Ext{t[5 * W], (int32_t)t[6 * W], t[7 * W]});
  }
  CVG_GLOBAL double* tot = gmem(pd.tot);
  tot[0 * W + j] = S;
  tot[1 * W + j] = Q;
  tot[2 * W + j] = mn.v1;
  tot[3 * W + j] = (double)mn.f1;
  tot[4 * W + j] = mn.v2;
  tot[5 * W + j] = mx.v1;
  tot[6 * W + j] = (double)mx.f1;
  tot[7 * W + j] = mx.v2;
}

// One thread per (fold, column): Lemma 14 and Lemma 7 downdates, Lemma 12
// on shifted values, and the constant-column rule.  items: (prob, fold);
// grid.y = blocks of 256 columns.
__global__ __launch_bounds__(256) void train_stats_kernel(const ProbDesc* __restrict__ pds,
                                                          const Item* __restrict__ items) {
  const Item it = items[blockIdx.x];
  const ProbDesc& pd = pds[it.prob];
  const int32_t p = it.a;
  const int64_t W = pd.W;
  const int64_t j = (int64_t)blockIdx.y * blockDim.x + threadIdx.x;
  if (j >= W) return;
  const int64_t fs = (int64_t)pd.P * W;
  const int64_t e = (int64_t)p * W + j;
  const CVG_GLOBAL int64_t* offsets = gmem(pd.offsets);
  const int64_t nv = offsets[p + 1] - offsets[p];
  const int64_t nt = pd.N - nv;
  const double NT = (double)nt;
  const CVG_GLOBAL double* tot = gmem((const double*)pd.tot);
  const CVG_GLOBAL double* fold = gmem((const double*)pd.fold);
  const double sT = tot[0 * W + j] - fold[e];             // Lemma 14
  const double qT = tot[1 * W + j] - fold[fs + e];
  const double mu = sT / NT;                              // Lemma 7 (shifted)
  const double tmn = (int32_t)tot[3 * W + j] == p ? tot[4 * W + j] : tot[2 * W + j];
  const double tmx = (int32_t)tot[6 * W + j] == p ? tot[7 * W + j] : tot[5 * W + j];
  const bool constant = tmn == tmx;
  double sd;
  if (nt - pd.ddof < 1) {
    sd = NAN;                                             // not scalable (Definition 6)
  } else if (constant) {
    sd = 1.0;                                             // Algorithm 7 step 24
  } else {
    // Lemma 12 on shifted values: (|T| mu^2 + sum x^2 - 2 mu sum x) / (|T| - ddof)
    const double var = (NT * mu * mu + qT - 2.0 * mu * sT) / (double)(nt - pd.ddof);
    sd = sqrt(var > 0.0 ? var : 0.0);
    if (sd == 0.0) sd = 1.0;
  }
  gmem(pd.tr_sum)[e] = sT;
  gmem(pd.tr_mean)[e] = constant ? 0.0 : mu;
  gmem(pd.tr_std)[e] = sd;
  gmem(pd.tr_mu)[e] = constant ? tmn : gmem((const double*)pd.pivot)[j] + mu;
  gmem(pd.tr_const)[e] = constant ? 1 : 0;
  if (j == 0) gmem(pd.ntrain)[p] = nt;
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

void launch_stats_reduce(const ProbDesc* pd, const Item* fold_items, int64_t n_items,
                         int32_t max_col_blocks64, hipStream_t s) {
  if (n_items <= 0) return;
  dim3 grid((unsigned)n_items, (unsigned)max_col_blocks64);
  stats_reduce_kernel<<<grid, 256, 0, s>>>(pd, fold_items);
  CVG_LAUNCH_CHECK();
}

void launch_fold_sums_rows(cvgram_dtype dt, const ProbDesc* pd, const Item* fold_items,
                           int64_t n_items, int32_t max_col_blocks64, hipStream_t s) {
  if (n_items <= 0) return;
  dim3 grid((unsigned)n_items, (unsigned)max_col_blocks64);
  if (dt == CVGRAM_F64)
    fold_sums_rows_kernel<double><<<grid, 256, 0, s>>>(pd, fold_items);
  else
    fold_sums_rows_kernel<float><<<grid, 256, 0, s>>>(pd, fold_items);
  CVG_LAUNCH_CHECK();
}

void launch_fold_totals(const ProbDesc* pd, const Item* range_items, int64_t n_range_items,
                        const Item* colblock_items, int64_t n_items, hipStream_t s) {
  if (n_range_items <= 0 || n_items <= 0) return;
  fold_totals_part_kernel<<<(unsigned)n_range_items, 256, 0, s>>>(pd, range_items);
  CVG_LAUNCH_CHECK();
  fold_totals_final_kernel<<<(unsigned)n_items, 64, 0, s>>>(pd, colblock_items);
  CVG_LAUNCH_CHECK();
}

void launch_train_stats(const ProbDesc* pd, const Item* fold_items, int64_t n_items,
                        int32_t max_col_blocks256, hipStream_t s) {
  if (n_items <= 0) return;
  dim3 grid((unsigned)n_items, (unsigned)max_col_blocks256);
  train_stats_kernel<<<grid, 256, 0, s>>>(pd, fold_items);
  CVG_LAUNCH_CHECK();
}

void launch_fold_stats(const double* tr_mu, const double* tr_std, int32_t p, int64_t K,
                       int64_t M, double* mx, double* sx, double* my, double* sy, hipStream_t s) {
  fold_stats_kernel<<<(unsigned)((K + M + 255) / 256), 256, 0, s>>>(tr_mu, tr_std, p, K, M, mx,
                                                                     sx, my, sy);
  CVG_LAUNCH_CHECK();
}

}  // namespace cvg
