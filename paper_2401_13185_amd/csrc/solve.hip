// Per-fold ridge regression on the device: B = (A + lambda I)^{-1} R for a
// batch of symmetric positive definite A (K x K) and right-hand sides R
// (K x M), all FP64 and row-major, one per (fold, lambda).  This consumes
// the training products directly (the models the paper names for them,
// Section 1: RR, and OLS for lambda = 0).
//
// Blocked right-looking Cholesky A = L L^T with 32 x 32 blocks:
//   for each block column j
//     diag:   L_jj = chol(A_jj) and its inverse, in LDS (one workgroup per matrix)
//     panel:  L_ij = A_ij L_jj^{-T} for every block row i > j
//     update: A_ik -= L_ij L_kj^T for every j < k <= i (lower triangle)
// then R is overwritten by L^{-T} L^{-1} R with the same blocks (forward and
// backward substitution through the stored inverses of the diagonal blocks,
// one launch for both).
// A matrix whose pivot is not positive (A + lambda I not positive definite)
// sets its flag and continues with NaN.
//
// Arithmetic: FP64 FMA on the vector units; every sum runs in a fixed order
// (deterministic).
#include <cmath>

#include "internal.h"

namespace cvg {
namespace {

constexpr int NB = 32;         // block edge
constexpr int kSolveRows = 128;  // rows of L staged per pass of a substitution update
constexpr int kThreads = 256;  // 8 rows x 32 columns per pass, 4 passes per block

// A + lambda I and a copy of R from the products (p-major, lambda-minor)
__global__ __launch_bounds__(kThreads) void ridge_setup_kernel(
    const double* __restrict__ xtx, const double* __restrict__ xty,
    const double* __restrict__ lambdas, int32_t n_lambda, int64_t K, int64_t M,
    double* __restrict__ A, double* __restrict__ R) {
  const int64_t mat = blockIdx.y;  // fold * n_lambda + lambda
  const int64_t f = mat / n_lambda;
  const double lam = lambdas[mat % n_lambda];
  const int64_t KK = K * K, KM = K * M;
  const CVG_GLOBAL double* src = gmem(xtx) + f * KK;
  CVG_GLOBAL double* dst = gmem(A) + mat * KK;
  for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < KK; e += (int64_t)gridDim.x * kThreads) {
    const int64_t i = e / K, j = e - i * K;
    dst[e] = src[e] + (i == j ? lam : 0.0);
  }
  const CVG_GLOBAL double* rs = gmem(xty) + f * KM;
  CVG_GLOBAL double* rd = gmem(R) + mat * KM;
  for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < KM; e += (int64_t)gridDim.x * kThreads)
    rd[e] = rs[e];
}

// diagonal block j of every matrix: Cholesky in LDS (column by column), the
// inverse of the factor by forward substitution, both written back; blocks
// past K are padded with the identity.  flags[mat] = 1 on a non-positive pivot.
__global__ __launch_bounds__(kThreads) void chol_diag_kernel(double* __restrict__ A,
                                                             double* __restrict__ Linv,
                                                             int32_t* __restrict__ flags,
                                                             int64_t K, int32_t j, int32_t nblk) {
  __shared__ double L[NB][NB + 1];
  __shared__ double I[NB][NB + 1];
  const int64_t mat = blockIdx.x;
  CVG_GLOBAL double* a = gmem(A) + mat * K * K;
  const int t = threadIdx.x, tx = t % NB, ty = t / NB;
  const int64_t r0 = (int64_t)j * NB;
  for (int r = ty; r < NB; r += kThreads / NB) {
    const int64_t i = r0 + r, c = r0 + tx;
    L[r][tx] = (i < K && c < K) ? a[i * K + c] : (r == tx ? 1.0 : 0.0);
  }
  __syncthreads();
  // right-looking on the block: column c finishes, then updates the rest
  for (int c = 0; c < NB; ++c) {
    if (t == 0) {
      const double d = L[c][c];
      if (!(d > 0.0)) flags[mat] = 1;
      L[c][c] = d > 0.0 ? sqrt(d) : NAN;
    }
    __syncthreads();
    if (t > c && t < NB) L[t][c] = L[t][c] / L[c][c];
    __syncthreads();
    for (int r = ty; r < NB; r += kThreads / NB)
      if (r > c && tx > c && tx <= r) L[r][tx] = fma(-L[r][c], L[tx][c], L[r][tx]);
    __syncthreads();
  }
  // inverse of the lower factor, L X = I, by right-looking elimination over
  // the rows of X: at step c row c is divided by the pivot and then removed
  // from the rows below, all 32 x 32 entries in parallel (each entry sums in
  // increasing c, the order of plain forward substitution)
  for (int r = ty; r < NB; r += kThreads / NB) I[r][tx] = r == tx ? 1.0 : 0.0;
  __syncthreads();
  for (int c = 0; c < NB; ++c) {
    if (t < NB) I[c][t] = I[c][t] / L[c][c];
    __syncthreads();
    for (int r = ty; r < NB; r += kThreads / NB)
      if (r > c) I[r][tx] = fma(-L[r][c], I[c][tx], I[r][tx]);
    __syncthreads();
  }
  CVG_GLOBAL double* li = gmem(Linv) + (mat * nblk + j) * NB * NB;
  for (int r = ty; r < NB; r += kThreads / NB) {
    const int64_t i = r0 + r, c = r0 + tx;
    if (i < K && c < K) a[i * K + c] = tx <= r ? L[r][tx] : 0.0;
    li[r * NB + tx] = I[r][tx];
  }
}

// panel: L_ij = A_ij Linv_jj^T for block rows i > j.  grid (matrices, rows below)
__global__ __launch_bounds__(kThreads) void chol_panel_kernel(double* __restrict__ A,
                                                              const double* __restrict__ Linv,
                                                              int64_t K, int32_t j, int32_t nblk) {
  __shared__ double Ab[NB][NB + 1];
  __shared__ double Li[NB][NB + 1];
  const int64_t mat = blockIdx.x;
  const int32_t ib = j + 1 + (int32_t)blockIdx.y;
  CVG_GLOBAL double* a = gmem(A) + mat * K * K;
  const CVG_GLOBAL double* li = gmem(Linv) + (mat * nblk + j) * NB * NB;
  const int t = threadIdx.x, tx = t % NB, ty = t / NB;
  const int64_t r0 = (int64_t)ib * NB, c0 = (int64_t)j * NB;
  for (int r = ty; r < NB; r += kThreads / NB) {
    const int64_t i = r0 + r, c = c0 + tx;
    Ab[r][tx] = (i < K && c < K) ? a[i * K + c] : 0.0;
    Li[r][tx] = li[r * NB + tx];
  }
  __syncthreads();
  for (int r = ty; r < NB; r += kThreads / NB) {
    double s = 0.0;
    for (int k = 0; k <= tx; ++k) s = fma(Ab[r][k], Li[tx][k], s);  // (A Linv^T)[r][tx]
    const int64_t i = r0 + r, c = c0 + tx;
    if (i < K && c < K) a[i * K + c] = s;
  }
}

// trailing update A_ik -= L_ij L_kj^T for j < k <= i.  grid (matrices, lower
// triangle of the remaining blocks)
__global__ __launch_bounds__(kThreads) void chol_update_kernel(double* __restrict__ A, int64_t K,
                                                               int32_t j) {
  __shared__ double Li[NB][NB + 1];
  __shared__ double Lk[NB][NB + 1];
  const int64_t mat = blockIdx.x;
  // blockIdx.y -> (ii, kk) with 0 <= kk <= ii, counted row by row
  int32_t q = (int32_t)blockIdx.y, ii = 0;
  while (q > ii) {
    q -= ii + 1;
    ++ii;
  }
  const int32_t ib = j + 1 + ii, kb = j + 1 + q;
  CVG_GLOBAL double* a = gmem(A) + mat * K * K;
  const int t = threadIdx.x, tx = t % NB, ty = t / NB;
  const int64_t c0 = (int64_t)j * NB;
  for (int r = ty; r < NB; r += kThreads / NB) {
    const int64_t i = (int64_t)ib * NB + r, k = (int64_t)kb * NB + r, c = c0 + tx;
    Li[r][tx] = (i < K && c < K) ? a[i * K + c] : 0.0;
    Lk[r][tx] = (k < K && c < K) ? a[k * K + c] : 0.0;
  }
  __syncthreads();
  for (int r = ty; r < NB; r += kThreads / NB) {
    const int64_t i = (int64_t)ib * NB + r, k = (int64_t)kb * NB + tx;
    if (i >= K || k >= K || k > i) continue;
    double s = 0.0;
    for (int c = 0; c < NB; ++c) s = fma(Li[r][c], Lk[tx][c], s);
    a[i * K + k] -= s;
  }
}

// Both substitutions in one launch: workgroup (matrix, block of 32 columns
// of R) walks the block steps itself.
//   forward step j:  Z_j = Linv_jj R_j;    R_i -= L_ij Z_j     for i > j
//   backward step j: W_j = Linv_jj^T R_j;  R_i -= L_ji^T W_j   for i < j
// The updates run over (row, column) pairs of the other block rows, so a
// narrow R (M of a few columns) keeps every lane busy.  Each workgroup owns
// its rows x columns of R: its own writes are the only ones it reads back
// (ordered by the barrier between steps).
__global__ __launch_bounds__(kThreads) void tri_solve_kernel(const double* __restrict__ A,
                                                             const double* __restrict__ Linv,
                                                             double* __restrict__ R, int64_t K,
                                                             int64_t M, int32_t nblk) {
  __shared__ double Z[NB][NB + 1];
  __shared__ double Li[NB][NB + 1];
  __shared__ double Rb[NB][NB + 1];
  __shared__ double Ls[kSolveRows][NB + 1];
  const int64_t mat = blockIdx.x;
  const int64_t m0 = (int64_t)blockIdx.y * NB;
  const int64_t mw = M - m0 < NB ? M - m0 : NB;  // columns of R in this block
  const CVG_GLOBAL double* a = gmem(A) + mat * K * K;
  CVG_GLOBAL double* rr = gmem(R) + mat * K * M;
  const int t = threadIdx.x, tx = t % NB, ty = t / NB;
  for (int pass = 0; pass < 2; ++pass) {
    const bool backward = pass == 1;
    for (int32_t jj = 0; jj < nblk; ++jj) {
      const int32_t j = backward ? nblk - 1 - jj : jj;
      const int64_t r0 = (int64_t)j * NB;
      const CVG_GLOBAL double* li = gmem(Linv) + (mat * nblk + j) * NB * NB;
      for (int r = ty; r < NB; r += kThreads / NB) {
        const int64_t i = r0 + r;
        Rb[r][tx] = (i < K && tx < mw) ? rr[i * M + m0 + tx] : 0.0;
        Li[r][tx] = li[r * NB + tx];
      }
      __syncthreads();
      for (int r = ty; r < NB; r += kThreads / NB) {
        double sum = 0.0;
        if (!backward)
          for (int k = 0; k <= r; ++k) sum = fma(Li[r][k], Rb[k][tx], sum);
        else
          for (int k = r; k < NB; ++k) sum = fma(Li[k][r], Rb[k][tx], sum);
        Z[r][tx] = sum;
        const int64_t i = r0 + r;
        if (i < K && tx < mw) rr[i * M + m0 + tx] = sum;
      }
      __syncthreads();
      // the other block rows: forward i >= r0 + NB, backward i < r0; the
      // block column of L they need is staged in LDS kSolveRows rows at a
      // time (coalesced loads, all in flight), the dot products then read LDS
      const int64_t lo = backward ? 0 : r0 + NB, hi = backward ? r0 : K;
      const int64_t cmax = K - r0 < NB ? K - r0 : NB;  // columns of the block inside K
      for (int64_t i0 = lo; i0 < hi; i0 += kSolveRows) {
        const int64_t nr = hi - i0 < kSolveRows ? hi - i0 : kSolveRows;
        for (int e = t; e < kSolveRows * NB; e += kThreads) {
          // forward: Ls[ri][c] = L_ij = A[i0 + ri][r0 + c]
          // backward: Ls[ri][c] = (L_ji)^T = A[r0 + c][i0 + ri]
          const int ri = backward ? e % kSolveRows : e / NB;
          const int c = backward ? e / kSolveRows : e % NB;
          double v = 0.0;
          if (ri < nr && c < cmax)
            v = backward ? a[(r0 + c) * K + i0 + ri] : a[(i0 + ri) * K + r0 + c];
          Ls[ri][c] = v;
        }
        __syncthreads();
        for (int64_t e = t; e < nr * mw; e += kThreads) {
          const int ri = (int)(e / mw);
          const int mm = (int)(e % mw);
          double sum = 0.0;
#pragma unroll
          for (int c = 0; c < NB; ++c) sum = fma(Ls[ri][c], Z[c][mm], sum);
          rr[(i0 + ri) * M + m0 + mm] -= sum;
        }
        __syncthreads();
      }
    }
  }
}

}  // namespace

void ridge_solve(const double* xtx, const double* xty, const double* lambdas, int32_t n_folds,
                 int32_t n_lambda, int64_t K, int64_t M, double* A, double* R, double* Linv,
                 int32_t* flags, hipStream_t s) {
  const int64_t n_mat = (int64_t)n_folds * n_lambda;
  if (n_mat <= 0) return;
  const int32_t nblk = (int32_t)((K + NB - 1) / NB);
  {
    const int64_t per = (K * K + kThreads - 1) / kThreads;
    dim3 grid((unsigned)(per < 1024 ? per : 1024), (unsigned)n_mat);
    ridge_setup_kernel<<<grid, kThreads, 0, s>>>(xtx, xty, lambdas, n_lambda, K, M, A, R);
    CVG_LAUNCH_CHECK();
  }
  for (int32_t j = 0; j < nblk; ++j) {
    chol_diag_kernel<<<(unsigned)n_mat, kThreads, 0, s>>>(A, Linv, flags, K, j, nblk);
    CVG_LAUNCH_CHECK();
    const int32_t below = nblk - j - 1;
    if (below > 0) {
      chol_panel_kernel<<<dim3((unsigned)n_mat, (unsigned)below), kThreads, 0, s>>>(A, Linv, K, j,
                                                                                    nblk);
      CVG_LAUNCH_CHECK();
      chol_update_kernel<<<dim3((unsigned)n_mat, (unsigned)(below * (below + 1) / 2)), kThreads,
                           0, s>>>(A, K, j);
      CVG_LAUNCH_CHECK();
    }
  }
  if (M <= 0) return;
  const unsigned mb = (unsigned)((M + NB - 1) / NB);
  tri_solve_kernel<<<dim3((unsigned)n_mat, mb), kThreads, 0, s>>>(A, Linv, R, K, M, nblk);
  CVG_LAUNCH_CHECK();
}

}  // namespace cvg
