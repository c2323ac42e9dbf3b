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
// backward substitution through the stored inverses of the diagonal blocks).
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
  // inverse of the lower factor, one column per thread: L X = I
  if (t < NB) {
    const int col = t;
    for (int r = 0; r < NB; ++r) {
      double s = r == col ? 1.0 : 0.0;
      for (int k = col; k < r; ++k) s = fma(-L[r][k], I[k][col], s);
      I[r][col] = r < col ? 0.0 : s / L[r][r];
    }
  }
  __syncthreads();
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

// forward step j: Z_j = Linv_jj R_j; then R_i -= L_ij Z_j for i > j.
// backward step j: W_j = Linv_jj^T R_j; then R_i -= L_ji^T W_j for i < j.
// grid (matrices, column blocks of R of 32); one workgroup walks the rows.
__global__ __launch_bounds__(kThreads) void tri_solve_step_kernel(const double* __restrict__ A,
                                                                  const double* __restrict__ Linv,
                                                                  double* __restrict__ R,
                                                                  int64_t K, int64_t M, int32_t j,
                                                                  int32_t nblk, int backward) {
  __shared__ double Z[NB][NB + 1];
  __shared__ double Li[NB][NB + 1];
  __shared__ double Rb[NB][NB + 1];
  const int64_t mat = blockIdx.x;
  const int64_t m0 = (int64_t)blockIdx.y * NB;
  const CVG_GLOBAL double* a = gmem(A) + mat * K * K;
  const CVG_GLOBAL double* li = gmem(Linv) + (mat * nblk + j) * NB * NB;
  CVG_GLOBAL double* rr = gmem(R) + mat * K * M;
  const int t = threadIdx.x, tx = t % NB, ty = t / NB;
  const int64_t r0 = (int64_t)j * NB;
  for (int r = ty; r < NB; r += kThreads / NB) {
    const int64_t i = r0 + r, m = m0 + tx;
    Rb[r][tx] = (i < K && m < M) ? rr[i * M + m] : 0.0;
    Li[r][tx] = li[r * NB + tx];
  }
  __syncthreads();
  for (int r = ty; r < NB; r += kThreads / NB) {
    double s = 0.0;
    if (!backward)
      for (int k = 0; k <= r; ++k) s = fma(Li[r][k], Rb[k][tx], s);
    else
      for (int k = r; k < NB; ++k) s = fma(Li[k][r], Rb[k][tx], s);
    Z[r][tx] = s;
    const int64_t i = r0 + r, m = m0 + tx;
    if (i < K && m < M) rr[i * M + m] = s;
  }
  __syncthreads();
  // propagate to the other block rows (one block row per pass of the loop)
  const int32_t lo = backward ? 0 : j + 1, hi = backward ? j : nblk;
  for (int32_t ib = lo; ib < hi; ++ib) {
    for (int r = ty; r < NB; r += kThreads / NB) {
      const int64_t i = (int64_t)ib * NB + r, m = m0 + tx;
      if (i >= K || m >= M) continue;
      double s = 0.0;
      if (!backward) {
        // L_ij = A[i][r0 + c]
        for (int c = 0; c < NB; ++c) {
          const int64_t cc = r0 + c;
          if (cc < K) s = fma(a[i * K + cc], Z[c][tx], s);
        }
      } else {
        // (L_ji)^T[r][c] = A[r0 + c][i]
        for (int c = 0; c < NB; ++c) {
          const int64_t cc = r0 + c;
          if (cc < K) s = fma(a[cc * K + i], Z[c][tx], s);
        }
      }
      rr[i * M + m] -= s;
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
  for (int32_t j = 0; j < nblk; ++j) {
    tri_solve_step_kernel<<<dim3((unsigned)n_mat, mb), kThreads, 0, s>>>(A, Linv, R, K, M, j, nblk,
                                                                         0);
    CVG_LAUNCH_CHECK();
  }
  for (int32_t j = nblk - 1; j >= 0; --j) {
    tri_solve_step_kernel<<<dim3((unsigned)n_mat, mb), kThreads, 0, s>>>(A, Linv, R, K, M, j, nblk,
                                                                         1);
    CVG_LAUNCH_CHECK();
  }
}

}  // namespace cvg
