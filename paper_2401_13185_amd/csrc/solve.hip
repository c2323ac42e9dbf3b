// Per-fold ridge regression on the device: B = (A + lambda I)^{-1} R for a
// batch of symmetric positive definite A (K x K) and right-hand sides R
// (K x M), all FP64 and row-major, one per (fold, lambda).  This consumes
// the training products directly (the models the paper names for them,
// Section 1: RR, and OLS for lambda = 0).
//
// The systems are copied into padded workspaces first: A to Kp x Kp with the
// identity in the padding, R to Kp x Mp with zeros (Kp, Mp multiples of 32),
// so no kernel below needs a bounds check and every load can be issued
// without waiting for the one before it.
//
// Blocked right-looking Cholesky A = L L^T with 32 x 32 blocks:
//   for each block column j
//     diag:   L_jj = chol(A_jj) and its inverse, in registers (one wave per matrix)
//     panel:  L_ij = A_ij L_jj^{-T} for every block row i > j (also stored
//             transposed in the upper triangle)
//     update: A_ik -= L_ij L_kj^T for every j < k <= i (lower triangle)
// then R is overwritten by L^{-T} L^{-1} R with the same blocks (forward and
// backward substitution through the stored inverses of the diagonal blocks,
// one launch for both), and copied out.
// A matrix whose pivot is not positive (A + lambda I not positive definite)
// sets its flag and continues with NaN.
//
// Arithmetic: FP64 FMA on the vector units; every sum runs in a fixed order
// (deterministic).
#include <cmath>

#include "internal.h"

namespace cvg {
namespace {

constexpr int NB = 32;                         // block edge
constexpr int kThreads = 256;                  // 8 rows x 32 columns per pass
constexpr int kRowStep = kThreads / NB;        // rows a pass covers
constexpr int kRowsPerThread = NB / kRowStep;  // passes per block
constexpr int kWave = 64;
// the substitutions: the first kThreads threads handle the 32 x 32 blocks,
// all of them one row each of the update; 512 threads (up to 512 rows in one
// pass) where a row's registers allow two waves per SIMD, else 256
template <int MW>
constexpr int solve_threads() {
  return MW <= 16 ? 512 : kThreads;
}

// padded systems: A + lambda I in Kp x Kp (identity in the padding) and R in
// Kp x Mp (zeros in the padding), from the products (p-major, lambda-minor)
__global__ __launch_bounds__(kThreads) void ridge_setup_kernel(
    const double* __restrict__ xtx, const double* __restrict__ xty,
    const double* __restrict__ lambdas, int32_t n_lambda, int64_t K, int64_t M, int64_t Kp,
    int64_t Mp, double* __restrict__ A, double* __restrict__ R) {
  const int64_t mat = blockIdx.y;  // fold * n_lambda + lambda
  const int64_t f = mat / n_lambda;
  const double lam = lambdas[mat % n_lambda];
  const CVG_GLOBAL double* src = gmem(xtx) + f * K * K;
  CVG_GLOBAL double* dst = gmem(A) + mat * Kp * Kp;
  for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < Kp * Kp;
       e += (int64_t)gridDim.x * kThreads) {
    const int64_t i = e / Kp, j = e - i * Kp;
    dst[e] = (i < K && j < K) ? src[i * K + j] + (i == j ? lam : 0.0) : (i == j ? 1.0 : 0.0);
  }
  const CVG_GLOBAL double* rs = gmem(xty) + f * K * M;
  CVG_GLOBAL double* rd = gmem(R) + mat * Kp * Mp;
  for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < Kp * Mp;
       e += (int64_t)gridDim.x * kThreads) {
    const int64_t i = e / Mp, m = e - i * Mp;
    rd[e] = (i < K && m < M) ? rs[i * M + m] : 0.0;
  }
}

// B[mat] = the first K x M of the padded R[mat]
__global__ __launch_bounds__(kThreads) void ridge_store_kernel(const double* __restrict__ R,
                                                               int64_t K, int64_t M, int64_t Kp,
                                                               int64_t Mp, double* __restrict__ B) {
  const int64_t mat = blockIdx.y;
  const CVG_GLOBAL double* rs = gmem(R) + mat * Kp * Mp;
  CVG_GLOBAL double* bd = gmem(B) + mat * K * M;
  for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < K * M;
       e += (int64_t)gridDim.x * kThreads) {
    const int64_t i = e / M, m = e - i * M;
    bd[e] = rs[i * Mp + m];
  }
}

// the value that lane `lane` holds in x, in every lane (a wave-wide
// broadcast through the scalar registers)
__device__ __forceinline__ double from_lane(double x, int lane) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// diagonal block j of every matrix, one wave per matrix, all in registers:
// lanes 0..31 hold the rows of the block and factor it column by column
// (right-looking); lanes 32..63 hold the columns of the factor's inverse and
// run the forward substitution L X = I in the same steps, since step c of
// the substitution needs only column c of L, final once step c of the
// factorisation has divided it.  Both updates are one FMA with a broadcast
// operand: the factor rows take L[r][k] -= L[r][c] L[k][c] (c < k <= r), the
// inverse columns X[k][t] -= L[k][c] X[c][t] (k > c); every entry sums in
// increasing c.  The factor goes to the lower triangle of the block (zeros
// above), its inverse to Linv; flags[mat] = 1 on a non-positive pivot.
__global__ __launch_bounds__(kWave) void chol_diag_kernel(double* __restrict__ A,
                                                          double* __restrict__ Linv,
                                                          int32_t* __restrict__ flags, int64_t Kp,
                                                          int32_t j, int32_t nblk) {
  const int64_t mat = blockIdx.x;
  const int l = threadIdx.x;
  const bool fac = l < NB;  // a factor row, else an inverse column
  const int q = l % NB;     // its row / column index
  const int64_t r0 = (int64_t)j * NB;
  CVG_GLOBAL double* arow = gmem(A) + mat * Kp * Kp + (r0 + q) * Kp + r0;
  double u[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    const double v = arow[k];
    u[k] = (fac && k <= q) ? v : (q == k ? 1.0 : 0.0);
  }
  bool bad = false;
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    const double d = from_lane(u[c], c);  // pivot: A[c][c] after the earlier steps
    bad = bad || !(d > 0.0);
    const double piv = d > 0.0 ? sqrt(d) : NAN;
    // L[q][c] below the pivot, X[c][q] in an inverse column (a factor row
    // above the pivot divides a value that is never read)
    u[c] = fac && q == c ? piv : u[c] / piv;
#pragma unroll
    for (int k = c + 1; k < NB; ++k) {
      const double lkc = from_lane(u[c], k);  // L[k][c]
      // factor rows with q < k update entries above the diagonal: never read
      u[k] = fma(-u[c], lkc, u[k]);
    }
  }
  if (l == 0 && bad) flags[mat] = 1;
  if (fac) {
#pragma unroll
    for (int k = 0; k < NB; ++k) arow[k] = k <= q ? u[k] : 0.0;
  } else {
    CVG_GLOBAL double* li = gmem(Linv) + (mat * nblk + j) * NB * NB;
#pragma unroll
    for (int r = 0; r < NB; ++r) li[r * NB + q] = u[r];
  }
}

// panel: L_ij = A_ij Linv_jj^T for block rows i > j, written to the lower
// triangle and, transposed, to block (j, i) of the upper triangle (which the
// factorisation never reads; the substitutions read the factor along rows of
// A from there).  grid (matrices, rows below)
__global__ __launch_bounds__(kThreads) void chol_panel_kernel(double* __restrict__ A,
                                                              const double* __restrict__ Linv,
                                                              int64_t Kp, int32_t j, int32_t nblk) {
  __shared__ double Ab[NB][NB + 1];
  __shared__ double Li[NB][NB + 1];
  __shared__ double Lt[NB][NB + 1];
  const int64_t mat = blockIdx.x;
  const int32_t ib = j + 1 + (int32_t)blockIdx.y;
  CVG_GLOBAL double* a = gmem(A) + mat * Kp * Kp;
  const CVG_GLOBAL double* li = gmem(Linv) + (mat * nblk + j) * NB * NB;
  const int t = threadIdx.x, tx = t % NB, ty = t / NB;
  const int64_t r0 = (int64_t)ib * NB, c0 = (int64_t)j * NB;
  double va[kRowsPerThread], vl[kRowsPerThread];
#pragma unroll
  for (int q = 0; q < kRowsPerThread; ++q) {
    const int r = ty + kRowStep * q;
    va[q] = a[(r0 + r) * Kp + c0 + tx];
    vl[q] = li[r * NB + tx];
  }
#pragma unroll
  for (int q = 0; q < kRowsPerThread; ++q) {
    Ab[ty + kRowStep * q][tx] = va[q];
    Li[ty + kRowStep * q][tx] = vl[q];
  }
  __syncthreads();
  // rows ty + kRowStep * q of (A Linv^T)[.][tx], sharing Linv's row tx
  double s[kRowsPerThread];
#pragma unroll
  for (int q = 0; q < kRowsPerThread; ++q) s[q] = 0.0;
  for (int k = 0; k <= tx; ++k) {
    const double b = Li[tx][k];
#pragma unroll
    for (int q = 0; q < kRowsPerThread; ++q) s[q] = fma(Ab[ty + kRowStep * q][k], b, s[q]);
  }
#pragma unroll
  for (int q = 0; q < kRowsPerThread; ++q) {
    const int r = ty + kRowStep * q;
    a[(r0 + r) * Kp + c0 + tx] = s[q];
    Lt[r][tx] = s[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kRowsPerThread; ++q) {  // A[c0 + c][r0 + tx] = L[r0 + tx][c0 + c]
    const int c = ty + kRowStep * q;
    a[(c0 + c) * Kp + r0 + tx] = Lt[tx][c];
  }
}

// trailing update A_ik -= L_ij L_kj^T for j < k <= i.  grid (matrices, lower
// triangle of the remaining blocks)
__global__ __launch_bounds__(kThreads) void chol_update_kernel(double* __restrict__ A, int64_t Kp,
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
  CVG_GLOBAL double* a = gmem(A) + mat * Kp * Kp;
  const int t = threadIdx.x, tx = t % NB, ty = t / NB;
  const int64_t c0 = (int64_t)j * NB;
  CVG_GLOBAL double* out = a + (int64_t)ib * NB * Kp + (int64_t)kb * NB + tx;  // A_ik[0][tx]
  double vi[kRowsPerThread], vk[kRowsPerThread], vo[kRowsPerThread];
#pragma unroll
  for (int p = 0; p < kRowsPerThread; ++p) {
    const int r = ty + kRowStep * p;
    vi[p] = a[((int64_t)ib * NB + r) * Kp + c0 + tx];
    vk[p] = a[((int64_t)kb * NB + r) * Kp + c0 + tx];
    vo[p] = out[r * Kp];
  }
#pragma unroll
  for (int p = 0; p < kRowsPerThread; ++p) {
    Li[ty + kRowStep * p][tx] = vi[p];
    Lk[ty + kRowStep * p][tx] = vk[p];
  }
  __syncthreads();
  // rows ty + kRowStep * p of the product, sharing L_kj's row tx
  double s[kRowsPerThread];
#pragma unroll
  for (int p = 0; p < kRowsPerThread; ++p) s[p] = 0.0;
#pragma unroll 8
  for (int c = 0; c < NB; ++c) {
    const double b = Lk[tx][c];
#pragma unroll
    for (int p = 0; p < kRowsPerThread; ++p) s[p] = fma(Li[ty + kRowStep * p][c], b, s[p]);
  }
#pragma unroll
  for (int p = 0; p < kRowsPerThread; ++p) {
    const int r = ty + kRowStep * p;
    if (ib != kb || tx <= r) out[r * Kp] = vo[p] - s[p];
  }
}

// Both substitutions in one launch: workgroup (matrix, block of 32 columns
// of R) walks the block steps itself.
//   forward step j:  Z_j = Linv_jj R_j;    R_i -= L_ij Z_j     for i > j
//   backward step j: W_j = Linv_jj^T R_j;  R_i -= L_ji^T W_j   for i < j
// In both passes the coefficient of Z[c] in row i is A[r0 + c][i]: the
// factor's block row j in the lower triangle (backward, i < r0) or the
// transposed copy of its block column j in the upper triangle (forward,
// i >= r0 + 32).  One thread per row of R reads those 32 values down a column
// of A, consecutive threads consecutive columns, all loads in flight.  The
// rows of the next step's block go on to it through LDS as they are updated,
// and the next diagonal inverse is loaded during the update, so a step waits
// on memory once.  Each workgroup owns its rows x columns of R: its own
// writes are the only ones it reads back (ordered by the barriers between
// steps).  Padding rows of the last block (past K) stay zero.  MW (8, 16 or
// 32) is the width of R each row update carries in registers: at least the
// block's columns of B, the rest padding zeros that stay zero.
template <int MW, bool FAST>
__global__ __launch_bounds__(solve_threads<MW>()) void tri_solve_kernel(const double* __restrict__ A,
                                                             const double* __restrict__ Linv,
                                                             double* __restrict__ R, int64_t K,
                                                             int64_t M, int64_t Kp, int64_t Mp,
                                                             int32_t nblk) {
  __shared__ double Z[NB][NB + 1];
  __shared__ double Li[2][NB][NB + 1];
  __shared__ double Rb[NB][NB + 1];
  const int64_t mat = blockIdx.x;
  const int64_t m0 = (int64_t)blockIdx.y * NB;
  const CVG_GLOBAL double* a = gmem(A) + mat * Kp * Kp;
  CVG_GLOBAL double* rr = gmem(R) + mat * Kp * Mp + m0;
  const int t = threadIdx.x, tx = t % NB, ty = t / NB;
  const bool blk = t < kThreads;  // one of the threads that handle a 32 x 32 block
  // FAST: Kp <= the thread count and MW <= 16 (the launch checks)
  constexpr bool fast = FAST;
  auto load_li = [&](int32_t j, double* vl) {
    const CVG_GLOBAL double* li = gmem(Linv) + (mat * nblk + j) * NB * NB;
#pragma unroll
    for (int q = 0; q < kRowsPerThread; ++q) vl[q] = li[(ty + kRowStep * q) * NB + tx];
  };
  int buf = 0;
  for (int pass = 0; pass < 2; ++pass) {
    const bool backward = pass == 1;
    {
      // the pass's first block: its rows of R and its inverse from memory
      const int32_t j = backward ? nblk - 1 : 0;
      const int64_t r0 = (int64_t)j * NB;
      if (blk) {
        double vr[kRowsPerThread], vl[kRowsPerThread];
#pragma unroll
        for (int q = 0; q < kRowsPerThread; ++q) vr[q] = rr[(r0 + ty + kRowStep * q) * Mp + tx];
        load_li(j, vl);
#pragma unroll
        for (int q = 0; q < kRowsPerThread; ++q) {
          Rb[ty + kRowStep * q][tx] = vr[q];
          Li[buf][ty + kRowStep * q][tx] = vl[q];
        }
      }
      __syncthreads();
    }
    // Rows of R in registers (Kp <= the thread count, MW <= 16): thread t
    // keeps row t for the whole pass, so an update reads no R from memory,
    // and the coefficients of its next step are loaded at the end of this
    // one, while the barrier and the next block's Z are in progress.
    double rv[MW], lc[NB];
    if (fast) {
      const int32_t j = backward ? nblk - 1 : 0;
      const int64_t lo = backward ? 0 : (int64_t)(j + 1) * NB, hi = backward ? (int64_t)j * NB : Kp;
      if (t < Kp) {
#pragma unroll
        for (int mm = 0; mm < MW; ++mm) rv[mm] = rr[(int64_t)t * Mp + mm];
      }
      if (t >= lo && t < hi) {
#pragma unroll
        for (int c = 0; c < NB; ++c) lc[c] = a[((int64_t)j * NB + c) * Kp + t];
      }
    }
    for (int32_t jj = 0; jj < nblk; ++jj) {
      const int32_t j = backward ? nblk - 1 - jj : jj;
      const int64_t r0 = (int64_t)j * NB;
      const bool last = jj + 1 == nblk;
      const int32_t jn = backward ? j - 1 : j + 1;  // the next step's block
      const int64_t n0 = (int64_t)jn * NB;
      if (blk) {
#pragma unroll
        for (int q = 0; q < kRowsPerThread; ++q) {
          const int r = ty + kRowStep * q;
          // all 32 terms, unrolled: the inverse block holds exact zeros
          // above its diagonal, so the terms outside the triangle add zero
          // and the sum is that of the triangle, in the same order
          double sum = 0.0;
          if (!backward) {
#pragma unroll
            for (int k = 0; k < NB; ++k) sum = fma(Li[buf][r][k], Rb[k][tx], sum);
          } else {
#pragma unroll
            for (int k = 0; k < NB; ++k) sum = fma(Li[buf][k][r], Rb[k][tx], sum);
          }
          Z[r][tx] = sum;
          rr[(r0 + r) * Mp + tx] = sum;
        }
      }
      __syncthreads();
      double vl[kRowsPerThread];
      if (!last && blk) load_li(jn, vl);
      const int64_t lo = backward ? 0 : r0 + NB, hi = backward ? r0 : Kp;
      if (fast) {
        if (t >= lo && t < hi) {
          double sum[MW];
#pragma unroll
          for (int mm = 0; mm < MW; ++mm) sum[mm] = 0.0;
#pragma unroll
          for (int c = 0; c < NB; ++c) {
#pragma unroll
            for (int mm = 0; mm < MW; ++mm) sum[mm] = fma(lc[c], Z[c][mm], sum[mm]);
            if (c % 4 == 3) __builtin_amdgcn_sched_barrier(0);
          }
#pragma unroll
          for (int mm = 0; mm < MW; ++mm) rv[mm] -= sum[mm];
          if (!last && t >= n0 && t < n0 + NB) {
#pragma unroll
            for (int mm = 0; mm < MW; ++mm) Rb[t - n0][mm] = rv[mm];
          }
        }
        // the next step's rows of the update: forward [n0 + 32, Kp), backward [0, n0)
        const int64_t lo_n = backward ? 0 : n0 + NB, hi_n = backward ? n0 : Kp;
        if (!last && t >= lo_n && t < hi_n) {
#pragma unroll
          for (int c = 0; c < NB; ++c) lc[c] = a[(n0 + c) * Kp + t];
        }
      }
      for (int64_t i = lo + t; !fast && i < hi; i += solve_threads<MW>()) {
        double lc[NB], rv[MW];
#pragma unroll
        for (int c = 0; c < NB; ++c) lc[c] = a[(r0 + c) * Kp + i];
#pragma unroll
        for (int mm = 0; mm < MW; ++mm) rv[mm] = rr[i * Mp + mm];
        double sum[MW];
#pragma unroll
        for (int mm = 0; mm < MW; ++mm) sum[mm] = 0.0;
#pragma unroll
        for (int c = 0; c < NB; ++c) {
#pragma unroll
          for (int mm = 0; mm < MW; ++mm) sum[mm] = fma(lc[c], Z[c][mm], sum[mm]);
          // keep the scheduler from hoisting every row of Z into registers
          if (c % 4 == 3) __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int mm = 0; mm < MW; ++mm) {
          rv[mm] -= sum[mm];
          rr[i * Mp + mm] = rv[mm];
        }
        if (!last && i >= n0 && i < n0 + NB) {
#pragma unroll
          for (int mm = 0; mm < MW; ++mm) Rb[i - n0][mm] = rv[mm];
        }
      }
      if (!last && blk) {
#pragma unroll
        for (int q = 0; q < kRowsPerThread; ++q) Li[buf ^ 1][ty + kRowStep * q][tx] = vl[q];
      }
      __syncthreads();
      buf ^= 1;
    }
  }
}

}  // namespace

void ridge_solve(const double* xtx, const double* xty, const double* lambdas, int32_t n_folds,
                 int32_t n_lambda, int64_t K, int64_t M, double* A, double* R, double* Linv,
                 int32_t* flags, double* B, hipStream_t s) {
  const int64_t n_mat = (int64_t)n_folds * n_lambda;
  if (n_mat <= 0 || K <= 0) return;
  const int32_t nblk = (int32_t)((K + NB - 1) / NB);
  const int64_t Kp = (int64_t)nblk * NB, Mp = (M + NB - 1) / NB * NB;
  {
    const int64_t per = (Kp * Kp + kThreads - 1) / kThreads;
    dim3 grid((unsigned)(per < 1024 ? per : 1024), (unsigned)n_mat);
    ridge_setup_kernel<<<grid, kThreads, 0, s>>>(xtx, xty, lambdas, n_lambda, K, M, Kp, Mp, A, R);
    CVG_LAUNCH_CHECK();
  }
  for (int32_t j = 0; j < nblk; ++j) {
    chol_diag_kernel<<<(unsigned)n_mat, kWave, 0, s>>>(A, Linv, flags, Kp, j, nblk);
    CVG_LAUNCH_CHECK();
    const int32_t below = nblk - j - 1;
    if (below > 0) {
      chol_panel_kernel<<<dim3((unsigned)n_mat, (unsigned)below), kThreads, 0, s>>>(A, Linv, Kp,
                                                                                    j, nblk);
      CVG_LAUNCH_CHECK();
      chol_update_kernel<<<dim3((unsigned)n_mat, (unsigned)(below * (below + 1) / 2)), kThreads,
                           0, s>>>(A, Kp, j);
      CVG_LAUNCH_CHECK();
    }
  }
  if (M <= 0) return;
  const dim3 grid((unsigned)n_mat, (unsigned)(Mp / NB));
  const bool fast = Kp <= solve_threads<16>();  // one row of R per thread
  if (M <= 8 && fast)
    tri_solve_kernel<8, true><<<grid, solve_threads<8>(), 0, s>>>(A, Linv, R, K, M, Kp, Mp, nblk);
  else if (M <= 8)
    tri_solve_kernel<8, false><<<grid, solve_threads<8>(), 0, s>>>(A, Linv, R, K, M, Kp, Mp, nblk);
  else if (M <= 16 && fast)
    tri_solve_kernel<16, true><<<grid, solve_threads<16>(), 0, s>>>(A, Linv, R, K, M, Kp, Mp, nblk);
  else if (M <= 16)
    tri_solve_kernel<16, false><<<grid, solve_threads<16>(), 0, s>>>(A, Linv, R, K, M, Kp, Mp, nblk);
  else
    tri_solve_kernel<NB, false><<<grid, solve_threads<NB>(), 0, s>>>(A, Linv, R, K, M, Kp, Mp, nblk);
  CVG_LAUNCH_CHECK();
  {
    const int64_t per = (K * M + kThreads - 1) / kThreads;
    dim3 grid((unsigned)(per < 1024 ? per : 1024), (unsigned)n_mat);
    ridge_store_kernel<<<grid, kThreads, 0, s>>>(R, K, M, Kp, Mp, B);
    CVG_LAUNCH_CHECK();
  }
}

}  // namespace cvg
