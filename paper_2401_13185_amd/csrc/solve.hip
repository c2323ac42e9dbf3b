// Per-fold ridge regression on the device: B = (A + lambda I)^{-1} R for a
// batch of symmetric positive definite A (K x K) and right-hand sides R
// (K x M), all FP64 and row-major, one per (fold, lambda).  This consumes
// the training products directly (the models the paper names for them,
// Section 1: RR, and OLS for lambda = 0).
//
// The systems are copied into padded workspaces first: A to Kp x Kp with the
// identity in the padding (Kp a multiple of 64) and R^T below it in
// Ma = ceil(M / 64) 64 rows with zeros in the padding, so no kernel below
// needs a bounds check and every load can be issued without waiting for the
// one before it.  The penalties travel in the setup kernel's arguments (up
// to 64; more from a device copy).
//
// Blocked right-looking Cholesky A = L L^T with 64 x 64 blocks:
//   for each block column s
//     diag:   L_ss = chol(A_ss) and its inverse (one workgroup per matrix:
//             two 32 x 32 one-wave factorisations in registers, joined by
//             products on the matrix cores); block 0 by extra workgroups
//             of the setup launch, block s > 0 inside the previous step's
//             update by the workgroup that finishes A_ss
//     panel:  L_is = A_is L_ss^{-T} for every block row i > s
//     update: A_ik -= L_is L_ks^T for every s < k <= i (lower triangle)
// R^T sits in extra block rows below A and takes the panel and update steps
// with it, so it leaves the factorisation as (L^{-1} R)^T (the forward
// substitution).  The backward substitution L^{-T} runs through the stored
// inverses of the factor's 32 x 32 diagonal blocks: for Kp <= 512 on the
// matrix cores, with the right-hand sides held in the accumulators and B
// written directly (that kernel also forms the last block column's panel of
// the R^T rows); beyond, one row per thread, from a transposed copy, and the
// result copied out.
// A matrix whose pivot is not positive (A + lambda I not positive definite)
// sets its flag and continues with NaN.
//
// Arithmetic: FP64 throughout; the panel, the trailing update (nearly all
// of the factorisation's flops), the diagonal step's block products and the
// matrix-core substitution on the FP64 matrix cores (v_mfma_f64_16x16x4f64),
// the rest FP64 FMA on the vector units.  Every sum
// runs in a fixed order (deterministic).
#include <cmath>

#include "internal.h"

namespace cvg {
namespace {

typedef double double2_t __attribute__((ext_vector_type(2)));
typedef double double4_t __attribute__((ext_vector_type(4)));

constexpr int NB = 32;                         // block edge of the substitutions
constexpr int NB2 = 64;                        // block edge of the factorisation
constexpr int LDB = NB2 + 2;                   // LDS row stride of a 64 x 64 block
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

// (matrix, block index) of a workgroup of a launch over n_mat matrices x ny
// blocks: grid (n_mat, ny), or, where ny would pass grid.y's limit, a 1-D
// grid of n_mat x ny workgroups, the matrix fastest (the same order)
__device__ inline void mat_and_block(int64_t n_mat, int64_t& mat, int32_t& y) {
  if (gridDim.y > 1) {
    mat = blockIdx.x;
    y = (int32_t)blockIdx.y;
  } else {
    const uint32_t n = (uint32_t)n_mat, b = blockIdx.x;
    mat = b % n;
    y = (int32_t)(b / n);
  }
}
inline dim3 mat_block_grid(int64_t n_mat, int64_t ny) {
  return ny <= 65535 ? dim3((unsigned)n_mat, (unsigned)ny) : dim3((unsigned)(n_mat * ny));
}

// Row-per-thread substitution (Kp > 512): R[mat] (Kp x Mp) = the first Mp
// rows of (L^{-1} R)^T below the factor, transposed: the substitution's
// input.  grid (Kp / 8, up to 65535 strides over the matrices)
__global__ __launch_bounds__(kThreads) void ridge_z_kernel(const double* __restrict__ A, int64_t Kp,
                                                           int64_t Kr, int64_t Mp, int64_t n_mat,
                                                           double* __restrict__ R) {
  for (int64_t mat = blockIdx.y; mat < n_mat; mat += gridDim.y) {
    const CVG_GLOBAL double* z = gmem(A) + mat * Kr * Kp + Kp * Kp;  // row m: Z^T[m][.]
    CVG_GLOBAL double* rd = gmem(R) + mat * Kp * Mp;
    const int64_t j0 = (int64_t)blockIdx.x * 8;
    for (int64_t e = threadIdx.x; e < 8 * Mp; e += kThreads) {
      const int64_t m = e / 8, j = j0 + e % 8;
      rd[j * Mp + m] = z[m * Kp + j];
    }
  }
}

// B[mat] = the first K x M of the padded R[mat] (grid.y strides over the
// matrices)
__global__ __launch_bounds__(kThreads) void ridge_store_kernel(const double* __restrict__ R,
                                                               int64_t K, int64_t M, int64_t Kp,
                                                               int64_t Mp, int64_t n_mat,
                                                               double* __restrict__ B) {
  for (int64_t mat = blockIdx.y; mat < n_mat; mat += gridDim.y) {
    const CVG_GLOBAL double* rs = gmem(R) + mat * Kp * Mp;
    CVG_GLOBAL double* bd = gmem(B) + mat * K * M;
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < K * M;
         e += (int64_t)gridDim.x * kThreads) {
      const int64_t i = e / M, m = e - i * M;
      bd[e] = rs[i * Mp + m];
    }
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

// Steps c = C0 .. C1 - 1 of a one-wave right-looking factorisation over the
// columns [C0, C1): a lane holds a factor row (fac; row q) or a column of the
// factor's inverse in u.  Step c: with the pivot p = sqrt(A[c][c]) a factor
// row takes L[q][c] = A[q][c] / p, an inverse column X[c][t] = X[c][t] / p
// (both as products with 1 / p); then both updates are one FMA with a
// broadcast operand (v_readlane): the factor rows L[q][k] -= L[q][c] L[k][c],
// the inverse columns X[k][t] -= L[k][c] X[c][t] (c < k < C1); every entry
// sums in increasing c.  Factor rows above the pivot update entries above
// the diagonal, which are never read.  bad is set on a non-positive pivot
// (the factorisation then continues with NaN).
template <int C0, int C1>
__device__ __forceinline__ void factor_steps(double (&u)[NB], int q, bool fac, bool& bad) {
#pragma unroll
  for (int c = C0; c < C1; ++c) {
    const double d = from_lane(u[c], c);  // pivot: A[c][c] after the earlier steps
    bad = bad || !(d > 0.0);
    // y = 1 / sqrt(d): the hardware estimate (about 23 good bits) and two
    // Newton steps y <- y (3 - d y^2) / 2, each doubling the good bits; then
    // sqrt(d) = d y, and the column is scaled by y instead of divided by
    // sqrt(d) (a chain of 7 dependent operations instead of about 25)
    double y = __builtin_amdgcn_rsq(d);
    const double hd = 0.5 * d;
    y = y * fma(-hd, y * y, 1.5);
    y = y * fma(-hd, y * y, 1.5);
    if (!(d > 0.0)) y = NAN;
    u[c] = fac && q == c ? d * y : u[c] * y;
#pragma unroll
    for (int k = c + 1; k < C1; ++k) u[k] = fma(-u[c], from_lane(u[c], k), u[k]);  // L[k][c]
  }
}

// One wave factors a 32 x 32 block held in LDS (rows q of S, lower triangle
// read) and inverts the factor, in registers except for three 16 x 16 x 16
// products: lanes 0..31 hold the rows of the block, lanes 32..63 the columns
// of the factor's inverse, which run the forward substitution L X = I in the
// same steps (step c of it needs only column c of L, final once step c of
// the factorisation has scaled it).  The block is split in 16-column halves,
//   [A11 .; A21 A22] = [L11 0; L21 L22] [L11 0; L21 L22]^T:
// the first 16 steps factor columns 0..15 of all 32 rows (L11, L21 = A21
// L11^{-T}) and invert L11; A22 -= L21 L21^T on the matrix cores; the next
// 16 steps factor and invert L22; the inverse's lower left quadrant is
// -L22^{-1} (L21 L11^{-1}) (two more products).  A step broadcasts only the
// factor entries of its half: 240 broadcasts instead of 496 for the whole
// block at once.  The factor goes back to S (lower triangle, zeros above),
// its inverse to Li (row-major, zeros above the diagonal).  LDS traffic
// between the phases stays within the wave, whose LDS accesses complete in
// order; the fences keep the compiler from moving them across phases.
__device__ __forceinline__ void factor32_wave(double* S, int ld, double* Li, int ldi, int l,
                                              bool& bad) {
  constexpr int H = NB / 2;
  const bool fac = l < NB;  // a factor row, else an inverse column
  const int q = l % NB;     // its row / column index
  const int fr = (l & 63) >> 4, fc = l & 15;
  double u[NB];
  // columns 0..15: rows of [A11; A21], inverse columns 0..15 (lanes 32..47)
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    const double v = k < H ? S[q * ld + k] : 0.0;
    u[k] = k >= H ? 0.0 : (fac ? (k <= q ? v : 0.0) : (q == k ? 1.0 : 0.0));
  }
  factor_steps<0, H>(u, q, fac, bad);
  // L11 (zeros above it and in the upper right quadrant) and L21 to S,
  // L11^{-1} to Li
  if (fac) {
#pragma unroll
    for (int k = 0; k < NB; ++k)
      if (q < H || k < H) S[q * ld + k] = k < H && k <= q ? u[k] : 0.0;
  } else if (q < H) {
#pragma unroll
    for (int r = 0; r < H; ++r) Li[r * ldi + q] = u[r];
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  // A22 -= L21 L21^T: element e of lane (fr, fc) is (H + 4 e + fr, H + fc)
  {
    double4_t c;
#pragma unroll
    for (int e = 0; e < 4; ++e) c[e] = S[(H + 4 * e + fr) * ld + H + fc];
#pragma unroll
    for (int kk = 0; kk < H / 4; ++kk) {
      const double w = S[(H + fc) * ld + 4 * kk + fr];  // L21[fc][4 kk + fr]
      c = __builtin_amdgcn_mfma_f64_16x16x4f64(-w, w, c, 0, 0, 0);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) S[(H + 4 * e + fr) * ld + H + fc] = c[e];
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  // columns 16..31: rows 16..31 of A22, inverse columns 16..31 (lanes 48..63)
#pragma unroll
  for (int k = H; k < NB; ++k) {
    const double v = S[q * ld + k];
    u[k] = fac ? (q >= H && k <= q ? v : 0.0) : (q == k ? 1.0 : 0.0);
  }
  factor_steps<H, NB>(u, q, fac, bad);
  if (fac && q >= H) {
#pragma unroll
    for (int k = H; k < NB; ++k) S[q * ld + k] = k <= q ? u[k] : 0.0;
  } else if (!fac && q >= H) {
#pragma unroll
    for (int r = H; r < NB; ++r) Li[r * ldi + q] = u[r];
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  // T = L21 L11^{-1}, kept in Li's upper right quadrant for the moment
  {
    double4_t c = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kk = 0; kk < H / 4; ++kk)
      c = __builtin_amdgcn_mfma_f64_16x16x4f64(S[(H + fc) * ld + 4 * kk + fr],
                                               Li[(4 * kk + fr) * ldi + fc], c, 0, 0, 0);
#pragma unroll
    for (int e = 0; e < 4; ++e) Li[(4 * e + fr) * ldi + H + fc] = c[e];
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  // lower left quadrant of the inverse: -L22^{-1} T; then the zeros of the
  // upper right one (each lane clears the entries of T it wrote, after the
  // wave's reads of them)
  {
    double4_t c = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kk = 0; kk < H / 4; ++kk)
      c = __builtin_amdgcn_mfma_f64_16x16x4f64(Li[(H + fc) * ldi + H + 4 * kk + fr],
                                               Li[(4 * kk + fr) * ldi + H + fc], c, 0, 0, 0);
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      Li[(H + 4 * e + fr) * ldi + fc] = -c[e];
      Li[(4 * e + fr) * ldi + H + fc] = 0.0;
    }
  }
}

// a 64 x 64 block from global memory (row stride ld, even) to LDS (row
// stride LDB): thread t moves columns 2 (t % 32), +1 of rows t / 32 + 8 p,
// so each wave instruction moves two whole 512-byte rows in 16-byte pieces
__device__ inline void load_block64(const CVG_GLOBAL double* g, int64_t ld, double* S, int t) {
  const int r0 = t >> 5, c = (t & 31) * 2;
  double2_t v[8];
#pragma unroll
  for (int p = 0; p < 8; ++p) v[p] = *(const CVG_GLOBAL double2_t*)&g[(r0 + 8 * p) * ld + c];
#pragma unroll
  for (int p = 0; p < 8; ++p) *(double2_t*)&S[(r0 + 8 * p) * LDB + c] = v[p];
}

// C = X Y^T (32 x 32 over 32 terms; NEG: C = init - X Y^T) on the FP64
// matrix cores, wave w computing the 16 x 16 tile (tm, tn) = (w / 2, w % 2);
// X[r][c] at X[r * ldx + c]; Y[q][c] at Y[q * ldy + c], or at Y[c * ldy + q]
// when YT.  Element e of the result in lane (fr, fc) is
// C[16 tm + 4 e + fr][16 tn + fc].
template <bool YT, bool NEG>
__device__ inline double4_t mma32(const double* X, int ldx, const double* Y, int ldy, int tm,
                                  int tn, int fr, int fc, double4_t acc) {
#pragma unroll
  for (int kk = 0; kk < NB / 4; ++kk) {
    const double x = X[(16 * tm + fc) * ldx + 4 * kk + fr];
    const double y = YT ? Y[(4 * kk + fr) * ldy + 16 * tn + fc] : Y[(16 * tn + fc) * ldy + 4 * kk + fr];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(NEG ? -x : x, y, acc, 0, 0, 0);
  }
  return acc;
}

// Diagonal block s (64 x 64) of matrix mat by one 256-thread workgroup, the
// block already in S (LDS, row stride LDB, lower triangle valid; I1, I2: LDS
// scratch of 32 x 33 doubles each; the block's upper right quadrant, which
// is above the diagonal, holds a 32 x 32 intermediate).  The block is the 2 x 2 arrangement of 32 x 32 blocks
//   [A11 .; A21 A22] = [L11 0; L21 L22] [L11 0; L21 L22]^T
// so L11 = chol(A11) (one wave, above), L21 = A21 L11^{-T},
// L22 = chol(A22 - L21 L21^T) (one wave), and the inverse of the factor is
//   [L11^{-1} 0; -L22^{-1} L21 L11^{-1}  L22^{-1}].
// Written back: the factor to the block's lower triangle; the 64 x 64
// inverse to Linv64 (the panel step's operand) and the two 32 x 32 diagonal
// inverses to Linv32 (the backward substitution's).  The four 32 x 32
// products on the FP64 matrix cores, a 16 x 16 tile per wave.
__device__ __forceinline__ void diag64_body(double* S, double* I1, double* I2,
                                            CVG_GLOBAL double* a,
                            double* __restrict__ Linv64, double* __restrict__ Linv32,
                            int32_t* __restrict__ flags, int64_t Kp, int64_t mat, int32_t s,
                            int32_t nb64, int t) {
  constexpr int LI = NB + 1;
  double* T = S + NB;  // the upper right quadrant, row stride LDB
  CVG_GLOBAL double* blk = a + (int64_t)s * NB2 * Kp + (int64_t)s * NB2;
  const int lane = t & 63, w = t >> 6;
  const int fr = lane >> 4, fc = lane & 15, tm = w >> 1, tn = w & 1;
  const double4_t zero = {0.0, 0.0, 0.0, 0.0};
  // this lane's entries of a wave's tile: (16 tm + 4 e + fr, 16 tn + fc)
  auto at = [&](double* M, int ld, int e) -> double& {
    return M[(16 * tm + 4 * e + fr) * ld + 16 * tn + fc];
  };
  bool bad = false;  // meaningful in wave 0
  if (t < kWave) factor32_wave(S, LDB, I1, LI, t, bad);
  __syncthreads();
  double* S21 = S + NB * LDB;       // rows 32.., columns 0..
  double* S22 = S + NB * LDB + NB;  // rows 32.., columns 32..
  {
    // L21 = A21 L11^{-T}
    const double4_t c = mma32<false, false>(S21, LDB, I1, LI, tm, tn, fr, fc, zero);
    __syncthreads();  // every wave's reads of A21 are done
#pragma unroll
    for (int e = 0; e < 4; ++e) at(S21, LDB, e) = c[e];
  }
  __syncthreads();
  {
    // A22 -= L21 L21^T (each lane rewrites the entries it read)
    double4_t c;
#pragma unroll
    for (int e = 0; e < 4; ++e) c[e] = at(S22, LDB, e);
    c = mma32<false, true>(S21, LDB, S21, LDB, tm, tn, fr, fc, c);
#pragma unroll
    for (int e = 0; e < 4; ++e) at(S22, LDB, e) = c[e];
  }
  __syncthreads();
  if (t < kWave) factor32_wave(S22, LDB, I2, LI, t, bad);
  {
    // T = L21 L11^{-1}
    const double4_t c = mma32<true, false>(S21, LDB, I1, LI, tm, tn, fr, fc, zero);
#pragma unroll
    for (int e = 0; e < 4; ++e) at(T, LDB, e) = c[e];
  }
  __syncthreads();
  // the inverse's lower left quadrant: -L22^{-1} T
  const double4_t vq = mma32<true, false>(I2, LI, T, LDB, tm, tn, fr, fc, zero);
  CVG_GLOBAL double* li = gmem(Linv64) + (mat * nb64 + s) * NB2 * NB2;
  CVG_GLOBAL double* l32 = gmem(Linv32) + (mat * 2 * nb64 + 2 * s) * NB * NB;
#pragma unroll
  for (int e = 0; e < 4; ++e)
    li[(NB + 16 * tm + 4 * e + fr) * NB2 + 16 * tn + fc] = -vq[e];
  const int q = t % NB, rb = t / NB;  // this thread: column q of rows rb + 8 p
#pragma unroll
  for (int p = 0; p < kRowsPerThread; ++p) {
    const int r = rb + kRowStep * p;
    li[r * NB2 + q] = I1[r * LI + q];
    li[r * NB2 + NB + q] = 0.0;
    li[(NB + r) * NB2 + NB + q] = I2[r * LI + q];
    l32[r * NB + q] = I1[r * LI + q];
    l32[NB * NB + r * NB + q] = I2[r * LI + q];
    blk[r * Kp + q] = S[r * LDB + q];                      // L11
    blk[(NB + r) * Kp + q] = S[(NB + r) * LDB + q];        // L21
    blk[(NB + r) * Kp + NB + q] = S[(NB + r) * LDB + NB + q];  // L22
  }
  if (t == 0 && bad) flags[mat] = 1;
}

// The padded systems and their first diagonal block, in one launch.
// Padded system: A + lambda I in Kp x Kp (identity in the padding) and,
// below it, R^T in Ma rows of Kp (zeros in the padding), from the products
// (p-major, lambda-minor).  Of the square part only the 64 x 64 blocks on and
// below the diagonal are written: nothing reads the blocks above.  The rows
// of R^T are factored with the matrix (they become (L^{-1} R)^T: the forward
// substitution).
// grid: folds x n_lambda + folds x (copy blocks of a fold) workgroups.  The
// first n_mat workgroups factor diagonal block 0 of one matrix each (read
// from the products; the later diagonal blocks are factored by the trailing
// update that finishes them), dispatched first so that they run beside the
// copies instead of after them.  The others copy one 64 x 64 block (on or
// below the diagonal but block (0, 0), or of the R^T rows) into every
// penalty's matrix of one fold, two neighbouring columns of eight rows per
// thread, reading each product entry once.  The diagonal workgroups zero their matrix's flag
// first (only later diagonal steps set flags after them).
__global__ __launch_bounds__(kThreads) void ridge_setup_kernel(
    const double* __restrict__ xtx, const double* __restrict__ xty, RidgeLambdas lv,
    const double* __restrict__ lambdas, int32_t n_folds, int32_t n_lambda, int64_t K, int64_t M,
    int64_t Kp, int64_t Kr, double* __restrict__ A, double* __restrict__ Linv64,
    double* __restrict__ Linv32, int32_t* __restrict__ flags, int32_t nb64) {
  __shared__ double S[NB2 * LDB];
  __shared__ double I1[NB * (NB + 1)], I2[NB * (NB + 1)];
  // copy blocks per fold: the lower triangle of 64 x 64 blocks but (0, 0),
  // and the R^T rows' blocks
  const int64_t nblk = (Kp / NB2) * (Kp / NB2 + 1) / 2 - 1 + (Kr - Kp) / NB2 * (Kp / NB2);
  const int64_t b = blockIdx.x, n_mat = (int64_t)n_folds * n_lambda;
  const bool diag = b < n_mat;
  const int64_t f = diag ? b / n_lambda : (b - n_mat) / nblk;
  const int t = threadIdx.x;
  const CVG_GLOBAL double* src = gmem(xtx) + f * K * K;
  const CVG_GLOBAL double* rs = gmem(xty) + f * K * M;
  auto value = [&](int64_t i, int64_t j) {
    if (i >= Kp) {  // R^T
      const int64_t m = i - Kp;
      return (m < M && j < K) ? rs[j * M + m] : 0.0;
    }
    return (i < K && j < K) ? src[i * K + j] : (i == j ? 1.0 : 0.0);
  };
  // penalty l: by value, or from the device array when there are more
  auto lam_of = [&](int32_t l) { return lambdas ? lambdas[l] : lv.v[l]; };
  if (diag) {
    const int64_t mat = b;
    const double lam = lam_of((int32_t)(b % n_lambda));
    if (t == 0) flags[mat] = 0;  // diag64_body (thread 0 too) sets it on a bad pivot
    const int r0 = t >> 5, c = (t & 31) * 2;
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      const int r = r0 + 8 * p;
      double2_t v;
      v.x = value(r, c) + (r < K && r == c ? lam : 0.0);
      v.y = value(r, c + 1) + (r < K && r == c + 1 ? lam : 0.0);
      *(double2_t*)&S[r * LDB + c] = v;
    }
    __syncthreads();
    diag64_body(S, I1, I2, gmem(A) + mat * Kr * Kp, Linv64, Linv32, flags, Kp, mat, 0, nb64,
                t);
    return;
  }
  // a copy workgroup: one 64 x 64 block of every penalty's matrix of the
  // fold, the blocks on and below the diagonal counted row by row from
  // block (1, 0), then the R^T rows' blocks
  CVG_GLOBAL double* dst = gmem(A) + f * n_lambda * Kr * Kp;
  int32_t bi, bk;
  {
    const int32_t idx = (int32_t)((b - n_mat) % nblk) + 1;  // 0 would be block (0, 0)
    const int32_t ntri = nb64 * (nb64 + 1) / 2;
    if (idx < ntri) {
      int32_t kk = idx, ii = 0;
      while (kk > ii) {
        kk -= ii + 1;
        ++ii;
      }
      bi = ii;
      bk = kk;
    } else {
      const int32_t r = idx - ntri;
      bi = nb64 + r / nb64;
      bk = r % nb64;
    }
  }
  // this thread: columns c, c + 1 of rows r0 + 8 p of the block; the loads
  // first, all in flight together, then the copies
  const int r0 = t >> 5, c = (t & 31) * 2;
  const int64_t i0 = (int64_t)bi * NB2 + r0, j = (int64_t)bk * NB2 + c;
  double2_t v[NB2 / 8];
#pragma unroll
  for (int p = 0; p < NB2 / 8; ++p) {
    v[p].x = value(i0 + 8 * p, j);
    v[p].y = value(i0 + 8 * p, j + 1);
  }
  for (int32_t l = 0; l < n_lambda; ++l) {
    const double lam = lam_of(l);
#pragma unroll
    for (int p = 0; p < NB2 / 8; ++p) {
      const int64_t i = i0 + 8 * p;
      // lambda on the diagonal of the K x K part
      double2_t w = v[p];
      if (i < K && i == j) w.x += lam;
      if (i < K && i == j + 1) w.y += lam;
      *(CVG_GLOBAL double2_t*)&dst[(l * Kr + i) * Kp + j] = w;
    }
  }
}

// C[r][q] += sum_c sign * X[r][c] Y[q][c] over a 64 x 64 tile, X and Y 64 x 64
// in LDS: wave w computes rows 32 (w / 2) .., columns 32 (w % 2) .. as 2 x 2
// blocks of v_mfma_f64_16x16x4f64 over 16 steps of 4 c.  Element e of
// acc[a][b] in lane (fr = lane / 16, fc = lane % 16) is
//   C[32 wm + 16 a + 4 e + fr][32 wn + 16 b + fc].
template <bool NEG>
__device__ inline void mma64(const double* X, const double* Y, double4_t (&acc)[2][2], int wm,
                             int wn, int fr, int fc) {
#pragma unroll 4
  for (int kk = 0; kk < NB2 / 4; ++kk) {
    double af[2], bf[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const double x = X[(32 * wm + 16 * u + fc) * LDB + 4 * kk + fr];
      af[u] = NEG ? -x : x;
    }
#pragma unroll
    for (int w = 0; w < 2; ++w) bf[w] = Y[(32 * wn + 16 * w + fc) * LDB + 4 * kk + fr];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int w = 0; w < 2; ++w)
        acc[u][w] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[u], bf[w], acc[u][w], 0, 0, 0);
  }
}


// panel: L_is = A_is Linv_ss^T for block rows i > s (64 x 64 blocks, FP64
// MFMA), in place; the naug block rows below the matrix (R^T) take the same
// step (products only for their rows below M).  A workgroup forms 32 rows
// of a block (half the chain of products of a whole block, and LDS for
// three workgroups a CU): wave w the 16 rows 16 (w / 2) .. and 32 columns
// 32 (w % 2) ... grid (mat_block_grid): matrices x 2 x (block rows below
// s: nb64 - 1 - s of the matrix, then naug), the two halves of a block
// adjacent.
__global__ __launch_bounds__(kThreads) void chol_panel64_kernel(double* __restrict__ A,
                                                                const double* __restrict__ Linv64,
                                                                int64_t Kp, int64_t Kr, int64_t M,
                                                                int64_t n_mat, int32_t s,
                                                                int32_t nb64) {
  __shared__ double Xs[NB * LDB], Ys[NB2 * LDB];
  int64_t mat;
  int32_t y;
  mat_and_block(n_mat, mat, y);
  const int32_t ib = s + 1 + (y >> 1);  // >= nb64: a row block of R^T
  const int h = y & 1;                  // rows 32 h .. 32 h + 31
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int fr = lane >> 4, fc = lane & 15, wm = w >> 1, wn = w & 1;
  CVG_GLOBAL double* a = gmem(A) + mat * Kr * Kp;
  CVG_GLOBAL double* blk = a + ((int64_t)ib * NB2 + NB * h) * Kp + (int64_t)s * NB2;
  const CVG_GLOBAL double* li = gmem(Linv64) + (mat * nb64 + s) * NB2 * NB2;
  const int r0 = t >> 5, c0 = (t & 31) * 2;  // thread: columns c0, c0 + 1 of rows r0 + 8 p
  {
    double2_t v[NB / 8];
#pragma unroll
    for (int p = 0; p < NB / 8; ++p) v[p] = *(const CVG_GLOBAL double2_t*)&blk[(r0 + 8 * p) * Kp + c0];
#pragma unroll
    for (int p = 0; p < NB / 8; ++p) *(double2_t*)&Xs[(r0 + 8 * p) * LDB + c0] = v[p];
  }
  load_block64(li, NB2, Ys, t);
  __syncthreads();
  // the wave's rows hold rows of the system (a block of R^T: below row M)
  const bool live = ib < nb64 || M - (int64_t)(ib - nb64) * NB2 - NB * h - 16 * wm > 0;
  double4_t acc[2] = {double4_t{0.0, 0.0, 0.0, 0.0}, double4_t{0.0, 0.0, 0.0, 0.0}};
  if (live) {
#pragma unroll 4
    for (int kk = 0; kk < NB2 / 4; ++kk) {
      const double x = Xs[(16 * wm + fc) * LDB + 4 * kk + fr];
#pragma unroll
      for (int v = 0; v < 2; ++v)
        acc[v] = __builtin_amdgcn_mfma_f64_16x16x4f64(
            x, Ys[(32 * wn + 16 * v + fc) * LDB + 4 * kk + fr], acc[v], 0, 0, 0);
    }
  }
  __syncthreads();  // every wave's reads of Xs are done
#pragma unroll
  for (int v = 0; v < 2; ++v)
#pragma unroll
    for (int e = 0; e < 4; ++e) Xs[(16 * wm + 4 * e + fr) * LDB + 32 * wn + 16 * v + fc] = acc[v][e];
  __syncthreads();
#pragma unroll
  for (int p = 0; p < NB / 8; ++p)
    *(CVG_GLOBAL double2_t*)&blk[(r0 + 8 * p) * Kp + c0] = *(const double2_t*)&Xs[(r0 + 8 * p) * LDB + c0];
}

// trailing update A_ik -= L_is L_ks^T for s < k <= i (64 x 64 blocks, FP64
// MFMA accumulating onto A_ik: the negated L_is is the first operand).
// Workgroup 0 of a matrix owns block (s + 1, s + 1), the next diagonal
// block: once its update is complete (no other workgroup writes it), it
// keeps the block in LDS and factors it (diag64_body), so the next step's
// diagonal work runs beside the rest of this update instead of in a launch
// of its own.  Every other block is updated by two workgroups of 32 rows
// each (half the chain of products of a whole block, and LDS for three
// workgroups a CU): wave w the 16 rows 16 (w / 2) .. and 32 columns
// 32 (w % 2) .. of its half.  Waves whose tile lies above the diagonal of a
// diagonal block, or in the zero rows of R^T, have nothing to compute.
// grid (mat_block_grid): matrices x (1 + 2 x the other blocks: the lower
// triangle of the remaining blocks counted row by row, then naug x
// (nb64 - 1 - s) blocks of the R^T rows below the matrix; the halves of a
// block adjacent)
__global__ __launch_bounds__(kThreads) void chol_update64_kernel(double* __restrict__ A,
                                                                 double* __restrict__ Linv64,
                                                                 double* __restrict__ Linv32,
                                                                 int32_t* __restrict__ flags,
                                                                 int64_t Kp, int64_t Kr, int64_t M,
                                                                 int64_t n_mat, int32_t s,
                                                                 int32_t nb64) {
  // P: a 64-row block; Q: a 32-row half (non-owners) or the diagonal step's
  // two 32 x 33 inverses (the owner)
  __shared__ double P[NB2 * LDB], Q[NB * LDB];
  static_assert(2 * NB * (NB + 1) <= NB * LDB, "the two inverses must fit in Q");
  int64_t mat;
  int32_t y;
  mat_and_block(n_mat, mat, y);
  const int32_t below = nb64 - 1 - s;
  const int32_t tri = below * (below + 1) / 2;
  const bool owner = y == 0;  // block (s + 1, s + 1)
  const int32_t bidx = owner ? 0 : 1 + (y - 1) / 2;
  const int h = owner ? 0 : (y - 1) & 1;  // rows 32 h .. of the block
  int32_t ib, kb;
  if (bidx < tri) {
    int32_t kk = bidx, ii = 0;
    while (kk > ii) {
      kk -= ii + 1;
      ++ii;
    }
    ib = s + 1 + ii;
    kb = s + 1 + kk;
  } else {  // a block of the R^T rows
    const int32_t r = bidx - tri, ia = r / below;
    ib = nb64 + ia;
    kb = s + 1 + (r - ia * below);
  }
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int fr = lane >> 4, fc = lane & 15, wm = w >> 1, wn = w & 1;
  CVG_GLOBAL double* a = gmem(A) + mat * Kr * Kp;
  if (!owner) {
    CVG_GLOBAL double* out = a + ((int64_t)ib * NB2 + NB * h) * Kp + (int64_t)kb * NB2;
    // rows 32 h + 16 wm .. + 15, columns 32 wn .. + 31 of the block
    const bool act = (ib != kb || NB * h + 16 * wm + 15 >= 32 * wn) &&
                     (ib < nb64 || M - (int64_t)(ib - nb64) * NB2 - NB * h - 16 * wm > 0);
    double4_t acc[2];
    if (act) {
#pragma unroll
      for (int v = 0; v < 2; ++v)
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[v][e] = out[(16 * wm + 4 * e + fr) * Kp + 32 * wn + 16 * v + fc];
    }
    // Q: rows 32 h .. of L_is; P: L_ks
    {
      const CVG_GLOBAL double* xs = a + ((int64_t)ib * NB2 + NB * h) * Kp + (int64_t)s * NB2;
      const int r0 = t >> 5, c0 = (t & 31) * 2;
      double2_t v[NB / 8];
#pragma unroll
      for (int p = 0; p < NB / 8; ++p) v[p] = *(const CVG_GLOBAL double2_t*)&xs[(r0 + 8 * p) * Kp + c0];
#pragma unroll
      for (int p = 0; p < NB / 8; ++p) *(double2_t*)&Q[(r0 + 8 * p) * LDB + c0] = v[p];
    }
    load_block64(a + (int64_t)kb * NB2 * Kp + (int64_t)s * NB2, Kp, P, t);
    __syncthreads();
    if (!act) return;
#pragma unroll 4
    for (int kk = 0; kk < NB2 / 4; ++kk) {
      const double x = -Q[(16 * wm + fc) * LDB + 4 * kk + fr];
#pragma unroll
      for (int v = 0; v < 2; ++v)
        acc[v] = __builtin_amdgcn_mfma_f64_16x16x4f64(
            x, P[(32 * wn + 16 * v + fc) * LDB + 4 * kk + fr], acc[v], 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 2; ++v)
#pragma unroll
      for (int e = 0; e < 4; ++e) out[(16 * wm + 4 * e + fr) * Kp + 32 * wn + 16 * v + fc] = acc[v][e];
    return;
  }
  // the owner: the whole diagonal block, A_ii -= L_is L_is^T (the wave of
  // the upper right quadrant idle), then its factorisation
  CVG_GLOBAL double* out = a + (int64_t)ib * NB2 * Kp + (int64_t)kb * NB2;
  const bool idle = wm < wn;
  double4_t acc[2][2];
  if (!idle) {
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int v = 0; v < 2; ++v)
#pragma unroll
        for (int e = 0; e < 4; ++e)
          acc[u][v][e] = out[(32 * wm + 16 * u + 4 * e + fr) * Kp + 32 * wn + 16 * v + fc];
  }
  load_block64(a + (int64_t)ib * NB2 * Kp + (int64_t)s * NB2, Kp, P, t);
  __syncthreads();
  if (!idle) mma64<true>(P, P, acc, wm, wn, fr, fc);
  // the updated block to LDS (its lower triangle; the idle wave's quadrant
  // is above the diagonal), then the factorisation of it
  __syncthreads();  // every wave's reads of P are done
  if (!idle) {
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int v = 0; v < 2; ++v)
#pragma unroll
        for (int e = 0; e < 4; ++e)
          P[(32 * wm + 16 * u + 4 * e + fr) * LDB + 32 * wn + 16 * v + fc] = acc[u][v][e];
  }
  __syncthreads();
  diag64_body(P, Q, Q + NB * (NB + 1), a, Linv64, Linv32, flags, Kp, mat, s + 1, nb64, t);
}

// The backward substitution W = L^{-T} Z in one launch (Z = L^{-1} R, from
// the factorisation): workgroup (matrix, block of 32 columns of R) walks the
// block steps itself, last block first:
//   step j:  W_j = Linv_jj^T R_j;  R_i -= L_ji^T W_j   for i < j
// The coefficient of W[c] in row i is A[r0 + c][i], the factor's block row j
// in the lower triangle.  One thread per row of R reads those 32 values along
// a row of A, consecutive threads consecutive columns, all loads in flight.
// The rows of the next step's block go on to it through LDS as they are
// updated, and the next diagonal inverse is loaded during the update, so a
// step waits on memory once.  Each workgroup owns its rows x columns of R:
// its own writes are the only ones it reads back (ordered by the barriers
// between steps).  Padding rows of the last block (past K) stay zero.  MW
// (8, 16 or 32) is the width of R each row update carries in registers: at
// least the block's columns of B, the rest padding zeros that stay zero.
template <int MW, bool FAST>
__global__ __launch_bounds__(solve_threads<MW>()) void tri_solve_kernel(const double* __restrict__ A,
                                                             const double* __restrict__ Linv,
                                                             double* __restrict__ R, int64_t K,
                                                             int64_t M, int64_t Kp, int64_t Kr,
                                                             int64_t Mp, int32_t nblk) {
  __shared__ double Z[NB][NB + 1];
  __shared__ double Li[2][NB][NB + 1];
  __shared__ double Rb[NB][NB + 1];
  const int64_t mat = blockIdx.x;
  const int64_t m0 = (int64_t)blockIdx.y * NB;
  const CVG_GLOBAL double* a = gmem(A) + mat * Kr * Kp;
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
  {
    {
      // the first block (the last one): its rows of R and its inverse
      const int32_t j = nblk - 1;
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
    // keeps row t for the whole walk, so an update reads no R from memory,
    // and the coefficients of its next step are loaded at the end of this
    // one, while the barrier and the next block's Z are in progress.
    double rv[MW], lc[NB];
    if (fast) {
      const int32_t j = nblk - 1;
      const int64_t lo = 0, hi = (int64_t)j * NB;
      if (t < Kp) {
#pragma unroll
        for (int mm = 0; mm < MW; ++mm) rv[mm] = rr[(int64_t)t * Mp + mm];
      }
      if (t >= lo && t < hi) {
#pragma unroll
        for (int c = 0; c < NB; ++c) lc[c] = a[((int64_t)j * NB + c) * Kp + t];
      }
    }
#pragma unroll 1
    for (int32_t jj = 0; jj < nblk; ++jj) {
      const int32_t j = nblk - 1 - jj;
      const int64_t r0 = (int64_t)j * NB;
      const bool last = jj + 1 == nblk;
      const int32_t jn = j - 1;  // the next step's block
      const int64_t n0 = (int64_t)jn * NB;
      if (blk) {
#pragma unroll
        for (int q = 0; q < kRowsPerThread; ++q) {
          const int r = ty + kRowStep * q;
          // all 32 terms, unrolled: the inverse block holds exact zeros
          // above its diagonal, so the terms outside the triangle add zero
          // and the sum is that of the triangle, in the same order
          double sum = 0.0;
#pragma unroll
          for (int k = 0; k < NB; ++k) {
            sum = fma(Li[buf][k][r], Rb[k][tx], sum);
            if (k % 8 == 7) __builtin_amdgcn_sched_barrier(0);
          }
          Z[r][tx] = sum;
          rr[(r0 + r) * Mp + tx] = sum;
        }
      }
      // the stages below stay in order: the next coefficients' loads are
      // not hoisted above this step's sums (both sets would be live)
      __builtin_amdgcn_sched_barrier(0);
      __syncthreads();
      double vl[kRowsPerThread];
      if (!last && blk) load_li(jn, vl);
      const int64_t lo = 0, hi = r0;
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
        // the next step's rows of the update: [0, n0)
        __builtin_amdgcn_sched_barrier(0);
        const int64_t lo_n = 0, hi_n = n0;
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


// The backward substitution on the FP64 matrix cores, for Kp <= 512: one
// workgroup of 8 waves per (matrix, 16 columns of B).  The columns of
// R = (L^{-1} R)^T's transpose are read from the factorisation's R^T rows
// and stay in the accumulators for the whole walk: row tile tau (rows
// 16 tau .. 16 tau + 15) belongs to wave tau % 8, slot tau / 8, as one
// 16 x 16 v_mfma_f64_16x16x4f64 tile.  Step j (32 rows from r0 = 32 j, last
// block first):
//   1. the two owners put block j's rows (final: every later block's
//      update is applied) in LDS;
//   2. waves 0 and 1 form W_j = Linv_jj^T R_j, 16 rows each (8 MFMAs over
//      the 32 rows of the block), into LDS and into B (rows below K,
//      columns below M);
//   3. every wave updates its tiles above the block, R_i -= L_ji^T W_j
//      (8 MFMAs a tile, the negated coefficients L[r0 + c][i] as the first
//      operand, read along rows of the factor's block row j).
// The coefficients of the next step are loaded during this one's update.
// Only W crosses between waves (one LDS value per lane per MFMA), where a
// row-per-thread update reads all of W from LDS in every wave.
constexpr int kTsWaves = 8;
constexpr int kTsSlots = 4;  // 16-row tiles per wave: Kp <= 8 x 4 x 16
constexpr int kTsCols = 16;
__global__ __launch_bounds__(kTsWaves * kWave) void tri_solve_mfma_kernel(
    const double* __restrict__ A, const double* __restrict__ Linv, const double* __restrict__ Linv64,
    double* __restrict__ B, int64_t K, int64_t M, int64_t Kp, int64_t Kr, int32_t nblk) {
  __shared__ double Rb[NB][kTsCols + 1];
  __shared__ double Zs[NB][kTsCols + 1];
  const int64_t mat = blockIdx.x;
  const int64_t m0 = (int64_t)blockIdx.y * kTsCols;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int fr = lane >> 4, fc = lane & 15;
  const CVG_GLOBAL double* a = gmem(A) + mat * Kr * Kp;
  const int32_t ntile = (int32_t)(Kp / 16);
  // R[i][m0 + c] = R^T[m0 + c][i], rows of R^T below the factor.  The last
  // 64-row block has not been through its panel step (the factorisation
  // leaves it to this kernel): its four tiles are formed here as
  // Linv64_last (R^T rows)^T, 16 MFMAs over the block's 64 rows.
  const int32_t tlast = ntile - 4;  // first tile of the last 64-row block
  const int64_t rlast = Kp - NB2;
  double4_t acc[kTsSlots];
#pragma unroll
  for (int sl = 0; sl < kTsSlots; ++sl) {
    const int32_t tau = w + kTsWaves * sl;
    if (tau < tlast) {
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[sl][e] = a[(Kp + m0 + fc) * Kp + 16 * tau + 4 * e + fr];
    } else if (tau < ntile) {
      const CVG_GLOBAL double* li =
          gmem(Linv64) + (mat * (Kp / NB2) + Kp / NB2 - 1) * NB2 * NB2 + (16 * (tau - tlast) + fc) * NB2;
      const CVG_GLOBAL double* rt = a + (Kp + m0 + fc) * Kp + rlast;
      double4_t z = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kk = 0; kk < NB2 / 4; ++kk)
        z = __builtin_amdgcn_mfma_f64_16x16x4f64(li[4 * kk + fr], rt[4 * kk + fr], z, 0, 0, 0);
      acc[sl] = z;
    } else {
      acc[sl] = double4_t{0.0, 0.0, 0.0, 0.0};
    }
  }
  // coefficients of step j for the tiles above its block (negated as the
  // MFMA operand, so the loads are not waited for until the products):
  // cf[sl][kk] = L[32 j + 4 kk + fr][16 tau + fc]
  double cf[kTsSlots][8];
  auto load_cf = [&](int32_t j) {
#pragma unroll
    for (int sl = 0; sl < kTsSlots; ++sl) {
      const int32_t tau = w + kTsWaves * sl;
      if (tau < 2 * j) {
#pragma unroll
        for (int kk = 0; kk < 8; ++kk)
          cf[sl][kk] = a[((int64_t)j * NB + 4 * kk + fr) * Kp + 16 * tau + fc];
      }
    }
  };
  // Linv_jj^T for wave h < 2: lf[kk] = Linv_jj[4 kk + fr][16 h + fc]
  double lf[8];
  auto load_lf = [&](int32_t j) {
    if (w < 2) {
      const CVG_GLOBAL double* li = gmem(Linv) + (mat * nblk + j) * NB * NB;
#pragma unroll
      for (int kk = 0; kk < 8; ++kk) lf[kk] = li[(4 * kk + fr) * NB + 16 * w + fc];
    }
  };
  load_cf(nblk - 1);
  load_lf(nblk - 1);
#pragma unroll 1
  for (int32_t j = nblk - 1; j >= 0; --j) {
    const int64_t r0 = (int64_t)j * NB;
    // 1. block j's two tiles (2 j, 2 j + 1) to LDS
#pragma unroll
    for (int sl = 0; sl < kTsSlots; ++sl) {
      const int32_t tau = w + kTsWaves * sl;
      if (tau == 2 * j || tau == 2 * j + 1) {
        const int h = tau - 2 * j;
#pragma unroll
        for (int e = 0; e < 4; ++e) Rb[16 * h + 4 * e + fr][fc] = acc[sl][e];
      }
    }
    __syncthreads();
    // 2. W_j = Linv_jj^T R_j
    if (w < 2) {
      double4_t z = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kk = 0; kk < 8; ++kk)
        z = __builtin_amdgcn_mfma_f64_16x16x4f64(lf[kk], Rb[4 * kk + fr][fc], z, 0, 0, 0);
      const int64_t m = m0 + fc;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int rl = 16 * w + 4 * e + fr;
        Zs[rl][fc] = z[e];
        const int64_t r = r0 + rl;
        if (r < K && m < M) gmem(B)[(mat * K + r) * M + m] = z[e];
      }
    }
    __syncthreads();
    if (j > 0) load_lf(j - 1);
    // 3. R_i -= L_ji^T W_j for the tiles above the block
    double bz[8];
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) bz[kk] = Zs[4 * kk + fr][fc];
#pragma unroll
    for (int sl = 0; sl < kTsSlots; ++sl) {
      const int32_t tau = w + kTsWaves * sl;
      if (tau < 2 * j) {
#pragma unroll
        for (int kk = 0; kk < 8; ++kk)
          acc[sl] = __builtin_amdgcn_mfma_f64_16x16x4f64(-cf[sl][kk], bz[kk], acc[sl], 0, 0, 0);
      }
    }
    if (j > 0) load_cf(j - 1);
  }
}

}  // namespace

void ridge_solve(const double* xtx, const double* xty, const RidgeLambdas& lam,
                 const double* lambdas_dev, int32_t n_folds, int32_t n_lambda, int64_t K,
                 int64_t M, double* A, double* R, double* Linv, int32_t* flags, double* B,
                 hipStream_t s) {
  const int64_t n_mat = (int64_t)n_folds * n_lambda;
  if (n_mat <= 0 || K <= 0) return;
  const int64_t Kp = ridge_padded_k(K), Mp = (M + NB - 1) / NB * NB;
  const int32_t nb64 = (int32_t)(Kp / NB2), nblk = (int32_t)(Kp / NB);
  double* Linv64 = Linv;                                // [n_mat][nb64][64][64]
  double* Linv32 = Linv + n_mat * nb64 * NB2 * NB2;     // [n_mat][nblk][32][32]
  const int64_t Ma = ridge_aug_rows(M), Kr = Kp + Ma;
  const int32_t naug = (int32_t)(Ma / NB2);
  // the padded systems and diagonal block 0, then per block column s: the
  // panel below it (the matrix's block rows and the R^T rows) and the
  // trailing update, which also factors diagonal block s + 1
  const int64_t setup_blocks = (int64_t)nb64 * (nb64 + 1) / 2 - 1 + (int64_t)naug * nb64;
  ridge_setup_kernel<<<(unsigned)(n_mat + n_folds * setup_blocks), kThreads, 0, s>>>(
      xtx, xty, lam, lambdas_dev, n_folds, n_lambda, K, M, Kp, Kr, A, Linv64, Linv32, flags, nb64);
  CVG_LAUNCH_CHECK();
  // the substitution on the matrix cores forms the last block column's panel
  // (its R^T rows only) itself
  const bool mfma_solve = ridge_solve_on_matrix_cores(Kp, M);
  static_assert(kTsWaves * kTsSlots * 16 == 512, "the matrix-core substitution covers Kp <= 512");
  for (int32_t j = 0; j < nb64; ++j) {
    const int32_t below = nb64 - j - 1;
    if (below + naug > 0 && !(below == 0 && mfma_solve)) {
      chol_panel64_kernel<<<mat_block_grid(n_mat, 2 * (below + naug)), kThreads, 0, s>>>(
          A, Linv64, Kp, Kr, M, n_mat, j, nb64);
      CVG_LAUNCH_CHECK();
    }
    if (below > 0) {
      const int32_t blocks = below * (below + 1) / 2 + naug * below;
      chol_update64_kernel<<<mat_block_grid(n_mat, 2 * (int64_t)blocks - 1), kThreads, 0, s>>>(
          A, Linv64, Linv32, flags, Kp, Kr, M, n_mat, j, nb64);
      CVG_LAUNCH_CHECK();
    }
  }
  if (M <= 0) return;
  // the forward substitution is done ((L^{-1} R)^T below the factor, but for
  // the last block column with the substitution on the matrix cores)
  if (mfma_solve) {
    const dim3 grid((unsigned)n_mat, (unsigned)((M + kTsCols - 1) / kTsCols));
    tri_solve_mfma_kernel<<<grid, kTsWaves * kWave, 0, s>>>(A, Linv32, Linv64, B, K, M, Kp, Kr,
                                                             nblk);
    CVG_LAUNCH_CHECK();
    return;
  }
  const unsigned mat_y = (unsigned)(n_mat < 65535 ? n_mat : 65535);  // grid.y strides
  ridge_z_kernel<<<dim3((unsigned)(Kp / 8), mat_y), kThreads, 0, s>>>(A, Kp, Kr, Mp, n_mat, R);
  CVG_LAUNCH_CHECK();
  const dim3 grid((unsigned)n_mat, (unsigned)(Mp / NB));
  const bool fast = Kp <= solve_threads<16>();  // one row of R per thread
  if (M <= 8 && fast)
    tri_solve_kernel<8, true><<<grid, solve_threads<8>(), 0, s>>>(A, Linv32, R, K, M, Kp, Kr, Mp,
                                                                    nblk);
  else if (M <= 8)
    tri_solve_kernel<8, false><<<grid, solve_threads<8>(), 0, s>>>(A, Linv32, R, K, M, Kp, Kr, Mp,
                                                                     nblk);
  else if (M <= 16 && fast)
    tri_solve_kernel<16, true><<<grid, solve_threads<16>(), 0, s>>>(A, Linv32, R, K, M, Kp, Kr,
                                                                      Mp, nblk);
  else if (M <= 16)
    tri_solve_kernel<16, false><<<grid, solve_threads<16>(), 0, s>>>(A, Linv32, R, K, M, Kp, Kr,
                                                                       Mp, nblk);
  else
    tri_solve_kernel<NB, false><<<grid, solve_threads<NB>(), 0, s>>>(A, Linv32, R, K, M, Kp, Kr,
                                                                       Mp, nblk);
  CVG_LAUNCH_CHECK();
  {
    const int64_t per = (K * M + kThreads - 1) / kThreads;
    dim3 grid((unsigned)(per < 1024 ? per : 1024), mat_y);
    ridge_store_kernel<<<grid, kThreads, 0, s>>>(R, K, M, Kp, Mp, n_mat, B);
    CVG_LAUNCH_CHECK();
  }
}

}  // namespace cvg
