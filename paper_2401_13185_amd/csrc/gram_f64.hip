// Grouped validation-block Gram products in FP64 on the matrix cores.
//
// For every fold p (Algorithm 7 step 8, Lemmas 2-3) the library needs
// G_p = Z'_{V_p}^T Z'_{V_p} restricted to its first K rows, where
// Z' = [X - 1 c_x^T | Y - 1 c_y^T] is the pivot-shifted data.  All folds run
// in ONE launch: a work list holds (fold, row range, output tile) items; the
// rows of a fold are contiguous in the fold permutation, so an item streams
// rows perm[r0 .. r1) and gathers them from X and Y.  Only tiles on or above
// the diagonal of the K x K block are computed (the lower triangle is the
// mirror image), plus every tile of the K x M block.  Each item writes its
// FP64 tile to its own slab; slabs are summed later in a fixed order, so the
// result is deterministic (no floating-point atomics).
//
// The contraction runs along rows: both MFMA operands are read from row-major
// tiles of Z' staged in LDS (a BK x BM block of rows x columns), which is the
// natural layout of v_mfma_f64_16x16x4_f64's A (16 x 4) and B (4 x 16)
// fragments: lane l holds column (l mod 16) of row (l / 16) of the 4-row step.
// The 16 x 16 result is spread as row (4 e + l / 16), column (l mod 16) for
// element e of lane l (checked on the device).
#include "internal.h"

namespace cvg {
namespace {

typedef double double4_t __attribute__((ext_vector_type(4)));

constexpr int kBK = 16;        // rows per LDS stage (4 MFMA k-steps)
constexpr int kThreads = 256;  // 4 waves in a 2 x 2 layout

template <typename T>
__device__ inline double zload(const T* __restrict__ X, const T* __restrict__ Y, int64_t K,
                               int64_t M, int64_t row, int64_t j) {
  return j < K ? (double)X[row * K + j] : (double)Y[row * M + (j - K)];
}

template <typename TIn, int BM>
__global__ __launch_bounds__(kThreads) void gram_f64_kernel(
    const TIn* __restrict__ X, const TIn* __restrict__ Y, int64_t K, int64_t M,
    const int32_t* __restrict__ perm, const double* __restrict__ pivot,
    const GramWork* __restrict__ work, int64_t n_work, double* __restrict__ slabs) {
  constexpr int WT = BM / 2;        // wave tile edge
  constexpr int NB = WT / 16;       // MFMA blocks per wave edge
  constexpr int TPR = kThreads / kBK;  // loader threads per staged row
  constexpr int CPT = BM / TPR;     // columns per loader thread
  constexpr int LD = BM + 1;        // padded LDS row
  __shared__ double As[kBK * LD];
  __shared__ double Bs[kBK * LD];

  // XCD-aware mapping: consecutive workgroup ids go round-robin over the 8
  // XCDs; give each XCD a contiguous range of items so tiles that share rows
  // share one L2.
  const int64_t per = (int64_t)gridDim.x / 8;
  const int64_t item = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (item >= n_work) return;
  const GramWork w = work[item];
  const int64_t W = K + M;
  const int64_t i0 = (int64_t)w.ti * BM;
  const int64_t j0 = (int64_t)w.tj * BM;
  const bool diag = w.ti == w.tj;

  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const bool active = !(diag && wm > wn);  // wave tile strictly below the diagonal

  // loader: row lk of the stage, columns lc .. lc+CPT-1 of the tile
  const int lk = t / TPR;
  const int lc = (t % TPR) * CPT;
  double pa[CPT], pb[CPT];
  bool va[CPT], vb[CPT];
#pragma unroll
  for (int u = 0; u < CPT; ++u) {
    const int64_t gi = i0 + lc + u, gj = j0 + lc + u;
    va[u] = gi < K;
    vb[u] = gj < W;
    pa[u] = va[u] ? pivot[gi] : 0.0;
    pb[u] = vb[u] ? pivot[gj] : 0.0;
  }

  double ra[CPT], rb[CPT];
  auto load_stage = [&](int64_t r) {
    const int64_t rr = r + lk;
    const bool vr = rr < w.r1;
    const int64_t n = vr ? (int64_t)perm[rr] : 0;
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
      ra[u] = (vr && va[u]) ? (double)X[n * K + i0 + lc + u] - pa[u] : 0.0;
      rb[u] = (vr && vb[u]) ? zload(X, Y, K, M, n, j0 + lc + u) - pb[u] : 0.0;
    }
  };
  auto store_stage = [&]() {
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
      As[lk * LD + lc + u] = ra[u];
      Bs[lk * LD + lc + u] = rb[u];
    }
  };

  double4_t acc[NB][NB];
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[a][b] = double4_t{0.0, 0.0, 0.0, 0.0};

  const int fr = lane >> 4;   // fragment row inside a 4-row k-step
  const int fc = lane & 15;   // fragment column inside a 16-wide block

  load_stage(w.r0);
  store_stage();
  __syncthreads();
  for (int64_t r = w.r0; r < w.r1; r += kBK) {
    const bool has_next = r + kBK < w.r1;
    if (has_next) load_stage(r + kBK);
    if (active) {
#pragma unroll
      for (int kk = 0; kk < kBK / 4; ++kk) {
        double af[NB], bf[NB];
#pragma unroll
        for (int a = 0; a < NB; ++a) af[a] = As[(kk * 4 + fr) * LD + wm * WT + a * 16 + fc];
#pragma unroll
        for (int b = 0; b < NB; ++b) bf[b] = Bs[(kk * 4 + fr) * LD + wn * WT + b * 16 + fc];
#pragma unroll
        for (int a = 0; a < NB; ++a)
#pragma unroll
          for (int b = 0; b < NB; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bf[b], acc[a][b], 0, 0, 0);
      }
    }
    __syncthreads();
    if (has_next) {
      store_stage();
      __syncthreads();
    }
  }

  if (!active) return;
  double* out = slabs + (int64_t)w.slab * K * W;
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        // v_mfma_f64_16x16x4_f64 keeps row (4 * e + lane / 16) of the 16 x 16
        // block in element e of lane l's accumulator (column lane mod 16)
        const int64_t row = i0 + wm * WT + a * 16 + 4 * e + fr;
        const int64_t col = j0 + wn * WT + b * 16 + fc;
        if (row < K && col < W) out[row * W + col] = acc[a][b][e];
      }
}

template <typename TIn>
void launch_typed(const TIn* X, const TIn* Y, int64_t K, int64_t M, const int32_t* perm,
                  const double* pivot, const GramWork* work, int64_t n_work, int tile,
                  double* slabs, hipStream_t s) {
  const int64_t grid = 8 * ((n_work + 7) / 8);
  if (tile == 128)
    gram_f64_kernel<TIn, 128><<<(unsigned)grid, kThreads, 0, s>>>(X, Y, K, M, perm, pivot, work,
                                                                  n_work, slabs);
  else
    gram_f64_kernel<TIn, 64><<<(unsigned)grid, kThreads, 0, s>>>(X, Y, K, M, perm, pivot, work,
                                                                 n_work, slabs);
  CVG_LAUNCH_CHECK();
}

}  // namespace

void launch_gram_f64(const void* X, const void* Y, cvgram_dtype dt, int64_t K, int64_t M,
                     const int32_t* perm, const double* pivot, const GramWork* work,
                     int64_t n_work, int tile, double* slabs, hipStream_t s) {
  if (n_work <= 0) return;
  if (dt == CVGRAM_F64)
    launch_typed<double>((const double*)X, (const double*)Y, K, M, perm, pivot, work, n_work,
                         tile, slabs, s);
  else
    launch_typed<float>((const float*)X, (const float*)Y, K, M, perm, pivot, work, n_work, tile,
                        slabs, s);
}

}  // namespace cvg
