// Grouped validation-block Gram products in mixed precision on the matrix
// cores.  Same work list, tiles, slabs and fold grouping as the FP64 kernel
// (Algorithm 7 step 8 for all folds in one launch); only the arithmetic of
// the contraction differs:
//
//  * CVGRAM_MODE_FP32: z' = fp32(z - c) staged in LDS, v_mfma_f32_16x16x4_f32.
//  * CVGRAM_MODE_BF16X3: z' = fp32(z - c) split as hi = bf16(z'),
//    lo = bf16(z' - hi) (z' - hi is exact in FP32); each product is
//    hi*hi + hi*lo + lo*hi on v_mfma_f32_16x16x32_bf16 (the dropped lo*lo
//    term and the split remainder are about 2^-17 of the product).  The
//    pivot shift keeps |z'| near the column spread, so the split spends its
//    16 bits on the information that survives centering.
//
// In both modes the MFMA accumulates in FP32 over at most kFlushRows rows;
// the FP32 tile is then added into an FP64 register tile and cleared, so
// the FP32 rounding error does not grow with the fold size.  The FP64 tile
// is written to the item's slab as in the FP64 path.
#include "internal.h"

namespace cvg {
namespace {

typedef float float4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

constexpr int kThreads = 256;  // 4 waves, 2 x 2
constexpr int BM = 128;        // square output tile
constexpr int WT = BM / 2;     // wave tile
constexpr int NB = WT / 16;    // 16 x 16 MFMA blocks per wave edge
constexpr int kFlushRows = 256;

template <typename T>
__device__ inline float zload32(const T* __restrict__ X, const T* __restrict__ Y, int64_t K,
                                int64_t M, int64_t row, int64_t j, float piv) {
  // shift in the input precision's widest common type, then round to FP32
  if (j < K) return (float)((double)X[row * K + j] - (double)piv);
  return (float)((double)Y[row * M + (j - K)] - (double)piv);
}

template <>
__device__ inline float zload32<float>(const float* __restrict__ X, const float* __restrict__ Y,
                                       int64_t K, int64_t M, int64_t row, int64_t j, float piv) {
  return (j < K ? X[row * K + j] : Y[row * M + (j - K)]) - piv;
}

// ---------------------------------------------------------------------------
// FP32 MFMA variant
// ---------------------------------------------------------------------------
template <typename TIn>
__global__ __launch_bounds__(kThreads) void gram_f32_kernel(
    const TIn* __restrict__ X, const TIn* __restrict__ Y, int64_t K, int64_t M,
    const int32_t* __restrict__ perm, const double* __restrict__ pivot,
    const GramWork* __restrict__ work, int64_t n_work, double* __restrict__ slabs) {
  constexpr int BK = 16;
  constexpr int TPR = kThreads / BK;  // 16 loader threads per row
  constexpr int CPT = BM / TPR;       // 8 columns each
  constexpr int LD = BM + 4;
  __shared__ float As[BK * LD];
  __shared__ float Bs[BK * LD];

  const int64_t per = (int64_t)gridDim.x / 8;
  const int64_t item = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (item >= n_work) return;
  const GramWork w = work[item];
  const int64_t W = K + M;
  const int64_t i0 = (int64_t)w.ti * BM, j0 = (int64_t)w.tj * BM;
  const bool diag = w.ti == w.tj;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const bool active = !(diag && wm > wn);

  const int lk = t / TPR, lc = (t % TPR) * CPT;
  float pa[CPT], pb[CPT];
  bool va[CPT], vb[CPT];
#pragma unroll
  for (int u = 0; u < CPT; ++u) {
    const int64_t gi = i0 + lc + u, gj = j0 + lc + u;
    va[u] = gi < K;
    vb[u] = gj < W;
    pa[u] = va[u] ? (float)pivot[gi] : 0.f;
    pb[u] = vb[u] ? (float)pivot[gj] : 0.f;
  }
  float ra[CPT], rb[CPT];
  auto load_stage = [&](int64_t r) {
    const int64_t rr = r + lk;
    const bool vr = rr < w.r1;
    const int64_t n = vr ? (int64_t)perm[rr] : 0;
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
      ra[u] = (vr && va[u]) ? zload32(X, Y, K, M, n, i0 + lc + u, pa[u]) : 0.f;
      rb[u] = (vr && vb[u]) ? zload32(X, Y, K, M, n, j0 + lc + u, pb[u]) : 0.f;
    }
  };
  auto store_stage = [&]() {
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
      As[lk * LD + lc + u] = ra[u];
      Bs[lk * LD + lc + u] = rb[u];
    }
  };

  float4_t acc[NB][NB];
  double a64[NB][NB][4];
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      acc[a][b] = float4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int e = 0; e < 4; ++e) a64[a][b][e] = 0.0;
    }
  auto flush = [&]() {
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b) {
#pragma unroll
        for (int e = 0; e < 4; ++e) a64[a][b][e] += (double)acc[a][b][e];
        acc[a][b] = float4_t{0.f, 0.f, 0.f, 0.f};
      }
  };

  const int fr = lane >> 4, fc = lane & 15;
  load_stage(w.r0);
  store_stage();
  __syncthreads();
  int since = 0;
  for (int64_t r = w.r0; r < w.r1; r += BK) {
    const bool has_next = r + BK < w.r1;
    if (has_next) load_stage(r + BK);
    if (active) {
#pragma unroll
      for (int kk = 0; kk < BK / 4; ++kk) {
        float af[NB], bf[NB];
#pragma unroll
        for (int a = 0; a < NB; ++a) af[a] = As[(kk * 4 + fr) * LD + wm * WT + a * 16 + fc];
#pragma unroll
        for (int b = 0; b < NB; ++b) bf[b] = Bs[(kk * 4 + fr) * LD + wn * WT + b * 16 + fc];
#pragma unroll
        for (int a = 0; a < NB; ++a)
#pragma unroll
          for (int b = 0; b < NB; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[a], bf[b], acc[a][b], 0, 0, 0);
      }
      since += BK;
      if (since >= kFlushRows) {
        flush();
        since = 0;
      }
    }
    __syncthreads();
    if (has_next) {
      store_stage();
      __syncthreads();
    }
  }
  if (!active) return;
  flush();
  double* out = slabs + (int64_t)w.slab * K * W;
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        // FP32 16 x 16 MFMA results: element e of lane l is row 4 (l / 16) + e
        const int64_t row = i0 + wm * WT + a * 16 + fr * 4 + e;
        const int64_t col = j0 + wn * WT + b * 16 + fc;
        if (row < K && col < W) out[row * W + col] = a64[a][b][e];
      }
}

// ---------------------------------------------------------------------------
// split-bf16 variant (three bf16 products per FP32 product)
// ---------------------------------------------------------------------------
__device__ inline void split_bf16(float x, __bf16& hi, __bf16& lo) {
  hi = (__bf16)x;                 // round to nearest even
  lo = (__bf16)(x - (float)hi);   // x - hi is exact in FP32
}

template <typename TIn>
__global__ __launch_bounds__(kThreads) void gram_bf16x3_kernel(
    const TIn* __restrict__ X, const TIn* __restrict__ Y, int64_t K, int64_t M,
    const int32_t* __restrict__ perm, const double* __restrict__ pivot,
    const GramWork* __restrict__ work, int64_t n_work, double* __restrict__ slabs) {
  constexpr int BK = 32;            // rows per stage = one MFMA k-step
  constexpr int RPT = BK / 2;       // rows per loader thread (2 threads per column)
  constexpr int LDK = BK + 8;       // bf16 elements per column in LDS (80 bytes)
  // k-contiguous layout: [column][k]
  __shared__ __attribute__((aligned(16))) __bf16 Ahi[BM * LDK];
  __shared__ __attribute__((aligned(16))) __bf16 Alo[BM * LDK];
  __shared__ __attribute__((aligned(16))) __bf16 Bhi[BM * LDK];
  __shared__ __attribute__((aligned(16))) __bf16 Blo[BM * LDK];

  const int64_t per = (int64_t)gridDim.x / 8;
  const int64_t item = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  if (item >= n_work) return;
  const GramWork w = work[item];
  const int64_t W = K + M;
  const int64_t i0 = (int64_t)w.ti * BM, j0 = (int64_t)w.tj * BM;
  const bool diag = w.ti == w.tj;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const bool active = !(diag && wm > wn);

  // A diagonal tile whose columns all lie inside X has B == A: load it once.
  // (A diagonal tile that crosses column K also holds Y columns in B.)
  const bool same = diag && j0 + BM <= K;

  // loader: one column, RPT consecutive rows of the stage
  const int lcol = t % BM;
  const int lrow = (t / BM) * RPT;
  const int64_t gi = i0 + lcol, gj = j0 + lcol;
  const bool va = gi < K, vb = gj < W;
  const float pa = va ? (float)pivot[gi] : 0.f;
  const float pb = vb ? (float)pivot[gj] : 0.f;

  float ra[RPT], rb[RPT];
  auto load_stage = [&](int64_t r) {
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
      const int64_t rr = r + lrow + u;
      const bool vr = rr < w.r1;
      const int64_t n = vr ? (int64_t)perm[rr] : 0;
      ra[u] = (vr && va) ? zload32(X, Y, K, M, n, gi, pa) : 0.f;
      rb[u] = (vr && vb && !same) ? zload32(X, Y, K, M, n, gj, pb) : 0.f;
    }
  };
  auto store_stage = [&]() {
#pragma unroll
    for (int h = 0; h < RPT / 8; ++h) {
      bf16x8_t xh, xl, yh, yl;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        __bf16 a, b;
        split_bf16(ra[h * 8 + e], a, b);
        xh[e] = a;
        xl[e] = b;
        split_bf16(rb[h * 8 + e], a, b);
        yh[e] = a;
        yl[e] = b;
      }
      const int off = lcol * LDK + lrow + h * 8;
      *(bf16x8_t*)&Ahi[off] = xh;
      *(bf16x8_t*)&Alo[off] = xl;
      if (!same) {
        *(bf16x8_t*)&Bhi[off] = yh;
        *(bf16x8_t*)&Blo[off] = yl;
      }
    }
  };
  const __bf16* Bh = same ? Ahi : Bhi;
  const __bf16* Bl = same ? Alo : Blo;

  float4_t acc[NB][NB];
  double a64[NB][NB][4];
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      acc[a][b] = float4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int e = 0; e < 4; ++e) a64[a][b][e] = 0.0;
    }
  auto flush = [&]() {
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b) {
#pragma unroll
        for (int e = 0; e < 4; ++e) a64[a][b][e] += (double)acc[a][b][e];
        acc[a][b] = float4_t{0.f, 0.f, 0.f, 0.f};
      }
  };

  const int fr = lane >> 4, fc = lane & 15;
  load_stage(w.r0);
  store_stage();
  __syncthreads();
  int since = 0;
  for (int64_t r = w.r0; r < w.r1; r += BK) {
    const bool has_next = r + BK < w.r1;
    if (has_next) load_stage(r + BK);
    if (active) {
      bf16x8_t ah[NB], al[NB];
#pragma unroll
      for (int a = 0; a < NB; ++a) {
        const int off = (wm * WT + a * 16 + fc) * LDK + fr * 8;
        ah[a] = *(const bf16x8_t*)&Ahi[off];
        al[a] = *(const bf16x8_t*)&Alo[off];
      }
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int off = (wn * WT + b * 16 + fc) * LDK + fr * 8;
        const bf16x8_t bh = *(const bf16x8_t*)&Bh[off];
        const bf16x8_t bl = *(const bf16x8_t*)&Bl[off];
#pragma unroll
        for (int a = 0; a < NB; ++a) {
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[a], bh, acc[a][b], 0, 0, 0);
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bl, acc[a][b], 0, 0, 0);
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[a], bh, acc[a][b], 0, 0, 0);
        }
      }
      since += BK;
      if (since >= kFlushRows) {
        flush();
        since = 0;
      }
    }
    __syncthreads();
    if (has_next) {
      store_stage();
      __syncthreads();
    }
  }
  if (!active) return;
  flush();
  double* out = slabs + (int64_t)w.slab * K * W;
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t row = i0 + wm * WT + a * 16 + fr * 4 + e;
        const int64_t col = j0 + wn * WT + b * 16 + fc;
        if (row < K && col < W) out[row * W + col] = a64[a][b][e];
      }
}

template <typename TIn>
void launch_typed(cvgram_mode mode, const TIn* X, const TIn* Y, int64_t K, int64_t M,
                  const int32_t* perm, const double* pivot, const GramWork* work, int64_t n_work,
                  double* slabs, hipStream_t s) {
  const unsigned grid = (unsigned)(8 * ((n_work + 7) / 8));
  if (mode == CVGRAM_MODE_FP32)
    gram_f32_kernel<TIn><<<grid, kThreads, 0, s>>>(X, Y, K, M, perm, pivot, work, n_work, slabs);
  else
    gram_bf16x3_kernel<TIn><<<grid, kThreads, 0, s>>>(X, Y, K, M, perm, pivot, work, n_work,
                                                      slabs);
  CVG_LAUNCH_CHECK();
}

}  // namespace

int mixed_tile() { return BM; }

void launch_gram_mixed(cvgram_mode mode, const void* X, const void* Y, cvgram_dtype dt, int64_t K,
                       int64_t M, const int32_t* perm, const double* pivot, const GramWork* work,
                       int64_t n_work, double* slabs, hipStream_t s) {
  if (n_work <= 0) return;
  if (dt == CVGRAM_F64)
    launch_typed<double>(mode, (const double*)X, (const double*)Y, K, M, perm, pivot, work,
                         n_work, slabs, s);
  else
    launch_typed<float>(mode, (const float*)X, (const float*)Y, K, M, perm, pivot, work, n_work,
                        slabs, s);
}

}  // namespace cvg
