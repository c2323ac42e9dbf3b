// One pass over the data: gather the rows of every fold through the fold
// permutation, shift every column by its pivot, and write
//   (1) the packed operand panels of the grouped Gram launch, and
//   (2) per row-chunk FP64 partial column sums, sums of squares, minima and
//       maxima of the validation block the chunk belongs to
//       (Algorithm 7 steps 10, 17, 19).
//
// Element formats of the packed panels (see ProbDesc for the row/column
// spaces):
//   FP64 mode   double, row-major  Zp[row * Wp + col]
//   FP32 mode   float,  row-major  Zp[row * Wp + col]
//   BF16X3 mode two bf16 panels (hi, lo), k-contiguous in blocks of 32 rows:
//               Zp[((row / 32) * Wp + col) * 32 + row % 32]
// with z' = z - c in FP64 (FP64 mode) or fp32(z - c) (mixed modes), and the
// split hi = bf16(z'), lo = bf16(z' - hi).
//
// Work shape: a one-wave workgroup handles one chunk (whole 32-row panels
// of one fold) x kPackCols = 64 packed columns, so that narrow problems
// (K + M of a few dozen) and the Y columns at the end of a row keep almost
// every lane busy.  Lane l loads columns 4 (l % 16) .. + 3 of rows
// 8 (l / 16) .. + 7 of each panel (16-byte loads when the columns allow it:
// eight rows x one or two loads in flight per lane); the bf16 panels are
// transposed through LDS so that every global store is a contiguous 16-byte
// chunk of a fully written line.
#include <cmath>
#include <type_traits>

#include "internal.h"

namespace cvg {
namespace {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float float4_t __attribute__((ext_vector_type(4)));
typedef double double2_t __attribute__((ext_vector_type(2)));

// pivot: c_j = FP64 mean of n = min(N, 256) rows of column j of [X | Y]
// spread evenly over the whole column (rows floor(r N / n), r = 0 .. n-1), so
// that rows ordered by a drifting or sorted covariate still give a pivot
// near the column's mean (rounded to FP32 in the mixed modes).  A
// 1024-thread workgroup covers 64 columns: wave w sums sample rows w,
// w + 16, ... (at most 16, every load in flight at once), and the 16 wave
// sums are combined in a fixed order.
constexpr int kPivotThreads = 1024;
constexpr int kPivotWaves = kPivotThreads / 64;

template <typename T>
__device__ inline void pivot_cols(const CVG_GLOBAL T* X, const CVG_GLOBAL T* Y, int64_t N,
                                  int64_t K, int64_t M, int64_t col_block, int round_f32,
                                  CVG_GLOBAL double* out) {
  __shared__ double part[kPivotWaves][64];
  const int64_t rows = N < 256 ? N : 256;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t j = col_block * 64 + lane;
  double v[256 / kPivotWaves];
#pragma unroll
  for (int u = 0; u < 256 / kPivotWaves; ++u) v[u] = 0.0;
  if (j < K + M) {
    const CVG_GLOBAL T* base = j < K ? X + j : Y + (j - K);
    const int64_t ld = j < K ? K : M;
#pragma unroll
    for (int u = 0; u < 256 / kPivotWaves; ++u) {
      const int64_t r = w + (int64_t)kPivotWaves * u;
      if (r < rows) v[u] = (double)base[(r * N / rows) * ld];
    }
  }
#pragma unroll
  for (int h = 256 / kPivotWaves / 2; h > 0; h >>= 1)
#pragma unroll
    for (int u = 0; u < h; ++u) v[u] += v[u + h];
  part[w][lane] = v[0];
  __syncthreads();
  if (w == 0 && j < K + M) {
    double c = 0.0;
#pragma unroll
    for (int k = 0; k < kPivotWaves; ++k) c += part[k][lane];
    c /= (double)rows;
    if (round_f32) c = (double)(float)c;
    out[j] = c;
  }
}

// items: (prob, block of 64 columns)
template <typename T>
__global__ __launch_bounds__(kPivotThreads) void pivot_kernel(const ProbDesc* __restrict__ pds,
                                                              const Item* __restrict__ items,
                                                              int round_f32) {
  const Item it = items[blockIdx.x];
  const ProbDesc& pd = pds[it.prob];
  pivot_cols<T>(gmem((const T*)pd.X), gmem((const T*)pd.Y), pd.N, pd.K, pd.M, it.a, round_f32,
                gmem(pd.pivot));
}

// one problem, arguments by value (no descriptor yet): workgroup = block of 64 columns
template <typename T>
__global__ __launch_bounds__(kPivotThreads) void pivot_direct_kernel(const T* X, const T* Y,
                                                                     int64_t N, int64_t K,
                                                                     int64_t M, int round_f32,
                                                                     double* out) {
  pivot_cols<T>(gmem(X), gmem(Y), N, K, M, blockIdx.x, round_f32, gmem(out));
}

// source column (index into [X | Y], also the statistics index) of packed
// column jp, or -1 for a padding column
__device__ inline int64_t src_col(int64_t jp, int64_t K, int64_t Kp, int64_t M) {
  if (jp < K) return jp;
  if (jp >= Kp && jp - Kp < M) return K + (jp - Kp);
  return -1;
}

// four consecutive X columns of one row, 16-byte aligned
template <typename T>
__device__ inline void load_vec(const CVG_GLOBAL T* __restrict__ X, int64_t K, int64_t row,
                                int64_t col, double (&x)[4]) {
  if constexpr (sizeof(T) == 4) {
    const float4_t v = *(const CVG_GLOBAL float4_t*)&X[row * K + col];
    x[0] = v.x;
    x[1] = v.y;
    x[2] = v.z;
    x[3] = v.w;
  } else {
    const double2_t a = *(const CVG_GLOBAL double2_t*)&X[row * K + col];
    const double2_t b = *(const CVG_GLOBAL double2_t*)&X[row * K + col + 2];
    x[0] = a.x;
    x[1] = a.y;
    x[2] = b.x;
    x[3] = b.y;
  }
}

constexpr int LDK = kPanelRows + 8;  // bf16 per column in the LDS transpose (80 B)
constexpr int kPackThreads = kPackCols;    // one lane per 4 columns x 4 row groups
constexpr int kColGroups = kPackCols / 4;  // lanes per row group

template <typename T, int MODE>
__global__ __launch_bounds__(kPackThreads) void pack_kernel(const ProbDesc* __restrict__ pds,
                                                            const PackChunk* __restrict__ chunks,
                                                            int32_t ncb) {
  constexpr int kT = MODE == CVGRAM_MODE_BF16X3 ? kPackCols * LDK : 8;
  __shared__ __attribute__((aligned(16))) __bf16 th[kT];
  __shared__ __attribute__((aligned(16))) __bf16 tl[kT];
  __shared__ double red[kPackThreads * 4];

  // workgroup = (chunk, column block), column blocks fastest: the workgroups
  // reading one chunk's rows start together and take whole rows between
  // them (better DRAM page locality than column-block-major order)
  const int64_t chunk = (int64_t)blockIdx.x / ncb;
  const int32_t cbi = (int32_t)(blockIdx.x - chunk * ncb);
  const PackChunk ch = chunks[chunk];
  // descriptor fields in registers (the loops below store through other
  // pointers; no field is re-read from memory)
  const ProbDesc& pdr = pds[ch.prob];
  const int64_t Wp = pdr.Wp;
  const int64_t cb0 = (int64_t)cbi * kPackCols;
  if (cb0 >= Wp) return;  // uniform over the workgroup
  const CVG_GLOBAL T* __restrict__ X = gmem((const T*)pdr.X);
  const CVG_GLOBAL T* __restrict__ Y = gmem((const T*)pdr.Y);
  const CVG_GLOBAL int32_t* __restrict__ perm = gmem(pdr.perm);
  const CVG_GLOBAL double* __restrict__ pivot = gmem((const double*)pdr.pivot);
  void* const packed = pdr.packed;
  void* const packed_lo = pdr.packed_lo;
  CVG_GLOBAL double* const part = gmem(pdr.part);
  const int64_t n_chunks = pdr.n_chunks;
  const int x_vec = pdr.x_vec;
  const bool panel_f32 = pdr.panel_f32 != 0;
  const int64_t K = pdr.K, M = pdr.M, Kp = pdr.Kp, W = pdr.W;
  const int t = threadIdx.x, cg = t % kColGroups, rg = t / kColGroups;
  const int64_t jp0 = cb0 + 4 * cg;

  int64_t js[4];
  double piv[4];
  float pivf[4];
  bool any = false;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    js[u] = jp0 + u < Wp ? src_col(jp0 + u, K, Kp, M) : -1;
    piv[u] = js[u] >= 0 ? pivot[js[u]] : 0.0;
    pivf[u] = (float)piv[u];  // FP32-representable in the mixed modes
    any |= js[u] >= 0;
  }
  const bool vec = x_vec && jp0 + 3 < K;
  // per column: the source array and its row stride
  const CVG_GLOBAL T* src[4];
  int64_t ld[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    if (js[u] >= K) {
      src[u] = Y + (js[u] - K);
      ld[u] = M;
    } else {
      src[u] = X + (js[u] >= 0 ? js[u] : 0);
      ld[u] = K;
    }
  }
  double s[4] = {0, 0, 0, 0}, q[4] = {0, 0, 0, 0};
  double mn[4] = {INFINITY, INFINITY, INFINITY, INFINITY};
  double mx[4] = {-INFINITY, -INFINITY, -INFINITY, -INFINITY};

  // the chunk's permutation indices (source rows; -1 for padding rows),
  // staged in LDS once: the panel loop then waits on no global load but its
  // own data (loads and stores share one counter on this architecture)
  __shared__ int32_t prow[kMaxChunkRows];
  const int64_t nrows = ch.d1 - ch.d0;
  for (int64_t k = t; k < nrows; k += kPackThreads) {
    const int64_t src = ch.src0 + k;
    prow[k] = src < ch.src1 ? perm[src] : -1;
  }
  __syncthreads();
  // panel d0: this lane's 8 rows x 4 columns (zero for padding rows)
  auto load_panel = [&](auto fast_c, int64_t d0, double (&x)[8][4], bool (&v)[8]) {
    int32_t rows[8];
#pragma unroll
    for (int g = 0; g < 8; ++g) rows[g] = prow[d0 - ch.d0 + rg * 8 + g];
#pragma unroll
    for (int g = 0; g < 8; ++g) v[g] = any && rows[g] >= 0;
    if constexpr (decltype(fast_c)::value) {
      // all four columns are X columns: the eight rows' loads are issued
      // back to back with no branch between them (a padding row reads row 0
      // and is zeroed), so they are all in flight at once
#pragma unroll
      for (int g = 0; g < 8; ++g) load_vec(X, K, rows[g] >= 0 ? (int64_t)rows[g] : 0, js[0], x[g]);
#pragma unroll
      for (int g = 0; g < 8; ++g)
#pragma unroll
        for (int u = 0; u < 4; ++u) x[g][u] = v[g] ? x[g][u] : 0.0;
    } else {
      // a block reaching into Y or the padding, or unaligned X: each lane
      // reads its four columns from fixed sources (X, Y, or X column 0 for a
      // padding column), all eight rows' loads issued with no branch between
      // them (padding rows read row 0); what is not data is zeroed after
      if (vec) {
#pragma unroll
        for (int g = 0; g < 8; ++g) load_vec(X, K, rows[g] >= 0 ? (int64_t)rows[g] : 0, js[0], x[g]);
      } else {
#pragma unroll
        for (int g = 0; g < 8; ++g) {
          const int64_t r = rows[g] >= 0 ? (int64_t)rows[g] : 0;
#pragma unroll
          for (int u = 0; u < 4; ++u) x[g][u] = (double)src[u][r * ld[u]];
        }
      }
#pragma unroll
      for (int g = 0; g < 8; ++g)
#pragma unroll
        for (int u = 0; u < 4; ++u) x[g][u] = (v[g] && js[u] >= 0) ? x[g][u] : 0.0;
    }
  };
  // statistics and packed output of panel d0
  auto consume = [&](int64_t d0, const double (&x)[8][4], const bool (&v)[8]) {
#pragma unroll
    for (int g = 0; g < 8; ++g) {
      if (!v[g]) continue;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (js[u] < 0) continue;
        const double d = x[g][u] - piv[u];
        s[u] += d;
        q[u] = fma(d, d, q[u]);
        mn[u] = fmin(mn[u], x[g][u]);
        mx[u] = fmax(mx[u], x[g][u]);
      }
    }
    if constexpr (MODE == CVGRAM_MODE_BF16X3) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        bf16x8_t h, l;
#pragma unroll
        for (int g = 0; g < 8; ++g) {
          const bool ok = v[g] && js[u] >= 0;
          // z' = fp32(z - c): exact for FP32 input when c/2 <= z <= 2c
          // (Sterbenz), otherwise rounded once to FP32
          const float zf = !ok ? 0.f
                           : (sizeof(T) == 4 ? (float)x[g][u] - pivf[u]
                                             : (float)(x[g][u] - (double)pivf[u]));
          const __bf16 hh = (__bf16)zf;
          h[g] = hh;
          l[g] = (__bf16)(zf - (float)hh);
        }
        *(bf16x8_t*)&th[(4 * cg + u) * LDK + rg * 8] = h;
        *(bf16x8_t*)&tl[(4 * cg + u) * LDK + rg * 8] = l;
      }
      __syncthreads();
      CVG_GLOBAL __bf16* hi = gmem((__bf16*)packed);
      CVG_GLOBAL __bf16* lo = gmem((__bf16*)packed_lo);
      const int64_t base = ((d0 / kPanelRows) * Wp + cb0) * kPanelRows;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int qc = t + kPackThreads * k;  // 16-byte chunk: column qc / 4, rows 8 (qc % 4) ..
        if (cb0 + (qc >> 2) < Wp) {
          *(CVG_GLOBAL bf16x8_t*)&hi[base + qc * 8] =
              *(const bf16x8_t*)&th[(qc >> 2) * LDK + (qc & 3) * 8];
          *(CVG_GLOBAL bf16x8_t*)&lo[base + qc * 8] =
              *(const bf16x8_t*)&tl[(qc >> 2) * LDK + (qc & 3) * 8];
        }
      }
      __syncthreads();
    } else if constexpr (MODE == CVGRAM_MODE_FP32) {
      if (jp0 < Wp) {
        CVG_GLOBAL float* out = gmem((float*)packed);
#pragma unroll
        for (int g = 0; g < 8; ++g) {
          float4_t z;
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const bool ok = v[g] && js[u] >= 0;
            z[u] = !ok ? 0.f
                   : (sizeof(T) == 4 ? (float)x[g][u] - pivf[u]
                                     : (float)(x[g][u] - (double)pivf[u]));
          }
          *(CVG_GLOBAL float4_t*)&out[(d0 + rg * 8 + g) * Wp + jp0] = z;
        }
      }
    } else if (sizeof(T) == 4 && panel_f32) {
      // FP64 mode on FP32 panels (FP32 input, ProbDesc::panel_f32): the raw
      // FP32 values, shifted by the Gram launch as it loads them; a padding
      // row holds the column's pivot (an FP32 value in this mode) so that it
      // shifts to 0, a padding column 0
      if (jp0 < Wp) {
        CVG_GLOBAL float* out = gmem((float*)packed);
#pragma unroll
        for (int g = 0; g < 8; ++g) {
          float4_t z;
#pragma unroll
          for (int u = 0; u < 4; ++u) z[u] = js[u] < 0 ? 0.f : (v[g] ? (float)x[g][u] : pivf[u]);
          *(CVG_GLOBAL float4_t*)&out[(d0 + rg * 8 + g) * Wp + jp0] = z;
        }
      }
    } else {
      if (jp0 < Wp) {
        CVG_GLOBAL double* out = gmem((double*)packed);
#pragma unroll
        for (int g = 0; g < 8; ++g) {
          double2_t a, b;
          a.x = (v[g] && js[0] >= 0) ? x[g][0] - piv[0] : 0.0;
          a.y = (v[g] && js[1] >= 0) ? x[g][1] - piv[1] : 0.0;
          b.x = (v[g] && js[2] >= 0) ? x[g][2] - piv[2] : 0.0;
          b.y = (v[g] && js[3] >= 0) ? x[g][3] - piv[3] : 0.0;
          *(CVG_GLOBAL double2_t*)&out[(d0 + rg * 8 + g) * Wp + jp0] = a;
          *(CVG_GLOBAL double2_t*)&out[(d0 + rg * 8 + g) * Wp + jp0 + 2] = b;
        }
      }
    }
  };
  // two register sets, so the next panel's loads are issued before this
  // panel's stores and are not held up by them (loads and stores share one
  // wait counter)
  auto panels = [&](auto fast_c) {
    double xa[8][4], xb[8][4];
    bool va[8], vb[8];
    load_panel(fast_c, ch.d0, xa, va);
    for (int64_t d0 = ch.d0;; d0 += 2 * kPanelRows) {
      const int64_t n1 = d0 + kPanelRows;
      load_panel(fast_c, n1 < ch.d1 ? n1 : d0, xb, vb);
      consume(d0, xa, va);
      if (n1 >= ch.d1) break;
      const int64_t n2 = n1 + kPanelRows;
      load_panel(fast_c, n2 < ch.d1 ? n2 : n1, xa, va);
      consume(n1, xb, vb);
      if (n2 >= ch.d1) break;
    }
  };
  if (x_vec && cb0 + kPackCols <= K)
    panels(std::true_type{});  // a block of X columns only (16-byte loads)
  else
    panels(std::false_type{});  // reaches into Y or the padding, or unaligned X

  // combine the 4 row groups of each column, in row-group order
  const int64_t stride = n_chunks * W;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
#pragma unroll
    for (int u = 0; u < 4; ++u)
      red[t * 4 + u] = k == 0 ? s[u] : k == 1 ? q[u] : k == 2 ? mn[u] : mx[u];
    __syncthreads();
    if (rg == 0) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        double r = red[cg * 4 + u];
        for (int g = 1; g < 4; ++g) {
          const double o = red[(g * kColGroups + cg) * 4 + u];
          r = k < 2 ? r + o : (k == 2 ? fmin(r, o) : fmax(r, o));
        }
        if (js[u] >= 0) part[k * stride + (int64_t)ch.chunk * W + js[u]] = r;
      }
    }
    __syncthreads();
  }
}

template <typename T>
void launch_pack_typed(cvgram_mode mode, const ProbDesc* pd, const PackChunk* chunks,
                       int64_t n_chunks, int32_t max_col_blocks, hipStream_t s) {
  const int64_t blocks = n_chunks * max_col_blocks;
  if (blocks > INT32_MAX) {
    set_error("pack: too many chunks for one launch");
    throw Fail{CVGRAM_EINVAL};
  }
  const unsigned grid = (unsigned)blocks;
  const int32_t ncb = max_col_blocks;
  if (mode == CVGRAM_MODE_FP64)
    pack_kernel<T, CVGRAM_MODE_FP64><<<grid, kPackThreads, 0, s>>>(pd, chunks, ncb);
  else if (mode == CVGRAM_MODE_FP32)
    pack_kernel<T, CVGRAM_MODE_FP32><<<grid, kPackThreads, 0, s>>>(pd, chunks, ncb);
  else
    pack_kernel<T, CVGRAM_MODE_BF16X3><<<grid, kPackThreads, 0, s>>>(pd, chunks, ncb);
  CVG_LAUNCH_CHECK();
}

}  // namespace

void launch_pivot(cvgram_dtype dt, bool round_f32, const ProbDesc* pd, const Item* items,
                  int64_t n_items, hipStream_t s) {
  if (n_items <= 0) return;
  if (dt == CVGRAM_F64)
    pivot_kernel<double><<<(unsigned)n_items, kPivotThreads, 0, s>>>(pd, items,
                                                                     round_f32 ? 1 : 0);
  else
    pivot_kernel<float><<<(unsigned)n_items, kPivotThreads, 0, s>>>(pd, items,
                                                                    round_f32 ? 1 : 0);
  CVG_LAUNCH_CHECK();
}

void launch_pivot_direct(cvgram_dtype dt, bool round_f32, const void* X, const void* Y,
                         int64_t N, int64_t K, int64_t M, double* out, hipStream_t s) {
  const unsigned blocks = (unsigned)((K + M + 63) / 64);
  if (dt == CVGRAM_F64)
    pivot_direct_kernel<double><<<blocks, kPivotThreads, 0, s>>>(
        (const double*)X, (const double*)Y, N, K, M, round_f32 ? 1 : 0, out);
  else
    pivot_direct_kernel<float><<<blocks, kPivotThreads, 0, s>>>(
        (const float*)X, (const float*)Y, N, K, M, round_f32 ? 1 : 0, out);
  CVG_LAUNCH_CHECK();
}

void launch_pack(cvgram_mode mode, cvgram_dtype dt, const ProbDesc* pd, const PackChunk* chunks,
                 int64_t n_chunks, int32_t max_col_blocks, hipStream_t s) {
  if (n_chunks <= 0) return;
  if (dt == CVGRAM_F64)
    launch_pack_typed<double>(mode, pd, chunks, n_chunks, max_col_blocks, s);
  else
    launch_pack_typed<float>(mode, pd, chunks, n_chunks, max_col_blocks, s);
}

}  // namespace cvg
