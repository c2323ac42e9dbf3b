// One pass over the data: gather the rows of every fold through the fold
// permutation, shift every column by its pivot, and write
//   (1) the packed operand panels of the grouped Gram launch, and
//   (2) per row-chunk FP64 partial column sums, sums of squares, minima and
//       maxima of the validation block the chunk belongs to
//       (Algorithm 7 steps 10, 17, 19).
//
// Packed row space: folds follow each other in label order, each padded with
// zero rows to a multiple of kPanelRows, so every Gram work item streams a
// contiguous, aligned block of rows with no bounds checks.  Packed column
// space (width Wp): X columns [0, K), zeros up to Kp, Y columns [Kp, Kp + M),
// zeros up to Wp.  Element formats:
//   FP64 mode   double, row-major  Zp[row * Wp + col]
//   FP32 mode   float,  row-major  Zp[row * Wp + col]
//   BF16X3 mode two bf16 panels (hi, lo), k-contiguous in blocks of 32 rows:
//               Zp[((row / 32) * Wp + col) * 32 + row % 32]
// The split is hi = bf16(z'), lo = bf16(z' - hi) with z' = fp32(z - c).
#include <cmath>

#include "internal.h"

namespace cvg {
namespace {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

template <typename T>
__global__ __launch_bounds__(256) void pivot_kernel(const T* __restrict__ X,
                                                    const T* __restrict__ Y, int64_t rows,
                                                    int64_t K, int64_t M, int round_f32,
                                                    double* __restrict__ pivot) {
  // one workgroup per column block; each wave sums a strided subset of rows
  __shared__ double part[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t j = (int64_t)blockIdx.x * 64 + lane;
  double s = 0.0;
  if (j < K + M)
    for (int64_t r = w; r < rows; r += 4)
      s += j < K ? (double)X[r * K + j] : (double)Y[r * M + (j - K)];
  part[w][lane] = s;
  __syncthreads();
  if (w == 0 && j < K + M) {
    double c = ((part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane])) / (double)rows;
    if (round_f32) c = (double)(float)c;
    pivot[j] = c;
  }
}

// source column of packed column jp (or -1 for padding) and its stats index
__device__ inline int64_t src_col(int64_t jp, int64_t K, int64_t Kp, int64_t M) {
  if (jp < K) return jp;
  if (jp >= Kp && jp - Kp < M) return K + (jp - Kp);
  return -1;
}

template <typename T>
__device__ inline double zval(const T* __restrict__ X, const T* __restrict__ Y, int64_t K,
                              int64_t M, int64_t row, int64_t j) {
  return j < K ? (double)X[row * K + j] : (double)Y[row * M + (j - K)];
}

// grid.x = chunks, grid.y = blocks of 256 packed columns.  A chunk covers a
// whole number of 32-row panels of one fold.
// part layout: [4][n_chunks][W] (sum, sumsq, min, max of the real rows)
template <typename T, int MODE>
__global__ __launch_bounds__(256) void pack_kernel(
    const T* __restrict__ X, const T* __restrict__ Y, int64_t K, int64_t M, int64_t Kp,
    int64_t Wp, const int32_t* __restrict__ perm, const PackChunk* __restrict__ chunks,
    int64_t n_chunks, const double* __restrict__ pivot, void* __restrict__ packed,
    void* __restrict__ packed_lo, double* __restrict__ part) {
  const int64_t W = K + M;
  const int64_t jp = (int64_t)blockIdx.y * 256 + threadIdx.x;
  const int64_t c = blockIdx.x;
  if (jp >= Wp) return;
  const PackChunk ch = chunks[c];
  const int64_t js = src_col(jp, K, Kp, M);
  const double piv = js >= 0 ? pivot[js] : 0.0;
  const float pivf = (float)piv;  // the pivot is FP32-representable in the mixed modes
  double s = 0.0, q = 0.0, mn = INFINITY, mx = -INFINITY;

  for (int64_t d0 = ch.d0; d0 < ch.d1; d0 += kPanelRows) {
    double x[kPanelRows];
    bool v[kPanelRows];
#pragma unroll
    for (int u = 0; u < kPanelRows; ++u) {
      const int64_t src = ch.src0 + (d0 - ch.d0) + u;
      v[u] = js >= 0 && src < ch.src1;
      x[u] = v[u] ? zval(X, Y, K, M, (int64_t)perm[src], js) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kPanelRows; ++u) {
      if (!v[u]) continue;
      const double d = x[u] - piv;
      s += d;
      q = fma(d, d, q);
      mn = fmin(mn, x[u]);
      mx = fmax(mx, x[u]);
    }
    if constexpr (MODE == CVGRAM_MODE_BF16X3) {
      __bf16* hi = (__bf16*)packed;
      __bf16* lo = (__bf16*)packed_lo;
      bf16x8_t vh[kPanelRows / 8], vl[kPanelRows / 8];
#pragma unroll
      for (int u = 0; u < kPanelRows; ++u) {
        // z' = fp32(z - c): exact FP32 subtraction for FP32 input
        const float zf = !v[u] ? 0.f
                         : (sizeof(T) == 4 ? (float)x[u] - pivf : (float)(x[u] - (double)pivf));
        const __bf16 h = (__bf16)zf;
        vh[u / 8][u % 8] = h;
        vl[u / 8][u % 8] = (__bf16)(zf - (float)h);
      }
      const int64_t base = ((d0 / kPanelRows) * Wp + jp) * kPanelRows;
#pragma unroll
      for (int g = 0; g < kPanelRows / 8; ++g) {
        *(bf16x8_t*)&hi[base + g * 8] = vh[g];
        *(bf16x8_t*)&lo[base + g * 8] = vl[g];
      }
    } else if constexpr (MODE == CVGRAM_MODE_FP32) {
      float* out = (float*)packed;
#pragma unroll
      for (int u = 0; u < kPanelRows; ++u)
        out[(d0 + u) * Wp + jp] = !v[u] ? 0.f
                                  : (sizeof(T) == 4 ? (float)x[u] - pivf
                                                    : (float)(x[u] - (double)pivf));
    } else {
      double* out = (double*)packed;
#pragma unroll
      for (int u = 0; u < kPanelRows; ++u) out[(d0 + u) * Wp + jp] = v[u] ? x[u] - piv : 0.0;
    }
  }
  if (js >= 0) {
    const int64_t stride = n_chunks * W;
    part[0 * stride + c * W + js] = s;
    part[1 * stride + c * W + js] = q;
    part[2 * stride + c * W + js] = mn;
    part[3 * stride + c * W + js] = mx;
  }
}

template <typename T>
void launch_pack_typed(cvgram_mode mode, const T* X, const T* Y, int64_t K, int64_t M,
                       int64_t Kp, int64_t Wp, const int32_t* perm, const PackChunk* chunks,
                       int64_t n_chunks, const double* pivot, void* packed, void* packed_lo,
                       double* part, hipStream_t s) {
  dim3 grid((unsigned)n_chunks, (unsigned)((Wp + 255) / 256));
  if (mode == CVGRAM_MODE_FP64)
    pack_kernel<T, CVGRAM_MODE_FP64><<<grid, 256, 0, s>>>(X, Y, K, M, Kp, Wp, perm, chunks,
                                                          n_chunks, pivot, packed, packed_lo,
                                                          part);
  else if (mode == CVGRAM_MODE_FP32)
    pack_kernel<T, CVGRAM_MODE_FP32><<<grid, 256, 0, s>>>(X, Y, K, M, Kp, Wp, perm, chunks,
                                                          n_chunks, pivot, packed, packed_lo,
                                                          part);
  else
    pack_kernel<T, CVGRAM_MODE_BF16X3><<<grid, 256, 0, s>>>(X, Y, K, M, Kp, Wp, perm, chunks,
                                                            n_chunks, pivot, packed, packed_lo,
                                                            part);
  CVG_LAUNCH_CHECK();
}

}  // namespace

void launch_pivot(const void* X, const void* Y, cvgram_dtype dt, bool round_f32, int64_t N,
                  int64_t K, int64_t M, double* pivot, hipStream_t s) {
  const int64_t rows = N < 256 ? N : 256;
  const unsigned blocks = (unsigned)((K + M + 63) / 64);
  if (dt == CVGRAM_F64)
    pivot_kernel<double><<<blocks, 256, 0, s>>>((const double*)X, (const double*)Y, rows, K, M,
                                                round_f32 ? 1 : 0, pivot);
  else
    pivot_kernel<float><<<blocks, 256, 0, s>>>((const float*)X, (const float*)Y, rows, K, M,
                                               round_f32 ? 1 : 0, pivot);
  CVG_LAUNCH_CHECK();
}

void launch_pack(cvgram_mode mode, const void* X, const void* Y, cvgram_dtype dt, int64_t K,
                 int64_t M, int64_t Kp, int64_t Wp, const int32_t* perm, const PackChunk* chunks,
                 int64_t n_chunks, const double* pivot, void* packed, void* packed_lo,
                 double* part, hipStream_t s) {
  if (n_chunks <= 0) return;
  if (dt == CVGRAM_F64)
    launch_pack_typed<double>(mode, (const double*)X, (const double*)Y, K, M, Kp, Wp, perm,
                              chunks, n_chunks, pivot, packed, packed_lo, part, s);
  else
    launch_pack_typed<float>(mode, (const float*)X, (const float*)Y, K, M, Kp, Wp, perm, chunks,
                             n_chunks, pivot, packed, packed_lo, part, s);
}

}  // namespace cvg
