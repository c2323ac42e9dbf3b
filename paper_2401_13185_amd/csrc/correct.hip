// Per-fold training products from the full and validation-block Grams.
//
// With Z' the pivot-shifted data (shift c per column), s'_T the shifted
// training column sums, mu' = s'_T / |T| and sigma the training deviations,
// an entry (i, j) of fold p is built from the shifted training Gram
//     g = G'[i][j] - G'_p[i][j]                     (Lemmas 2-3, Algorithm 7 step 9)
// as
//     raw      = g + c_i s'_j + s'_i c_j + |T| c_i c_j   (exact undo of the shift)
//     centred  = g - |T| (mu'_i mu'_j)                 (Propositions 7-8; outer
//                                                     product first, then |T|)
//     scaled   = (raw or centred) / (sigma_i sigma_j)   (Propositions 15-16, Table 1)
// A column constant over T_p has sigma = 1 and its centred row/column is
// exactly zero.  All arithmetic is FP64; the store rounds to the output type.
//
// Work decomposition: one workgroup per (32 x 32 output tile, fold).  X^T X
// tiles cover the upper triangle only; the lower triangle is written from
// the same values through an LDS transpose, so X^T X is bit-symmetric.
#include "internal.h"

namespace cvg {
namespace {

constexpr int TS = kCorrTile;  // 32
constexpr int kThreads = 256;
constexpr int kRowsPerThread = TS * TS / kThreads;  // 4

__global__ __launch_bounds__(256) void reduce_slabs_kernel(const double* __restrict__ slabs,
                                                           int64_t n_slabs, int64_t elems,
                                                           double* __restrict__ G) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= elems) return;
  double s = 0.0;
  for (int64_t k = 0; k < n_slabs; ++k) s += slabs[k * elems + e];
  G[e] = s;
}

template <typename OutT>
__device__ void correct_tile(const CorrectArgs& A, int32_t f);

// grid.x = tiles, grid.y strides over the folds (a grid dimension other than
// x is limited to 65535 blocks)
template <typename OutT>
__global__ __launch_bounds__(kThreads) void correct_kernel(CorrectArgs A, int32_t n_folds) {
  for (int32_t f = blockIdx.y; f < n_folds; f += gridDim.y) {
    correct_tile<OutT>(A, f);
    __syncthreads();
  }
}

template <typename OutT>
__device__ void correct_tile(const CorrectArgs& A, int32_t f) {
  const int32_t p = A.p_begin + f;
  __shared__ double T[TS][TS + 1];
  __shared__ double rc[TS], ra[TS], rmu[TS], rsd[TS];
  __shared__ double cc[TS], ca[TS], cmu[TS], csd[TS];
  __shared__ uint8_t rcs[TS], ccs[TS];

  const int tile = blockIdx.x;
  const bool is_xy = tile >= A.n_tiles_xx;
  const int bi = A.tiles[2 * tile];
  const int bj = A.tiles[2 * tile + 1];
  const bool diag = !is_xy && bi == bj;
  const int64_t K = A.K, M = A.M, W = A.W;
  const int64_t ncols = is_xy ? M : K;
  const int64_t coff = is_xy ? K : 0;  // column offset of the tile inside Z

  const int t = threadIdx.x;
  const int tx = t % TS, ty = t / TS;
  const int64_t pw = (int64_t)p * W;
  if (t < TS) {
    const int64_t i = (int64_t)bi * TS + t;
    if (i < K) {
      rc[t] = A.pivot[i];
      ra[t] = A.tr_sum[pw + i];
      rmu[t] = A.tr_mean[pw + i];
      rsd[t] = A.tr_std[pw + i];
      rcs[t] = A.tr_const[pw + i];
    }
  } else if (t < 2 * TS) {
    const int u = t - TS;
    const int64_t j = (int64_t)bj * TS + u;
    if (j < ncols) {
      const int64_t z = coff + j;
      cc[u] = A.pivot[z];
      ca[u] = A.tr_sum[pw + z];
      cmu[u] = A.tr_mean[pw + z];
      csd[u] = A.tr_std[pw + z];
      ccs[u] = A.tr_const[pw + z];
    }
  }
  __syncthreads();

  const double NT = (double)A.ntrain[p];
  const int32_t sb = A.slab_begin[p], se = A.slab_begin[p + 1];
  const int64_t slab_elems = K * W;

  double raw[kRowsPerThread], cen[kRowsPerThread];
  bool ok[kRowsPerThread];
#pragma unroll
  for (int r = 0; r < kRowsPerThread; ++r) {
    const int il = ty + 8 * r, jl = tx;
    const int64_t i = (int64_t)bi * TS + il;
    const int64_t j = (int64_t)bj * TS + jl;
    ok[r] = i < K && j < ncols && (!diag || il <= jl);
    raw[r] = 0.0;
    cen[r] = 0.0;
    if (!ok[r]) continue;
    const int64_t e = i * W + coff + j;
    double gp = 0.0;
    for (int32_t s = sb; s < se; ++s) gp += A.slabs[(int64_t)s * slab_elems + e];
    const double g = A.G[e] - gp;
    raw[r] = g + (rc[il] * ca[jl] + ra[il] * cc[jl]) + NT * (rc[il] * cc[jl]);
    cen[r] = (rcs[il] || ccs[jl]) ? 0.0 : g - NT * (rmu[il] * cmu[jl]);
  }

  if (!is_xy) {
    for (int c = 0; c < CVGRAM_XTX_CLASSES; ++c) {
      OutT* out = (OutT*)A.out_xx[c];
      if (!out) continue;
      out += (int64_t)f * A.fold_stride_xx;
      const bool centred = c & 2, scaled = c & 1;
      double v[kRowsPerThread];
#pragma unroll
      for (int r = 0; r < kRowsPerThread; ++r) {
        const int il = ty + 8 * r, jl = tx;
        v[r] = centred ? cen[r] : raw[r];
        if (scaled && ok[r]) v[r] = v[r] / (rsd[il] * csd[jl]);
        if (ok[r]) T[il][jl] = v[r];
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < kRowsPerThread; ++r) {
        const int il = ty + 8 * r, jl = tx;
        const int64_t i = (int64_t)bi * TS + il;
        const int64_t j = (int64_t)bj * TS + jl;
        if (diag) {
          if (i < K && j < K) out[i * K + j] = (OutT)(il <= jl ? T[il][jl] : T[jl][il]);
        } else {
          if (ok[r]) out[i * K + j] = (OutT)v[r];
          // transposed block: rows of bj, columns of bi
          const int64_t ti = (int64_t)bj * TS + il;
          const int64_t tj = (int64_t)bi * TS + jl;
          if (ti < K && tj < K) out[ti * K + tj] = (OutT)T[jl][il];
        }
      }
      __syncthreads();
    }
  } else {
    for (int c = 0; c < CVGRAM_XTY_CLASSES; ++c) {
      OutT* out = (OutT*)A.out_xy[c];
      if (!out) continue;
      out += (int64_t)f * A.fold_stride_xy;
      const bool centred = c & 4, scx = c & 2, scy = c & 1;
#pragma unroll
      for (int r = 0; r < kRowsPerThread; ++r) {
        if (!ok[r]) continue;
        const int il = ty + 8 * r, jl = tx;
        double v = centred ? cen[r] : raw[r];
        if (scx || scy) v = v / ((scx ? rsd[il] : 1.0) * (scy ? csd[jl] : 1.0));
        const int64_t i = (int64_t)bi * TS + il;
        const int64_t j = (int64_t)bj * TS + jl;
        out[i * M + j] = (OutT)v;
      }
    }
  }
}

}  // namespace

void launch_reduce_slabs(const double* slabs, int64_t n_slabs, int64_t elems, double* G,
                         hipStream_t s) {
  reduce_slabs_kernel<<<(unsigned)((elems + 255) / 256), 256, 0, s>>>(slabs, n_slabs, elems, G);
  CVG_LAUNCH_CHECK();
}

void launch_correct(const CorrectArgs& a, int32_t n_folds, bool out_f64, hipStream_t s) {
  const int32_t tiles = a.n_tiles_xx + a.n_tiles_xy;
  if (tiles <= 0 || n_folds <= 0) return;
  dim3 grid((unsigned)tiles, (unsigned)(n_folds < 65535 ? n_folds : 65535));
  if (out_f64)
    correct_kernel<double><<<grid, kThreads, 0, s>>>(a, n_folds);
  else
    correct_kernel<float><<<grid, kThreads, 0, s>>>(a, n_folds);
  CVG_LAUNCH_CHECK();
}

}  // namespace cvg
