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
#include <type_traits>

#include "internal.h"

namespace cvg {
namespace {

constexpr int TS = kCorrTile;  // 32

// workgroup barrier for LDS reuse only: waits for this wave's LDS accesses,
// not for its global stores (__syncthreads' fence would wait for those too)
__device__ __forceinline__ void lds_barrier() {
  // s_waitcnt fields: vmcnt 63 and expcnt 7 (no wait), lgkmcnt 0
  __builtin_amdgcn_s_waitcnt(0xc07f);
  asm volatile("s_barrier" ::: "memory");
}
constexpr int kThreads = 256;
constexpr int kRowsPerThread = TS * TS / kThreads;  // 4

// For every fold p, G'_p = sum of the fold's slabs (its row splits), written
// into the fold's first slab; G' = sum over folds in fold order.  Entries
// below the diagonal of the K x K block are never read (mirror image) and
// are skipped.  Fixed summation order: deterministic.
// items: (prob, block of kReduceElems entries of the K x W slab); each thread
// sums two neighbouring entries, with one 16-byte load per slab when the
// slab stride keeps the pair aligned (K W even).
typedef double double2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void load_pair(const CVG_GLOBAL double* p, bool vec, bool second,
                                          double& a, double& b) {
  if (vec) {
    const double2_t v = *(const CVG_GLOBAL double2_t*)p;
    a = v.x;
    b = v.y;
  } else {
    a = p[0];
    b = second ? p[1] : 0.0;
  }
}
__global__ __launch_bounds__(256) void reduce_slabs_kernel(const ProbDesc* __restrict__ pds,
                                                           const Item* __restrict__ items) {
  const Item it = items[blockIdx.x];
  const ProbDesc& pd = pds[it.prob];
  const int64_t K = pd.K, W = pd.W, elems = K * W;
  const int64_t e = (int64_t)it.a * kReduceElems + 2 * threadIdx.x;
  if (e >= elems) return;
  const bool second = e + 1 < elems;
  auto needed = [&](int64_t x) {
    const int64_t i = x / W, j = x - i * W;
    return !(j < K && j < i);
  };
  const bool n0 = needed(e), n1 = second && needed(e + 1);
  if (!n0 && !n1) return;
  const bool vec = (elems & 1) == 0;  // then e is even and the pair 16-byte aligned
  CVG_GLOBAL double* slabs = gmem(pd.slabs) + e;
  CVG_GLOBAL double* G = gmem(pd.G) + e;
  auto store = [&](CVG_GLOBAL double* q, double a, double b) {
    if (n0) q[0] = a;
    if (n1) q[1] = b;
  };
  // slabs [s0, s1) summed in slab order, eight loads in flight per group
  // (indices past the range read its last slab again and are not added)
  auto run = [&](auto vec_c) {
    constexpr bool V = decltype(vec_c)::value;
    auto sum_range = [&](int32_t s0, int32_t s1, double& f0, double& f1) {
      if (s1 - s0 == 1) {  // one slab (many small folds): nothing to add
        load_pair(slabs + (int64_t)s0 * elems, V, second, f0, f1);
        return;
      }
      for (int32_t k = s0; k < s1; k += 8) {
        double v0[8], v1[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int32_t ks = k + u < s1 ? k + u : s1 - 1;
          load_pair(slabs + (int64_t)ks * elems, V, second, v0[u], v1[u]);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          if (k + u == s0) {
            f0 = v0[u];
            f1 = v1[u];
          } else if (k + u < s1) {
            f0 += v0[u];
            f1 += v1[u];
          }
        }
      }
    };
    if (pd.fused) {
      // fused path: the slabs are row splits of the full Gram only
      double g0 = 0.0, g1 = 0.0;
      sum_range(0, pd.n_slabs, g0, g1);
      store(G, g0, g1);
      return;
    }
    const CVG_GLOBAL int32_t* slab_begin = gmem(pd.slab_begin);
    const int32_t P = pd.P;
    double g0 = 0.0, g1 = 0.0;
    int32_t a = slab_begin[0];
    for (int32_t p = 0; p < P; ++p) {
      const int32_t b = slab_begin[p + 1];
      double f0 = 0.0, f1 = 0.0;
      sum_range(a, b, f0, f1);
      if (b > a + 1) store(slabs + (int64_t)a * elems, f0, f1);
      g0 += f0;
      g1 += f1;
      a = b;
    }
    store(G, g0, g1);
  };
  if (vec)
    run(std::true_type{});
  else
    run(std::false_type{});
}

// element (row r, packed column col) of the packed panels as FP64: the
// shifted value the Gram launch multiplied (hi + lo in the bf16 split)
__device__ inline double packed_value(const ProbDesc& pd, int64_t r, int64_t col, int64_t Wp) {
  if (pd.panel_f32) {
    // raw FP32 values, shifted here (padding columns: 0)
    const int64_t sc = col < pd.Kp ? (col < pd.K ? col : -1)
                                   : (col - pd.Kp < pd.M ? pd.K + (col - pd.Kp) : -1);
    if (sc < 0) return 0.0;
    return (double)gmem((const float*)pd.packed)[r * Wp + col] - gmem(pd.pivot)[sc];
  }
  if (pd.mode == CVGRAM_MODE_FP64) return gmem((const double*)pd.packed)[r * Wp + col];
  if (pd.mode == CVGRAM_MODE_FP32) return (double)gmem((const float*)pd.packed)[r * Wp + col];
  const int64_t k = ((r >> 5) * Wp + col) * 32 + (r & 31);
  return (double)((float)gmem((const __bf16*)pd.packed)[k] +
                  (float)gmem((const __bf16*)pd.packed_lo)[k]);
}

template <typename OutT>
__device__ void correct_tile(const ProbDesc& pd, const OutDesc& od, int32_t f, int tile) {
  __shared__ double T[TS][TS + 1];
  __shared__ double rc[TS], ra[TS], rmu[TS], rsd[TS];
  __shared__ double cc[TS], ca[TS], cmu[TS], csd[TS];
  __shared__ uint8_t rcs[TS], ccs[TS];
  // leakage comparison: all-row shifted sums, deviations, constant flags
  __shared__ double rS[TS], cS[TS], rsg[TS], csg[TS];
  __shared__ uint8_t rgc[TS], cgc[TS];

  const int32_t p = od.p_begin + f;
  const bool is_xy = tile >= pd.n_ctiles_xx;
  const CVG_GLOBAL int32_t* ctiles = gmem(pd.ctiles);
  const int bi = ctiles[2 * tile];
  const int bj = ctiles[2 * tile + 1];
  const CVG_GLOBAL double* pivot = gmem((const double*)pd.pivot);
  const CVG_GLOBAL double* tr_sum = gmem((const double*)pd.tr_sum);
  const CVG_GLOBAL double* tr_mean = gmem((const double*)pd.tr_mean);
  const CVG_GLOBAL double* tr_std = gmem((const double*)pd.tr_std);
  const CVG_GLOBAL uint8_t* tr_const = gmem((const uint8_t*)pd.tr_const);
  const bool diag = !is_xy && bi == bj;
  const int64_t K = pd.K, M = pd.M, W = pd.W;
  const int64_t ncols = is_xy ? M : K;
  const int64_t coff = is_xy ? K : 0;  // column offset of the tile inside Z

  const int t = threadIdx.x;
  const int tx = t % TS, ty = t / TS;
  const int64_t pw = (int64_t)p * W;
  // this thread's entries; their full-data and (grouped path) fold Gram
  // values are loaded first, so that these loads and the statistics' loads
  // below are in flight together
  bool ok[kRowsPerThread];
  double gfull[kRowsPerThread], gfold[kRowsPerThread];
  {
    const CVG_GLOBAL double* G = gmem((const double*)pd.G);
    const CVG_GLOBAL double* gp_slab =
        pd.fused ? nullptr
                 : gmem((const double*)pd.slabs) + (int64_t)gmem(pd.slab_begin)[p] * K * W;
#pragma unroll
    for (int r = 0; r < kRowsPerThread; ++r) {
      const int il = ty + 8 * r, jl = tx;
      const int64_t i = (int64_t)bi * TS + il;
      const int64_t j = (int64_t)bj * TS + jl;
      ok[r] = i < K && j < ncols && (!diag || il <= jl);
      const int64_t e = i * W + coff + j;
      gfull[r] = ok[r] ? G[e] : 0.0;
      gfold[r] = ok[r] && gp_slab ? gp_slab[e] : 0.0;
    }
  }
  if (t < TS) {
    const int64_t i = (int64_t)bi * TS + t;
    if (i < K) {
      rc[t] = pivot[i];
      ra[t] = tr_sum[pw + i];
      rmu[t] = tr_mean[pw + i];
      rsd[t] = tr_std[pw + i];
      rcs[t] = tr_const[pw + i];
    }
  } else if (t < 2 * TS) {
    const int u = t - TS;
    const int64_t j = (int64_t)bj * TS + u;
    if (j < ncols) {
      const int64_t z = coff + j;
      cc[u] = pivot[z];
      ca[u] = tr_sum[pw + z];
      cmu[u] = tr_mean[pw + z];
      csd[u] = tr_std[pw + z];
      ccs[u] = tr_const[pw + z];
    }
  }
  if (od.leak) {
    // statistics of all N rows from the fold totals (Lemma 12 on shifted sums)
    const CVG_GLOBAL double* tot = gmem((const double*)pd.tot);
    const double Nd = (double)pd.N;
    auto all_rows = [&](int64_t z, double& S, double& sd, uint8_t& cst) {
      S = tot[0 * W + z];
      const double var = (tot[1 * W + z] - S * (S / Nd)) / (Nd - (double)pd.ddof);
      cst = tot[2 * W + z] == tot[5 * W + z] ? 1 : 0;
      sd = sqrt(var > 0.0 ? var : 0.0);
      if (cst || sd == 0.0) sd = 1.0;
    };
    if (t < TS) {
      const int64_t i = (int64_t)bi * TS + t;
      if (i < K) all_rows(i, rS[t], rsg[t], rgc[t]);
    } else if (t < 2 * TS) {
      const int u = t - TS;
      const int64_t j = (int64_t)bj * TS + u;
      if (j < ncols) all_rows(coff + j, cS[u], csg[u], cgc[u]);
    }
  }
  __syncthreads();

  const double NT = (double)gmem((const int64_t*)pd.ntrain)[p];

  // G'_p for this thread's entries: the fold's slab sum (grouped path), or
  // formed here from the fold's packed rows in fold order (fused path)
  double gp[kRowsPerThread] = {0.0, 0.0, 0.0, 0.0};
  if (pd.fused) {
    __shared__ double zi[TS][TS + 1], zj[TS][TS + 1];
    const int64_t r0 = gmem(pd.poff)[p], r1 = gmem(pd.poff)[p + 1];
    const int64_t Wp = pd.Wp;
    const int64_t pcol = is_xy ? pd.Kp : 0;  // packed column of the tile's first column
    for (int64_t c0 = r0; c0 < r1; c0 += TS) {
      const int nv = (int)(r1 - c0 < TS ? r1 - c0 : TS);
      for (int idx = t; idx < TS * TS; idx += kThreads) {
        const int v = idx / TS, c = idx % TS;
        const int64_t i = (int64_t)bi * TS + c, j = (int64_t)bj * TS + c;
        double a = 0.0, b = 0.0;
        if (v < nv) {
          if (i < K) a = packed_value(pd, c0 + v, i, Wp);
          if (j < ncols) b = packed_value(pd, c0 + v, pcol + j, Wp);
        }
        zi[v][c] = a;
        zj[v][c] = b;
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < kRowsPerThread; ++r) {
        const int il = ty + 8 * r, jl = tx;
        for (int v = 0; v < nv; ++v) gp[r] = fma(zi[v][il], zj[v][jl], gp[r]);
      }
      __syncthreads();
    }
  }
  double raw[kRowsPerThread], cen[kRowsPerThread], gT[kRowsPerThread];
#pragma unroll
  for (int r = 0; r < kRowsPerThread; ++r) {
    const int il = ty + 8 * r, jl = tx;
    raw[r] = 0.0;
    cen[r] = 0.0;
    gT[r] = 0.0;
    if (!ok[r]) continue;
    const double g = gfull[r] - (pd.fused ? gp[r] : gfold[r]);
    gT[r] = g;
    raw[r] = g + (rc[il] * ca[jl] + ra[il] * cc[jl]) + NT * (rc[il] * cc[jl]);
    cen[r] = (rcs[il] || ccs[jl]) ? 0.0 : g - NT * (rmu[il] * cmu[jl]);
  }

  if (od.leak) {
    // Leakage comparison (Section 4.1), one output pair.  Global: training
    // rows centred by a = all-row mean (or 0) and scaled by all-row
    // deviations: sum_T (z_i + al_i)(w_j + be_j) with al = c - a (shifted z).
    // Lindgren et al. (Lemma 11's Equation (20)): raw products minus
    // xbar_i (validation sum)_j + xbar_j (validation sum)_i - (N/P) xbar_i xbar_j.
    const double Nd = (double)pd.N, Pd = (double)pd.P;
    OutT* out = (OutT*)(is_xy ? od.xy[0] : od.xx[0]);
    if (!out) return;
    CVG_GLOBAL OutT* o = gmem(out);
    const bool ci = od.lcx, cj = is_xy ? od.lcy : od.lcx;
    const bool si = od.lsx, sj = is_xy ? od.lsy : od.lsx;
#pragma unroll
    for (int r = 0; r < kRowsPerThread; ++r) {
      if (!ok[r]) continue;
      const int il = ty + 8 * r, jl = tx;
      const int64_t i = (int64_t)bi * TS + il;
      const int64_t j = (int64_t)bj * TS + jl;
      double v;
      if (od.leak == 2) {
        const double xi = rc[il] + rS[il] / Nd, xj = cc[jl] + cS[jl] / Nd;
        const double vi = (rS[il] - ra[il]) + rc[il] * (Nd - NT);
        const double vj = (cS[jl] - ca[jl]) + cc[jl] * (Nd - NT);
        v = raw[r] - xi * vj - xj * vi + (Nd / Pd) * (xi * xj);
      } else {
        const double al = ci ? -rS[il] / Nd : rc[il];
        const double be = cj ? -cS[jl] / Nd : cc[jl];
        v = gT[r] + (al * ca[jl] + ra[il] * be) + NT * (al * be);
        if ((ci && rgc[il]) || (cj && cgc[jl])) v = 0.0;
        if (si || sj) v = v / ((si ? rsg[il] : 1.0) * (sj ? csg[jl] : 1.0));
      }
      if (is_xy) {
        o[i * M + j] = (OutT)v;
      } else {
        o[i * K + j] = (OutT)v;
        if (!diag || il != jl) o[j * K + i] = (OutT)v;
      }
    }
    return;
  }

  // The classes are written once and not read back here: non-temporal
  // stores keep them from displacing G and the statistics, which every fold
  // re-reads, from the caches (leave-one-out N = 1e5, K = 512: 203 -> 194 ms
  // for all folds' classes).
  if (!is_xy) {
    for (int c = 0; c < CVGRAM_XTX_CLASSES; ++c) {
      if (!od.xx[c]) continue;
      CVG_GLOBAL OutT* out = gmem((OutT*)od.xx[c]) + (int64_t)f * od.fold_stride_xx;
      const bool centred = c & 2, scaled = c & 1;
      double v[kRowsPerThread];
#pragma unroll
      for (int r = 0; r < kRowsPerThread; ++r) {
        const int il = ty + 8 * r, jl = tx;
        v[r] = centred ? cen[r] : raw[r];
        if (scaled && ok[r]) v[r] = v[r] / (rsd[il] * csd[jl]);
        if (ok[r]) T[il][jl] = v[r];
      }
      lds_barrier();
#pragma unroll
      for (int r = 0; r < kRowsPerThread; ++r) {
        const int il = ty + 8 * r, jl = tx;
        const int64_t i = (int64_t)bi * TS + il;
        const int64_t j = (int64_t)bj * TS + jl;
        if (diag) {
          if (i < K && j < K)
            __builtin_nontemporal_store((OutT)(il <= jl ? T[il][jl] : T[jl][il]), &out[i * K + j]);
        } else {
          if (ok[r]) __builtin_nontemporal_store((OutT)v[r], &out[i * K + j]);
          // transposed block: rows of bj, columns of bi
          const int64_t ti = (int64_t)bj * TS + il;
          const int64_t tj = (int64_t)bi * TS + jl;
          if (ti < K && tj < K) __builtin_nontemporal_store((OutT)T[jl][il], &out[ti * K + tj]);
        }
      }
      lds_barrier();
    }
  } else {
    for (int c = 0; c < CVGRAM_XTY_CLASSES; ++c) {
      if (!od.xy[c]) continue;
      CVG_GLOBAL OutT* out = gmem((OutT*)od.xy[c]) + (int64_t)f * od.fold_stride_xy;
      const bool centred = c & 4, scx = c & 2, scy = c & 1;
#pragma unroll
      for (int r = 0; r < kRowsPerThread; ++r) {
        if (!ok[r]) continue;
        const int il = ty + 8 * r, jl = tx;
        double v = centred ? cen[r] : raw[r];
        if (scx || scy) v = v / ((scx ? rsd[il] : 1.0) * (scy ? csd[jl] : 1.0));
        const int64_t i = (int64_t)bi * TS + il;
        const int64_t j = (int64_t)bj * TS + jl;
        __builtin_nontemporal_store((OutT)v, &out[i * M + j]);
      }
    }
  }
}

// one problem: grid.x = its correction tiles, grid.y strides over the folds
// (a grid dimension other than x is limited to 65535 blocks)
template <typename OutT>
__global__ __launch_bounds__(kThreads) void correct_single_kernel(const ProbDesc* __restrict__ pds,
                                                                  int32_t prob, OutDesc od,
                                                                  int32_t n_folds) {
  const ProbDesc& pd = pds[prob];
  for (int32_t f = blockIdx.y; f < n_folds; f += gridDim.y) {
    correct_tile<OutT>(pd, od, f, blockIdx.x);
    lds_barrier();  // the next fold reuses the LDS arrays
  }
}

// many problems: items (prob, fold, tile), outputs of every fold
template <typename OutT>
__global__ __launch_bounds__(kThreads) void correct_batch_kernel(const ProbDesc* __restrict__ pds,
                                                                 const OutDesc* __restrict__ outs,
                                                                 const Item* __restrict__ items) {
  const Item it = items[blockIdx.x];
  correct_tile<OutT>(pds[it.prob], outs[it.prob], it.a, it.b);
}

}  // namespace

void launch_reduce_slabs(const ProbDesc* pd, const Item* items, int64_t n_items, hipStream_t s) {
  if (n_items <= 0) return;
  reduce_slabs_kernel<<<(unsigned)n_items, kReduceElems / 2, 0, s>>>(pd, items);
  CVG_LAUNCH_CHECK();
}

void launch_correct_single(const ProbDesc* pd, int32_t prob, int32_t n_tiles, const OutDesc& out,
                           int32_t n_folds, bool out_f64, hipStream_t s) {
  if (n_tiles <= 0 || n_folds <= 0) return;
  dim3 grid((unsigned)n_tiles, (unsigned)(n_folds < 65535 ? n_folds : 65535));
  if (out_f64)
    correct_single_kernel<double><<<grid, kThreads, 0, s>>>(pd, prob, out, n_folds);
  else
    correct_single_kernel<float><<<grid, kThreads, 0, s>>>(pd, prob, out, n_folds);
  CVG_LAUNCH_CHECK();
}

void launch_correct_batch(const ProbDesc* pd, const OutDesc* outs, const Item* items,
                          int64_t n_items, bool out_f64, hipStream_t s) {
  if (n_items <= 0) return;
  if (out_f64)
    correct_batch_kernel<double><<<(unsigned)n_items, kThreads, 0, s>>>(pd, outs, items);
  else
    correct_batch_kernel<float><<<(unsigned)n_items, kThreads, 0, s>>>(pd, outs, items);
  CVG_LAUNCH_CHECK();
}

}  // namespace cvg
