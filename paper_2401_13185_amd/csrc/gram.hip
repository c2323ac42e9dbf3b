// Grouped validation-block Gram products on the matrix cores, from the
// packed panels written by the pack pass.
//
// For every fold p (Algorithm 7 step 8, Lemmas 2-3) the library needs
// G'_p = Z'_{V_p}^T Z'_{V_p} restricted to its first K rows, Z' being the
// pivot-shifted data.  All folds of all problems run in ONE launch over a
// work list of (problem, fold row range, output tile) items; a fold's rows
// are contiguous and zero-padded in the packed panels, so an item streams
// aligned 16-byte vector loads with no gathers and no bounds checks.
// Output tiles are BM x BM (BM = 64 or 128, chosen per problem): every tile
// on or above the diagonal of the K x K block.  When M <= 32 the K x M block
// rides on the diagonal tiles (no extra pass over X), else it gets separate
// tiles.  A 64-wide diagonal tile (and every BF16X3 one) gives its three
// upper 32 x 32 quadrants to three waves and the K x M block to the fourth;
// a 128-wide FP64 / FP32 diagonal tile splits its upper-triangle 16 x 16
// blocks and K x M blocks evenly over the four waves.  Each item writes its
// FP64 tile to its own slab (summed later in a fixed order: deterministic,
// no floating-point atomics).
//
// Arithmetic per mode:
//   FP64    v_mfma_f64_16x16x4_f64 on FP64 panels (or on FP32 panels of
//           FP32 input, shifted to FP64 as they are loaded), FP64
//           accumulation.
//   FP32    v_mfma_f32_16x16x4_f32 on FP32 panels.
//   BF16X3  three products hi*hi + hi*lo + lo*hi per FP32 product from the
//           hi/lo bf16 panels: v_mfma_f32_16x16x32_bf16 on 64- and 128-wide
//           tiles, v_mfma_f32_32x32x16_bf16 on 256 x 128 tiles (the kernel
//           at the end of this file).
// The FP32-accumulating modes add their FP32 tile into an FP64 register
// tile and clear it every 64 rows (FP32: 16 accumulating MFMAs) or 256 rows
// (BF16X3: 24, each summing 32 products; on 256 x 128 tiles into FP32
// totals every 512 rows), so FP32 rounding does not grow with the fold
// size.  The accumulated rounding error of a block is about
// half an FP32 ulp per accumulating step, and it does not average out on
// entries that sum positive products (the diagonal).  On the offset data
// of the precision-stress workload (N=1e6, K=1024) the FP32 mode's worst
// entry against its Cauchy-Schwarz scale was 1.9e-6 with a flush every 256
// rows and is 4.9e-7 with one every 64 (the Gram 6 % slower).
//
// Pipelining.  FP64 / FP32: LDS double buffer; the next stage's panel block
// is loaded into registers while the current stage runs on the matrix cores;
// one barrier per stage.  BF16X3: the panels are already k-contiguous, so
// stages go straight from global memory into a ring of four LDS buffers with
// direct-to-LDS loads (no register staging, no LDS store instructions), three
// stages ahead of the matrix cores; 16-byte chunks are XOR-swizzled per
// column so the fragment reads are free of bank conflicts.  Work items are
// mapped XCD-aware: each of the 8 XCDs runs its own range of the list (the
// planner balances the ranges and keeps the tiles that read the same rows
// in one range, where they share the XCD's L2).
#include "internal.h"

#include <type_traits>

namespace cvg {
namespace {

typedef double double2_t __attribute__((ext_vector_type(2)));
typedef double double4_t __attribute__((ext_vector_type(4)));
typedef float float4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

constexpr int kThreads = 256;
constexpr int kYW = kYDiagCols;    // Y columns handled inside diagonal tiles (32)
constexpr int kFlushRowsBf16 = 256;   // rows between FP64 flushes (BF16X3)
// row steps of 4 rows each wave keeps in flight in the direct FP64 loop
constexpr int kDirectDepth = 4;
// the loop runs kDirectDepth steps per pass over an item's kPanelRows / 4
// steps per panel, so the depth must divide them
static_assert((kPanelRows / 4) % kDirectDepth == 0, "direct depth must divide a panel's steps");

template <int MODE>
struct Mode;
template <>
struct Mode<CVGRAM_MODE_FP64> {
  typedef double E;
  typedef double4_t Acc;
  static constexpr int BK = 16;
  static constexpr int PAD = 16;      // rows of 144 / 80 doubles: the two rows of a
};                                    // 32-lane half of a fragment read use disjoint banks
template <>
struct Mode<CVGRAM_MODE_FP32> {
  typedef float E;
  typedef float4_t Acc;
  static constexpr int BK = 16;
  static constexpr int PAD = 16;      // rows of 144 / 80 floats: the 4 row groups of a
                                      // fragment read fall in different banks
  static constexpr int FLUSH = 64;    // rows between FP64 flushes
};
template <>
struct Mode<CVGRAM_MODE_BF16X3> {
  typedef __bf16 E;
  typedef float4_t Acc;
  static constexpr int BK = 32;       // one packed panel per stage
};

// row of element e of lane l's accumulator inside a 16 x 16 MFMA block
template <int MODE>
__device__ inline int acc_row(int e, int fr) {
  return MODE == CVGRAM_MODE_FP64 ? 4 * e + fr : 4 * fr + e;
}

template <int MODE, int BM>
struct Smem {
  static constexpr int LDA = BM + Mode<MODE>::PAD;
  static constexpr int LDY = kYW + Mode<MODE>::PAD;
  typename Mode<MODE>::E a[2][16 * LDA];
  // B operand (off-diagonal tiles) or the Y block (diagonal tiles) share
  // storage: a diagonal tile reuses A as B
  union {
    typename Mode<MODE>::E b[2][16 * LDA];
    typename Mode<MODE>::E y[2][16 * LDY];
  };
};
// ---------------------------------------------------------------------------
// global -> register staging of one stage (BK packed rows starting at row r)
// ---------------------------------------------------------------------------
// pivot of packed column pc (0 for a padding column): the shift FP32 panels
// of the FP64 mode get as they are loaded
__device__ inline double panel_pivot(const CVG_GLOBAL double* pivot, int64_t pc, int64_t K,
                                     int64_t Kp, int64_t M) {
  if (pc < Kp) return pc < K ? pivot[pc] : 0.0;
  return pc - Kp < M ? pivot[K + (pc - Kp)] : 0.0;
}

// FP64 / FP32: an operand block is 16 rows x BM columns, moved in 16-byte
// chunks; consecutive threads take consecutive chunks of a row, so both the
// global loads and the LDS stores are contiguous.  The Y block (16 x 32) is
// one chunk for each of the first 16 * 32 * sizeof(E) / 16 threads.  F32P
// (FP64 mode on FP32 panels): the chunks hold four FP32 values, stored to
// LDS as FP64 minus their columns' pivots (a thread's columns are the same
// in every stage, so their pivots are read once).
template <int MODE, int BM, bool F32P = false>
struct Stage {
  typedef typename Mode<MODE>::E E;                  // LDS element
  typedef typename std::conditional<F32P, float, E>::type LE;  // panel element
  typedef LE V16 __attribute__((ext_vector_type(16 / sizeof(LE))));
  static constexpr int EPC = 16 / sizeof(LE);       // elements per chunk
  static constexpr int CPR = BM / EPC;              // chunks per row
  static constexpr int RPR = kThreads / CPR;        // rows per round
  static constexpr int V = 16 / RPR;                // chunks per thread per operand
  static constexpr int YC = kYW / EPC;              // chunks per Y row
  V16 a[V], b[V], y;
  __device__ void load(const CVG_GLOBAL LE* Z, int64_t Wp, int64_t r, int64_t ca, int64_t cb,
                       int64_t cy, bool ld_b, bool ld_y, int t) {
    const int row0 = t / CPR, col = (t % CPR) * EPC;
#pragma unroll
    for (int u = 0; u < V; ++u)
      a[u] = *(const CVG_GLOBAL V16*)(Z + (r + row0 + RPR * u) * Wp + ca + col);
    if (ld_b) {
#pragma unroll
      for (int u = 0; u < V; ++u)
        b[u] = *(const CVG_GLOBAL V16*)(Z + (r + row0 + RPR * u) * Wp + cb + col);
    }
    if (ld_y && t < 16 * YC)
      y = *(const CVG_GLOBAL V16*)(Z + (r + t / YC) * Wp + cy + (t % YC) * EPC);
  }
  template <typename Piv>
  __device__ void store(Smem<MODE, BM>& s, int buf, bool st_b, bool st_y, int t,
                        const Piv& pv) const {
    constexpr int LDA = Smem<MODE, BM>::LDA, LDY = Smem<MODE, BM>::LDY;
    const int row0 = t / CPR, col = (t % CPR) * EPC;
    if constexpr (!F32P) {
#pragma unroll
      for (int u = 0; u < V; ++u) *(V16*)&s.a[buf][(row0 + RPR * u) * LDA + col] = a[u];
      if (st_b)
#pragma unroll
        for (int u = 0; u < V; ++u) *(V16*)&s.b[buf][(row0 + RPR * u) * LDA + col] = b[u];
      if (st_y && t < 16 * YC) *(V16*)&s.y[buf][(t / YC) * LDY + (t % YC) * EPC] = y;
    } else {
      // four FP32 values -> four shifted FP64 values (two 16-byte stores)
      auto put = [&](double* dst, const V16& v, const double* piv) {
        double2_t lo, hi;
        lo.x = (double)v[0] - piv[0];
        lo.y = (double)v[1] - piv[1];
        hi.x = (double)v[2] - piv[2];
        hi.y = (double)v[3] - piv[3];
        *(double2_t*)dst = lo;
        *(double2_t*)(dst + 2) = hi;
      };
#pragma unroll
      for (int u = 0; u < V; ++u) put(&s.a[buf][(row0 + RPR * u) * LDA + col], a[u], pv.a);
      if (st_b)
#pragma unroll
        for (int u = 0; u < V; ++u) put(&s.b[buf][(row0 + RPR * u) * LDA + col], b[u], pv.b);
      if (st_y && t < 16 * YC) put(&s.y[buf][(t / YC) * LDY + (t % YC) * EPC], y, pv.y);
    }
  }
};
// the pivots of one thread's stage columns (F32P) or nothing
template <bool F32P>
struct StagePivots {
  double a[4], b[4], y[4];
};
template <>
struct StagePivots<false> {};


// ---------------------------------------------------------------------------
// one stage of MFMA work for a wave: NA x NB blocks of 16 x 16, A columns
// from `acol0` of the A view, B columns from `bcol0` of the B view.
// ---------------------------------------------------------------------------
__device__ inline double4_t mfma_step(double a, double b, double4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline float4_t mfma_step(float a, float b, float4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <int NA, int NB, int NACC>
__device__ inline void mma_f64(const double* A, int lda, int acol0, const double* B, int ldb,
                               int bcol0, double4_t (&acc)[NACC], int fr, int fc) {
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    double af[NA], bf[NB];
#pragma unroll
    for (int a = 0; a < NA; ++a) af[a] = A[(kk * 4 + fr) * lda + acol0 + a * 16 + fc];
#pragma unroll
    for (int b = 0; b < NB; ++b) bf[b] = B[(kk * 4 + fr) * ldb + bcol0 + b * 16 + fc];
#pragma unroll
    for (int a = 0; a < NA; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b)
        acc[a * NB + b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bf[b], acc[a * NB + b], 0,
                                                               0, 0);
  }
}

template <int NA, int NB, int NACC>
__device__ inline void mma_f32(const float* A, int lda, int acol0, const float* B, int ldb,
                               int bcol0, float4_t (&acc)[NACC], int fr, int fc) {
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    float af[NA], bf[NB];
#pragma unroll
    for (int a = 0; a < NA; ++a) af[a] = A[(kk * 4 + fr) * lda + acol0 + a * 16 + fc];
#pragma unroll
    for (int b = 0; b < NB; ++b) bf[b] = B[(kk * 4 + fr) * ldb + bcol0 + b * 16 + fc];
#pragma unroll
    for (int a = 0; a < NA; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b)
        acc[a * NB + b] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[a], bf[b], acc[a * NB + b], 0,
                                                               0, 0);
  }
}

// BF16X3 stage buffers in LDS: per array, column c of the 32-row panel is
// 64 bytes (four 16-byte chunks of 8 rows); chunk k of column c sits at
// position k ^ swz(c).  Sixteen lanes reading one chunk of sixteen
// consecutive columns then hit sixteen different 16-byte bank groups (with
// 32 or with 64 banks of 4 bytes).
__device__ __forceinline__ int swz(int c) { return ((c >> 1) ^ (c >> 2)) & 3; }

// accumulator of a 32 x 32 output block (v_mfma_f32_32x32x16_bf16, the
// 256 x 128 kernel)
typedef float float16_t __attribute__((ext_vector_type(16)));

// One stage's fragments for NA x NB blocks of 16 x 16: A columns from
// `acol0`, B columns from `bcol0` (multiples of 16) of the swizzled buffers;
// `lfo` is the lane's byte offset fc * 64 + ((fr ^ swz(fc)) << 4).
template <int NA, int NB>
struct Frags {
  bf16x8_t ah[NA], al[NA], bh[NB], bl[NB];
  __device__ void load(const __bf16* Ah, const __bf16* Al, int acol0, const __bf16* Bh,
                       const __bf16* Bl, int bcol0, int lfo) {
#pragma unroll
    for (int a = 0; a < NA; ++a) {
      const int off = (acol0 + a * 16) * 64 + lfo;
      ah[a] = *(const bf16x8_t*)((const char*)Ah + off);
      al[a] = *(const bf16x8_t*)((const char*)Al + off);
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int off = (bcol0 + b * 16) * 64 + lfo;
      bh[b] = *(const bf16x8_t*)((const char*)Bh + off);
      bl[b] = *(const bf16x8_t*)((const char*)Bl + off);
    }
  }
};

// One of the three products over all blocks (consecutive MFMAs update
// different accumulators): pass 0 lo(A) hi(B), pass 1 hi(A) lo(B), pass 2
// hi(A) hi(B).
template <int PASS, int NA, int NB, int NACC>
__device__ inline void mfma_pass(const Frags<NA, NB>& f, float4_t (&acc)[NACC]) {
#pragma unroll
  for (int a = 0; a < NA; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b)
      acc[a * NB + b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
          PASS == 0 ? f.al[a] : f.ah[a], PASS == 1 ? f.bl[b] : f.bh[b], acc[a * NB + b], 0, 0, 0);
}

// ---------------------------------------------------------------------------
// diagonal 128 x 128 tiles (FP64 / FP32): only the upper triangle of its
// 8 x 8 blocks of 16 x 16 is needed (plus the K x M blocks when the tile
// carries them).  Wave W takes block rows W and 7 - W: (8 - W) + (W + 1) = 9
// blocks of the triangle and NYB blocks of the K x M block per row, the same
// count for every wave.  A block's fragment is the same register whether it
// serves as A or as B (both are columns of the same stage), so a wave reads
// the 8 - W fragments of blocks W .. 7 once per k-step.
// Accumulator order: row W's blocks (columns W .. 7), row 7 - W's blocks
// (columns 7 - W .. 7), then row W's and row 7 - W's K x M blocks.
// ---------------------------------------------------------------------------
template <int W, int NYB, typename E, typename Acc, int NACC>
__device__ inline void mma_diag_pairs(const E* A, int lda, const E* Yb, int ldy,
                                      Acc (&acc)[NACC], int fr, int fc) {
  constexpr int R0 = W, R1 = 7 - W, N0 = 8 - R0, N1 = 8 - R1;
  static_assert(N0 + N1 + 2 * NYB <= NACC, "accumulators");
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    E f[N0], y[NYB > 0 ? NYB : 1];
#pragma unroll
    for (int c = 0; c < N0; ++c) f[c] = A[(kk * 4 + fr) * lda + (R0 + c) * 16 + fc];
#pragma unroll
    for (int q = 0; q < NYB; ++q) y[q] = Yb[(kk * 4 + fr) * ldy + q * 16 + fc];
#pragma unroll
    for (int c = 0; c < N0; ++c) acc[c] = mfma_step(f[0], f[c], acc[c]);
#pragma unroll
    for (int c = 0; c < N1; ++c)
      acc[N0 + c] = mfma_step(f[R1 - R0], f[R1 - R0 + c], acc[N0 + c]);
#pragma unroll
    for (int q = 0; q < NYB; ++q) {
      acc[N0 + N1 + q] = mfma_step(f[0], y[q], acc[N0 + N1 + q]);
      acc[N0 + N1 + NYB + q] = mfma_step(f[R1 - R0], y[q], acc[N0 + N1 + NYB + q]);
    }
  }
}

template <int MODE, int W, int NYB, typename V>
__device__ inline void store_diag_pairs(CVG_GLOBAL double* out, int64_t ca, int fr, int fc,
                                        int64_t K, int64_t M, const V& value) {
  constexpr int R0 = W, R1 = 7 - W, N0 = 8 - R0, N1 = 8 - R1;
  const int64_t Wd = K + M;
#pragma unroll
  for (int i = 0; i < N0 + N1 + 2 * NYB; ++i) {
    const int rb = i < N0 ? R0 : (i < N0 + N1 ? R1 : (i < N0 + N1 + NYB ? R0 : R1));
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t row = ca + rb * 16 + acc_row<MODE>(e, fr);
      if (row >= K) continue;
      if (i < N0 + N1) {
        const int cblk = i < N0 ? R0 + i : R1 + (i - N0);
        const int64_t cl = ca + cblk * 16 + fc;
        if (cl < K) out[row * Wd + cl] = value(i, e);
      } else {
        const int q = (i - N0 - N1) % (NYB > 0 ? NYB : 1);
        const int64_t cl = q * 16 + fc;
        if (cl < M) out[row * Wd + K + cl] = value(i, e);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// epilogue shared by both kernels: the wave's FP64 results into the item's
// slab (rows of X, columns of X or Y; entries outside K x K / K x M skipped)
// ---------------------------------------------------------------------------
template <int MODE, int BM, int NACC, typename V>
__device__ inline void store_tile(CVG_GLOBAL double* out, int role, bool xy_tile, int64_t ca,
                                  int64_t cbl, int wm, int wn, int fr, int fc, int64_t K,
                                  int64_t M, const V& value) {
  constexpr int WT = BM / 2, NW = WT / 16, NY = BM / 16;
  const int64_t W = K + M;
  if (role == 0) {
#pragma unroll
    for (int a = 0; a < NW; ++a)
#pragma unroll
      for (int b = 0; b < NW; ++b)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int64_t row = ca + wm * WT + a * 16 + acc_row<MODE>(e, fr);
          const int64_t cl = cbl + wn * WT + b * 16 + fc;
          if (row >= K) continue;
          if (!xy_tile) {
            if (cl < K) out[row * W + cl] = value(a * NW + b, e);
          } else if (cl < M) {
            out[row * W + K + cl] = value(a * NW + b, e);
          }
        }
  } else if (role == 1) {
#pragma unroll
    for (int a = 0; a < NY; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int64_t row = ca + a * 16 + acc_row<MODE>(e, fr);
          const int64_t cl = b * 16 + fc;
          if (row < K && cl < M) out[row * W + K + cl] = value(a * 2 + b, e);
        }
  }
}

// ---------------------------------------------------------------------------
// FP64 / FP32 kernel: register-staged LDS double buffer
// ---------------------------------------------------------------------------
// FP32 panels in FP64 mode: held to two workgroups per CU (at most 256
// registers per lane), as the FP64 panels fit by themselves
template <int MODE, int BM, bool F32P>
__global__ __launch_bounds__(kThreads, F32P ? 2 : 1) void gram_kernel(
    const ProbDesc* __restrict__ pds,
                                                        const GramWork* __restrict__ work,
                                                        const int32_t* __restrict__ xcd) {
  typedef typename Mode<MODE>::Acc Acc;
  constexpr int BK = Mode<MODE>::BK;
  constexpr bool kF64 = MODE == CVGRAM_MODE_FP64;
  constexpr int WT = BM / 2;              // wave tile edge
  constexpr int NW = WT / 16;             // 16 x 16 blocks per wave tile edge
  constexpr int NY = BM / 16;             // blocks along the rows of the K x M block
  constexpr int NACC = NW * NW > 2 * NY ? NW * NW : 2 * NY;
  __shared__ __attribute__((aligned(16))) Smem<MODE, BM> sm;

  const int x = (int)(blockIdx.x % kXcds);
  const int64_t item = (int64_t)xcd[x] + blockIdx.x / kXcds;
  if (item >= xcd[x + 1]) return;
  const GramWork w = work[item];
  // descriptor fields in registers (never re-read inside the loop)
  const ProbDesc& pdr = pds[w.prob];
  const int64_t Wp = pdr.Wp, Kp = pdr.Kp, K = pdr.K, M = pdr.M;
  const int32_t nt = pdr.nt;
  typedef typename Stage<MODE, BM, F32P>::LE PE;  // panel element
  const CVG_GLOBAL PE* const packed = gmem((const PE*)pdr.packed);
  CVG_GLOBAL double* const slabs = gmem(pdr.slabs);
  const bool xy_diag = pdr.xy_diag != 0;
  const int t = threadIdx.x, lane = t & 63;
  // wave index made scalar in the FP32-accumulating modes: their roles then
  // branch uniformly; the FP64 loop keeps its vector form (fewer registers)
  const int wave = kF64 ? (t >> 6) : __builtin_amdgcn_readfirstlane(t >> 6);
  const int wm = wave >> 1, wn = wave & 1;
  const int fr = lane >> 4, fc = lane & 15;

  const bool xy_tile = w.tj >= nt;
  const bool diag = !xy_tile && w.ti == w.tj;
  const int64_t ca = (int64_t)w.ti * BM;                                    // A columns
  const int64_t cb = xy_tile ? Kp + (int64_t)(w.tj - nt) * BM : (int64_t)w.tj * BM;
  const bool ydiag = diag && xy_diag;      // K x M block inside this diagonal tile
  const bool ld_b = !diag;                  // diagonal tiles reuse A as B
  // wave roles: 0 = WT x WT sub-tile, 1 = BM x 32 K-by-M block, 2 = idle
  // (64-wide diagonal tiles; 128-wide ones split their triangle evenly)
  constexpr bool kPairs = BM == 128;
  const int role = (!kPairs && diag && wm == 1 && wn == 0) ? (ydiag ? 1 : 2) : 0;
  // K x M blocks of 16 columns a 128-wide diagonal tile computes
  const int nyb = ydiag ? (M <= 16 ? 1 : 2) : 0;

  Acc acc[NACC];
  double a64[NACC][4];
#pragma unroll
  for (int i = 0; i < NACC; ++i) {
    acc[i] = Acc{0, 0, 0, 0};
#pragma unroll
    for (int e = 0; e < 4; ++e) a64[i][e] = 0.0;
  }

  // Global loads run PF stages ahead of the matrix cores: the next stage's
  // panel block is in registers while the current one is consumed from LDS
  // (PF = 2 keeps two stages in flight; FP64 stages are 4x longer and keep
  // one, which also leaves room for two workgroups per CU).  The loop is
  // instantiated per tile kind (off-diagonal / diagonal / diagonal with the
  // K x M block) so that every stage issues the same loads: the wait before
  // an LDS store then covers exactly the stage being stored, not the loads
  // issued after it.  Loads past the last stage re-read the last stage.
  constexpr int PF = kF64 ? 1 : 2;
  const int64_t nst = (w.r1 - w.r0) / BK;
  int since = 0;
  auto flush = [&]() {
    if constexpr (!kF64) {
      since += BK;
      if (since >= Mode<CVGRAM_MODE_FP32>::FLUSH) {
        since = 0;
#pragma unroll
        for (int i = 0; i < NACC; ++i) {
#pragma unroll
          for (int e = 0; e < 4; ++e) a64[i][e] += (double)acc[i][e];
          acc[i] = Acc{0, 0, 0, 0};
        }
      }
    }
  };
  // FP32 panels: the pivots of this thread's stage columns
  StagePivots<F32P> pv;
  if constexpr (F32P) {
    typedef Stage<MODE, BM, true> S;
    const CVG_GLOBAL double* pivot = gmem((const double*)pdr.pivot);
    const int64_t col = (t % S::CPR) * S::EPC, ycol = (t % S::YC) * S::EPC;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      pv.a[e] = panel_pivot(pivot, ca + col + e, K, Kp, M);
      pv.b[e] = panel_pivot(pivot, cb + col + e, K, Kp, M);
      pv.y[e] = panel_pivot(pivot, Kp + ycol + e, K, Kp, M);
    }
  }
  auto main_loop = [&](auto diag_c, auto ydiag_c, auto nyb_c, auto wave_c) {
    constexpr bool DG = decltype(diag_c)::value;   // B is A
    constexpr bool YD = decltype(ydiag_c)::value;  // K x M block in this tile
    constexpr int NYB = decltype(nyb_c)::value;    // its blocks per row (pairs)
    constexpr int WV = decltype(wave_c)::value;    // the wave (pairs)
    Stage<MODE, BM, F32P> st[PF];
    auto load = [&](Stage<MODE, BM, F32P>& sg, int64_t s) {
      const int64_t r = w.r0 + (s < nst ? s : nst - 1) * BK;
      sg.load(packed, Wp, r, ca, cb, Kp, !DG, YD, t);
    };
    auto compute = [&](int buf) {
      if constexpr (kPairs && DG) {
        constexpr int LDA = Smem<MODE, BM>::LDA, LDY = Smem<MODE, BM>::LDY;
        const typename Mode<MODE>::E* A = sm.a[buf];
        const typename Mode<MODE>::E* Yb = sm.y[buf];
        mma_diag_pairs<WV, NYB>(A, LDA, Yb, LDY, acc, fr, fc);
      } else if constexpr (MODE == CVGRAM_MODE_FP64) {
        constexpr int LDA = Smem<MODE, BM>::LDA, LDY = Smem<MODE, BM>::LDY;
        const double* A = sm.a[buf];
        const double* B = DG ? sm.a[buf] : sm.b[buf];
        if (role == 0)
          mma_f64<NW, NW>(A, LDA, wm * WT, B, LDA, wn * WT, acc, fr, fc);
        else if (YD && role == 1)
          mma_f64<NY, 2>(A, LDA, 0, sm.y[buf], LDY, 0, acc, fr, fc);
      } else {
        constexpr int LDA = Smem<MODE, BM>::LDA, LDY = Smem<MODE, BM>::LDY;
        const float* A = sm.a[buf];
        const float* B = DG ? sm.a[buf] : sm.b[buf];
        if (role == 0)
          mma_f32<NW, NW>(A, LDA, wm * WT, B, LDA, wn * WT, acc, fr, fc);
        else if (YD && role == 1)
          mma_f32<NY, 2>(A, LDA, 0, sm.y[buf], LDY, 0, acc, fr, fc);
      }
    };
    load(st[0], 0);
    st[0].store(sm, 0, !DG, YD, t, pv);
    if constexpr (PF == 2) load(st[1], 1);
    __syncthreads();
    if constexpr (PF == 1) {
      for (int64_t s = 0; s < nst; ++s) {
        const int buf = (int)(s & 1);
        const bool more = s + 1 < nst;
        if (more) load(st[0], s + 1);
        compute(buf);
        flush();
        if (more) st[0].store(sm, buf ^ 1, !DG, YD, t, pv);
        __syncthreads();
      }
    } else {
      // stage s is in LDS buffer s & 1 and stage s+1 in registers; stage s+2
      // is loaded while stage s computes.  Unrolled by two so that the two
      // register sets keep fixed roles.
      auto step = [&](int64_t s, Stage<MODE, BM, F32P>& next, Stage<MODE, BM, F32P>& far) {
        const int buf = (int)(s & 1);
        load(far, s + 2);
        compute(buf);
        flush();
        if (s + 1 < nst) next.store(sm, buf ^ 1, !DG, YD, t, pv);
        __syncthreads();
      };
      int64_t s = 0;
      for (; s + 1 < nst; s += 2) {
        step(s, st[1], st[0]);
        step(s + 1, st[0], st[1]);
      }
      if (s < nst) step(s, st[1], st[0]);
    }
  };
  typedef std::integral_constant<int, 0> Y0;
  typedef std::integral_constant<int, 1> Y1;
  typedef std::integral_constant<int, 2> Y2;
  typedef std::integral_constant<int, 0> W0;
  typedef std::integral_constant<int, 1> W1;
  typedef std::integral_constant<int, 2> W2;
  typedef std::integral_constant<int, 3> W3;
  // a 128-wide diagonal tile runs a loop specialised for the wave, so that
  // every accumulator index is static inside it
  auto diag_loop = [&](auto w_c) {
    if (!ydiag)
      main_loop(std::true_type{}, std::false_type{}, Y0{}, w_c);
    else if (nyb == 1)
      main_loop(std::true_type{}, std::true_type{}, Y1{}, w_c);
    else
      main_loop(std::true_type{}, std::true_type{}, Y2{}, w_c);
  };
  // FP64 off-diagonal tiles of 128: every wave reads its MFMA fragments
  // straight from the panels, kDirectDepth row steps (4 rows each) ahead,
  // with no LDS staging and no workgroup barrier; the two waves that share
  // an operand half meet in the L1 cache.  Same products in the same order
  // as the staged loop (row steps in increasing row order).
  // FP32 panels: the values are loaded as FP32 (half the bytes) and shifted
  // to FP64 right before the MFMAs that use them, so the loads stay
  // kDirectDepth steps ahead
  auto direct_loop = [&]() {
    constexpr int D = kDirectDepth;
    const CVG_GLOBAL PE* za = packed + ca + wm * WT + fc;
    const CVG_GLOBAL PE* zb = packed + cb + wn * WT + fc;
    const int64_t nk = (w.r1 - w.r0) / 4;  // a multiple of 8: items are whole panels
    PE fa[D][NW], fb[D][NW];
    double pa[NW], pb[NW];
#pragma unroll
    for (int a = 0; a < NW; ++a) {
      pa[a] = 0.0;
      pb[a] = 0.0;
      if constexpr (F32P) {
        const CVG_GLOBAL double* pivot = gmem((const double*)pdr.pivot);
        pa[a] = panel_pivot(pivot, ca + wm * WT + fc + 16 * a, K, Kp, M);
        pb[a] = panel_pivot(pivot, cb + wn * WT + fc + 16 * a, K, Kp, M);
      }
    }
    auto load_k = [&](int d, int64_t k) {
      const int64_t off = (w.r0 + 4 * k + fr) * Wp;
#pragma unroll
      for (int a = 0; a < NW; ++a) fa[d][a] = za[off + 16 * a];
#pragma unroll
      for (int b = 0; b < NW; ++b) fb[d][b] = zb[off + 16 * b];
    };
#pragma unroll
    for (int d = 0; d < D; ++d) {
      load_k(d, d < nk ? d : nk - 1);
      __builtin_amdgcn_sched_barrier(0);  // the loop's order: its waits count from it
    }
    // FP32 panels: step k's operands are converted and shifted while step
    // k - 1's MFMAs run (two sets, alternating; D is even)
    static_assert(kDirectDepth % 2 == 0, "operand sets alternate per step");
    double xa[2][NW], xb[2][NW];
    auto convert = [&](int d, int slot) {
#pragma unroll
      for (int a = 0; a < NW; ++a) {
        xa[slot][a] = (double)fa[d][a] - pa[a];
        xb[slot][a] = (double)fb[d][a] - pb[a];
      }
    };
    if constexpr (F32P) convert(0, 0);
    for (int64_t k = 0; k < nk; k += D) {
#pragma unroll
      for (int d = 0; d < D; ++d) {
        if constexpr (F32P) {
#pragma unroll
          for (int a = 0; a < NW; ++a)
#pragma unroll
            for (int b = 0; b < NW; ++b)
              acc[a * NW + b] = mfma_step(xa[d & 1][a], xb[d & 1][b], acc[a * NW + b]);
          convert((d + 1) % D, (d + 1) & 1);  // step k + d + 1 (past the end: unused)
        } else {
#pragma unroll
          for (int a = 0; a < NW; ++a)
#pragma unroll
            for (int b = 0; b < NW; ++b)
              acc[a * NW + b] = mfma_step((double)fa[d][a], (double)fb[d][b], acc[a * NW + b]);
        }
        // the step D ahead (past the end: the last step again, unused),
        // issued here and not moved: its registers are free only now, and
        // it has the next D - 1 steps' MFMAs to arrive
        const int64_t kn = k + d + D;
        load_k(d, kn < nk ? kn : nk - 1);
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  };
  if (!diag) {
    if constexpr (kF64 && kPairs)
      direct_loop();
    else
      main_loop(std::false_type{}, std::false_type{}, Y0{}, W0{});
  } else if constexpr (kPairs) {
    switch (wave) {
      case 0: diag_loop(W0{}); break;
      case 1: diag_loop(W1{}); break;
      case 2: diag_loop(W2{}); break;
      default: diag_loop(W3{}); break;
    }
  } else if (!ydiag) {
    main_loop(std::true_type{}, std::false_type{}, Y0{}, W0{});
  } else {
    main_loop(std::true_type{}, std::true_type{}, Y2{}, W0{});
  }
  if (role == 2) return;
  CVG_GLOBAL double* out = slabs + (int64_t)w.slab * K * (K + M);
  auto value = [&](int i, int e) -> double {
    if constexpr (kF64)
      return acc[i][e];
    else
      return a64[i][e] + (double)acc[i][e];
  };
  if constexpr (kPairs) {
    if (diag) {
      auto store = [&](auto w_c, auto y_c) {
        store_diag_pairs<MODE, decltype(w_c)::value, decltype(y_c)::value>(out, ca, fr, fc, K, M,
                                                                           value);
      };
      auto by_wave = [&](auto y_c) {
        switch (wave) {
          case 0: store(W0{}, y_c); break;
          case 1: store(W1{}, y_c); break;
          case 2: store(W2{}, y_c); break;
          default: store(W3{}, y_c); break;
        }
      };
      if (nyb == 0)
        by_wave(Y0{});
      else if (nyb == 1)
        by_wave(Y1{});
      else
        by_wave(Y2{});
      return;
    }
  }
  store_tile<MODE, BM, NACC>(out, role, xy_tile, ca, xy_tile ? (int64_t)(w.tj - nt) * BM : cb, wm,
                             wn, fr, fc, K, M, value);
}

// ---------------------------------------------------------------------------
// BF16X3 kernel: direct-to-LDS loads into a ring of kStages buffers
// ---------------------------------------------------------------------------
constexpr int kStages = 4;

template <int BM>
struct DmaBuf {
  // [column][32 rows] bf16, swizzled 16-byte chunks (see swz)
  __bf16 ah[BM * 32], al[BM * 32], bh[BM * 32], bl[BM * 32], yh[kYW * 32], yl[kYW * 32];
};

// s_waitcnt with vmcnt = n and lgkmcnt = 0 (expcnt not waited on)
template <int n>
__device__ __forceinline__ void wait_vmcnt_lgkm0() {
  static_assert(n >= 0 && n < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((n & 15) | ((n >> 4) << 14) | (7 << 4));
}

// workgroup barrier that orders memory operations in the compiler but adds
// no wait of its own (the waits are explicit)
__device__ __forceinline__ void barrier_only() { asm volatile("s_barrier" ::: "memory"); }

// one 16-byte direct-to-LDS load per lane: lane l writes dst + 16 l
__device__ __forceinline__ void dma16(const CVG_GLOBAL char* src, __bf16* dst) {
  __builtin_amdgcn_global_load_lds((const CVG_GLOBAL void*)src,
                                   (__attribute__((address_space(3))) void*)dst, 16, 0, 0);
}

template <int BM>
__global__ __launch_bounds__(kThreads) void gram_bf16_kernel(const ProbDesc* __restrict__ pds,
                                                             const GramWork* __restrict__ work,
                                                             const int32_t* __restrict__ xcd) {
  constexpr int MODE = CVGRAM_MODE_BF16X3;
  constexpr int WT = BM / 2, NW = WT / 16, NY = BM / 16;
  constexpr int NACC = NW * NW > 2 * NY ? NW * NW : 2 * NY;
  constexpr int IA = BM / 64;  // 1 KB direct loads per wave per array per stage
  __shared__ __attribute__((aligned(1024))) DmaBuf<BM> sb0, sb1, sb2, sb3;

  const int x = (int)(blockIdx.x % kXcds);
  const int64_t item = (int64_t)xcd[x] + blockIdx.x / kXcds;
  if (item >= xcd[x + 1]) return;
  const GramWork w = work[item];
  const ProbDesc& pdr = pds[w.prob];
  const int64_t Wp = pdr.Wp, Kp = pdr.Kp, K = pdr.K, M = pdr.M;
  const int32_t nt = pdr.nt;
  const CVG_GLOBAL char* const Zh = gmem((const char*)pdr.packed);
  const CVG_GLOBAL char* const Zl = gmem((const char*)pdr.packed_lo);
  CVG_GLOBAL double* const slabs = gmem(pdr.slabs);
  const bool xy_diag = pdr.xy_diag != 0;
  const int t = threadIdx.x, lane = t & 63;
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const int wm = wave >> 1, wn = wave & 1;
  const int fr = lane >> 4, fc = lane & 15;

  const bool xy_tile = w.tj >= nt;
  const bool diag = !xy_tile && w.ti == w.tj;
  const int64_t ca = (int64_t)w.ti * BM;
  const int64_t cb = xy_tile ? Kp + (int64_t)(w.tj - nt) * BM : (int64_t)w.tj * BM;
  const bool ydiag = diag && xy_diag;
  const int role = (diag && wm == 1 && wn == 0) ? (ydiag ? 1 : 2) : 0;

  // byte offsets: source chunk of this lane inside a 1 KB block of 16
  // columns (a permutation of the block's chunks: the loads stay coalesced),
  // and this lane's fragment chunk inside a buffer
  const int lsrc = (lane >> 2) * 64 + (((lane & 3) ^ swz(lane >> 2)) << 4);
  const int lfo = fc * 64 + ((fr ^ swz(fc)) << 4);

  float4_t acc[NACC];
  double a64[NACC][4];
#pragma unroll
  for (int i = 0; i < NACC; ++i) {
    acc[i] = float4_t{0, 0, 0, 0};
#pragma unroll
    for (int e = 0; e < 4; ++e) a64[i][e] = 0.0;
  }
  const int64_t nst = (w.r1 - w.r0) / 32;
  const int64_t p0 = w.r0 / 32;  // first panel
  int since = 0;

  auto flush = [&]() {
    since += 32;
    if (since >= kFlushRowsBf16) {
      since = 0;
#pragma unroll
      for (int i = 0; i < NACC; ++i) {
#pragma unroll
        for (int e = 0; e < 4; ++e) a64[i][e] += (double)acc[i][e];
        acc[i] = float4_t{0, 0, 0, 0};
      }
    }
  };

  // The loop is instantiated per tile kind (B is A; K x M block in the
  // tile) and per wave role, so each wave's loop holds only its own
  // fragment registers; every instance runs the same sequence of barriers.
  auto main_loop = [&](auto diag_c, auto ydiag_c, auto role_c) {
    constexpr bool DG = decltype(diag_c)::value;
    constexpr bool YD = decltype(ydiag_c)::value;
    constexpr int R = decltype(role_c)::value;
    constexpr int FA = R == 1 ? NY : NW, FB = R == 1 ? 2 : NW;
    // direct loads per wave per stage (all waves issue the same number)
    constexpr int L = IA * (DG ? 2 : 4) + (YD ? 1 : 0);
    // stage s (clamped to the last one) into buffer b
    auto issue = [&](DmaBuf<BM>& b, int64_t s) {
      const int64_t panel = (p0 + (s < nst ? s : nst - 1)) * Wp;
      const CVG_GLOBAL char* ah = Zh + (panel + ca) * 64 + lsrc;
      const CVG_GLOBAL char* al = Zl + (panel + ca) * 64 + lsrc;
#pragma unroll
      for (int i = 0; i < IA; ++i) {
        const int blk = wave * IA + i;
        dma16(ah + blk * 1024, b.ah + blk * 512);
        dma16(al + blk * 1024, b.al + blk * 512);
      }
      if constexpr (!DG) {
        const CVG_GLOBAL char* bh = Zh + (panel + cb) * 64 + lsrc;
        const CVG_GLOBAL char* bl = Zl + (panel + cb) * 64 + lsrc;
#pragma unroll
        for (int i = 0; i < IA; ++i) {
          const int blk = wave * IA + i;
          dma16(bh + blk * 1024, b.bh + blk * 512);
          dma16(bl + blk * 1024, b.bl + blk * 512);
        }
      }
      if constexpr (YD) {
        // waves 0, 1: hi columns 0-15, 16-31; waves 2, 3: lo
        const CVG_GLOBAL char* src = (wave < 2 ? Zh : Zl) + (panel + Kp) * 64 + lsrc;
        dma16(src + (wave & 1) * 1024, (wave < 2 ? b.yh : b.yl) + (wave & 1) * 512);
      }
    };
    typedef Frags<FA, FB> F;
    auto load_frags = [&](F& f, const DmaBuf<BM>& b) {
      if constexpr (R == 0)
        f.load(b.ah, b.al, wm * WT, DG ? b.ah : b.bh, DG ? b.al : b.bl, wn * WT, lfo);
      else if constexpr (R == 1)
        f.load(b.ah, b.al, 0, b.yh, b.yl, 0, lfo);
    };
    // Step s: the fragments of stage s are in `cur`.  The first product pass
    // runs; then the wait and the barrier make stage s + 1 visible in every
    // wave and end every wave's reads of stage s's buffer, which receives
    // stage s + 4; stage s + 1's fragments are read into `nxt` while the
    // other two passes of stage s run.  Every step issues its loads, also
    // past the end of a partial last round (re-loading the last stage): the
    // compiler's wait bookkeeping for direct-to-LDS loads then stays exact,
    // and no read of one buffer waits for loads into the others.
    auto step = [&](int64_t s, const DmaBuf<BM>& next_buf, DmaBuf<BM>& target, F& cur, F& nxt) {
      if constexpr (R != 2) {
        if (s < nst) mfma_pass<0>(cur, acc);
      }
      wait_vmcnt_lgkm0<2 * L>();
      barrier_only();
      issue(target, s + 4);
      if constexpr (R != 2) {
        if (s + 1 < nst) load_frags(nxt, next_buf);
        if (s < nst) {
          mfma_pass<1>(cur, acc);
          mfma_pass<2>(cur, acc);
          flush();
        }
      }
    };
    F f0, f1;
    issue(sb0, 0);
    issue(sb1, 1);
    issue(sb2, 2);
    issue(sb3, 3);
    wait_vmcnt_lgkm0<3 * L>();
    barrier_only();
    if constexpr (R != 2) load_frags(f0, sb0);
    for (int64_t s = 0; s < nst; s += kStages) {
      step(s, sb1, sb0, f0, f1);
      step(s + 1, sb2, sb1, f1, f0);
      step(s + 2, sb3, sb2, f0, f1);
      step(s + 3, sb0, sb3, f1, f0);
    }
    wait_vmcnt_lgkm0<0>();  // the loads past the end
  };
  typedef std::integral_constant<int, 0> R0;
  typedef std::integral_constant<int, 1> R1;
  typedef std::integral_constant<int, 2> R2;
  if (!diag) {
    main_loop(std::false_type{}, std::false_type{}, R0{});
  } else if (ydiag) {
    if (role == 0)
      main_loop(std::true_type{}, std::true_type{}, R0{});
    else
      main_loop(std::true_type{}, std::true_type{}, R1{});
  } else {
    if (role == 0)
      main_loop(std::true_type{}, std::false_type{}, R0{});
    else
      main_loop(std::true_type{}, std::false_type{}, R2{});
  }
  if (role == 2) return;
  CVG_GLOBAL double* out = slabs + (int64_t)w.slab * K * (K + M);
  auto value = [&](int i, int e) -> double { return a64[i][e] + (double)acc[i][e]; };
  store_tile<MODE, BM, NACC>(out, role, xy_tile, ca, xy_tile ? (int64_t)(w.tj - nt) * BM : cb, wm,
                             wn, fr, fc, K, M, value);
}

// ---------------------------------------------------------------------------
// BF16X3 wide kernel: 256 x 128 workgroup tiles (tile code 256)
// ---------------------------------------------------------------------------
// Item (ti, tj): A = packed columns [256 ti, 256 ti + 256) (two 128-wide
// tiles of the K x K block stacked), B = the 128 columns of B block tj
// (tj < nt: X columns [128 tj, +128); tj >= nt: Y columns [128 (tj - nt),
// +128)).  Items exist for tj >= 2 ti.  Pairs with tj = 2 ti or 2 ti + 1
// straddle the diagonal: their B columns lie inside A's (no B loads); in
// tj = 2 ti the lower half of A is below the diagonal, and the waves on it
// compute the 256 x 32 K-by-M block instead (M <= 32) or idle.
// Eight waves, two per SIMD: wave (wm, wn), wm = 0..3, wn = 0..1, computes A
// columns 64 wm .. + 64 against B columns 64 wn .. + 64 as 2 x 2 output
// blocks of 32 x 32 (v_mfma_f32_32x32x16_bf16); on a diagonal pair with
// tj = 2 ti the waves wm = 2, 3 take 64 rows each of the K-by-M block.  While
// one wave of a SIMD waits on LDS or the stage barrier, the other issues its
// MFMAs (with one 128 x 64 wave tile per SIMD the kernel ran 6 % slower).
// Per 32-row stage each wave reads 16 KB of fragments from LDS, in four
// parts around the three products (lo(A) hi(B), hi(A) hi(B), hi(A) lo(B)):
// a part is re-read for the next stage as soon as the product that used it
// last is issued, so one register set serves.  The ring has three stages of
// 52 KB; the barrier at each stage frees the previous stage's buffer for the
// stage three ahead.  Per panel byte loaded the 256 x 128 workgroup tile
// does 4/3 the MFMA work of a 128 x 128 one.
// Accumulation: FP32 MFMA accumulators added into FP32 running totals every
// 512 rows (VALU adds round to nearest) -- the totals take the place of
// FP64 copies, which would leave room for one wave per SIMD only.  A block
// of 512 rows is 96 accumulating MFMAs; the accumulator's rounding is about
// half an FP32 ulp per step and does not average out on sums of positive
// products, so a block's worst relative error is about 48 ulp (3e-6).
constexpr int kWStages = 3;
constexpr int kWFlushRows = 512;
struct DmaBufW {
  // [column][32 rows] bf16, swizzled 16-byte chunks (see swz)
  __bf16 ah[256 * 32], al[256 * 32], bh[128 * 32], bl[128 * 32], yh[kYW * 32], yl[kYW * 32];
};

constexpr int kThreads8 = 512;  // eight waves
__global__ __launch_bounds__(kThreads8) void gram_bf16_wide_kernel(
    const ProbDesc* __restrict__ pds, const GramWork* __restrict__ work,
    const int32_t* __restrict__ xcd) {
  __shared__ __attribute__((aligned(1024))) DmaBufW sb0, sb1, sb2;
  const int x = (int)(blockIdx.x % kXcds);
  const int64_t item = (int64_t)xcd[x] + blockIdx.x / kXcds;
  if (item >= xcd[x + 1]) return;
  const GramWork w = work[item];
  const ProbDesc& pdr = pds[w.prob];
  const int64_t Wp = pdr.Wp, Kp = pdr.Kp, K = pdr.K, M = pdr.M;
  const int32_t nt = pdr.nt;  // B blocks of 128 along X's columns
  const CVG_GLOBAL char* const Zh = gmem((const char*)pdr.packed);
  const CVG_GLOBAL char* const Zl = gmem((const char*)pdr.packed_lo);
  CVG_GLOBAL double* const slabs = gmem(pdr.slabs);
  const bool xy_diag = pdr.xy_diag != 0;
  const int t = threadIdx.x, lane = t & 63;
  const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const int wm = wave >> 1, wn = wave & 1;

  const bool xy_tile = w.tj >= nt;
  const int dq = w.tj - 2 * w.ti;               // 0 or 1 on the diagonal pairs
  const bool diag = !xy_tile && (dq == 0 || dq == 1);
  const int64_t ca = (int64_t)w.ti * 256;
  const int64_t cb = xy_tile ? Kp + (int64_t)(w.tj - nt) * 128 : (int64_t)w.tj * 128;
  const bool ydiag = diag && dq == 0 && xy_diag;
  // 0: 64 x 64 sub-tile; 1: 64 x 32 of the K-by-M block; 2: idle
  const int role = (diag && dq == 0 && wm >= 2) ? (ydiag ? 1 : 2) : 0;

  const int lsrc = (lane >> 2) * 64 + (((lane & 3) ^ swz(lane >> 2)) << 4);
  const int lc = lane & 31, lh = lane >> 5;
  const int lfo[2] = {lc * 64 + ((lh ^ swz(lc)) << 4), lc * 64 + (((2 + lh) ^ swz(lc)) << 4)};

  constexpr int NACC = 4;
  float16_t acc[NACC], tot[NACC];
#pragma unroll
  for (int i = 0; i < NACC; ++i)
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      acc[i][e] = 0.f;
      tot[i][e] = 0.f;
    }
  const int64_t nst = (w.r1 - w.r0) / 32;
  const int64_t p0 = w.r0 / 32;  // first panel
  int since = 0;
  // the Y block's four 1 KB loads (hi and lo, two column halves each) go to
  // waves 0 .. 3
  const bool yload = wave < 4;

  auto main_loop = [&](auto dg_c, auto yd_c, auto role_c) {
    constexpr bool DG = decltype(dg_c)::value;   // B inside A
    constexpr bool YD = decltype(yd_c)::value;   // K x M block in this tile
    constexpr int R = decltype(role_c)::value;
    constexpr int FA = 2, FB = R == 1 ? 1 : 2;
    constexpr int NA = R == 2 ? 0 : FA;
    // direct loads per wave per stage (waves 0 .. 3 one more with the Y block)
    constexpr int L = 4 + (DG ? 0 : 2);
    const int bcol = (DG ? dq * 128 : 0) + wn * 64;
    auto wait_one_stage = [&]() {
      if (YD && yload)
        wait_vmcnt_lgkm0<L + 1>();
      else
        wait_vmcnt_lgkm0<L>();
    };
    auto issue = [&](DmaBufW& b, int64_t s) {
      const int64_t panel = (p0 + (s < nst ? s : nst - 1)) * Wp;
      const CVG_GLOBAL char* ah = Zh + (panel + ca) * 64 + lsrc;
      const CVG_GLOBAL char* al = Zl + (panel + ca) * 64 + lsrc;
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int blk = wave * 2 + i;
        dma16(ah + blk * 1024, b.ah + blk * 512);
        dma16(al + blk * 1024, b.al + blk * 512);
      }
      if constexpr (!DG) {
        const CVG_GLOBAL char* bh = Zh + (panel + cb) * 64 + lsrc;
        const CVG_GLOBAL char* bl = Zl + (panel + cb) * 64 + lsrc;
        dma16(bh + wave * 1024, b.bh + wave * 512);
        dma16(bl + wave * 1024, b.bl + wave * 512);
      }
      if constexpr (YD) {
        // waves 0, 1: hi columns 0-15, 16-31; waves 2, 3: lo
        if (yload) {
          const CVG_GLOBAL char* src = (wave < 2 ? Zh : Zl) + (panel + Kp) * 64 + lsrc;
          dma16(src + (wave & 1) * 1024, (wave < 2 ? b.yh : b.yl) + (wave & 1) * 512);
        }
      }
    };
    bf16x8_t fal[NA > 0 ? NA : 1][2], fah[NA > 0 ? NA : 1][2], fbh[FB][2], fbl[FB][2];
    const int acol = R == 1 ? (2 * (wm - 2) + wn) * 64 : wm * 64;
    auto rd = [&](const __bf16* base, int col0, int ks) -> bf16x8_t {
      return *(const bf16x8_t*)((const char*)base + col0 * 64 + lfo[ks]);
    };
    auto load_al = [&](const DmaBufW& b) {
#pragma unroll
      for (int a = 0; a < NA; ++a)
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) fal[a][ks] = rd(b.al, acol + a * 32, ks);
    };
    auto load_ah = [&](const DmaBufW& b) {
#pragma unroll
      for (int a = 0; a < NA; ++a)
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) fah[a][ks] = rd(b.ah, acol + a * 32, ks);
    };
    auto load_bh = [&](const DmaBufW& b) {
#pragma unroll
      for (int c = 0; c < FB; ++c)
#pragma unroll
        for (int ks = 0; ks < 2; ++ks)
          fbh[c][ks] = R == 1 ? rd(b.yh, c * 32, ks) : rd(DG ? b.ah : b.bh, bcol + c * 32, ks);
    };
    auto load_bl = [&](const DmaBufW& b) {
#pragma unroll
      for (int c = 0; c < FB; ++c)
#pragma unroll
        for (int ks = 0; ks < 2; ++ks)
          fbl[c][ks] = R == 1 ? rd(b.yl, c * 32, ks) : rd(DG ? b.al : b.bl, bcol + c * 32, ks);
    };
    auto product = [&](const bf16x8_t (&fa)[NA > 0 ? NA : 1][2], const bf16x8_t (&fb)[FB][2]) {
#pragma unroll
      for (int ks = 0; ks < 2; ++ks)
#pragma unroll
        for (int a = 0; a < NA; ++a)
#pragma unroll
          for (int c = 0; c < FB; ++c)
            acc[a * FB + c] =
                __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[a][ks], fb[c][ks], acc[a * FB + c], 0, 0, 0);
    };
    auto flush = [&]() {
      since += 32;
      if (since >= kWFlushRows) {
        since = 0;
#pragma unroll
        for (int i = 0; i < NA * FB; ++i)
#pragma unroll
          for (int e = 0; e < 16; ++e) {
            tot[i][e] += acc[i][e];
            acc[i][e] = 0.f;
          }
      }
    };
    // Stage s: lo(A) and hi(B) of stage s are in registers (read during
    // stage s - 1).  Its hi(A) and lo(B) are read, then the wait and the
    // barrier: every wave's reads of `cur` are done (it receives stage
    // s + 3) and stage s + 1 has landed in `next`.  The products follow with
    // no further wait -- all their operands were complete at the barrier --
    // while the next stage's parts are read into the registers each product
    // frees: lo(A) after the first, hi(B) after the second.  The last
    // product of stage s - 1 is still running on the matrix cores across the
    // reads and the barrier.  Scheduling barriers keep this order.  The reads
    // run also past the end (the buffer holds a re-loaded stage).
    auto step = [&](int64_t s, DmaBufW& cur, const DmaBufW& next) {
      if constexpr (R != 2) {
        load_ah(cur);
        load_bl(cur);
      }
      wait_one_stage();
      barrier_only();
      issue(cur, s + kWStages);
      if constexpr (R != 2) {
        __builtin_amdgcn_sched_barrier(0);
        if (s < nst) product(fal, fbh);
        __builtin_amdgcn_sched_barrier(0);
        load_al(next);
        __builtin_amdgcn_sched_barrier(0);
        if (s < nst) product(fah, fbh);
        __builtin_amdgcn_sched_barrier(0);
        load_bh(next);
        __builtin_amdgcn_sched_barrier(0);
        if (s < nst) {
          product(fah, fbl);
          flush();
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    };
    issue(sb0, 0);
    issue(sb1, 1);
    issue(sb2, 2);
    if (YD && yload)
      wait_vmcnt_lgkm0<2 * (L + 1)>();
    else
      wait_vmcnt_lgkm0<2 * L>();
    barrier_only();
    if constexpr (R != 2) {
      load_al(sb0);
      load_bh(sb0);
    }
    for (int64_t s = 0; s < nst; s += kWStages) {
      step(s, sb0, sb1);
      step(s + 1, sb1, sb2);
      step(s + 2, sb2, sb0);
    }
    wait_vmcnt_lgkm0<0>();  // the loads past the end
  };
  typedef std::integral_constant<int, 0> R0;
  typedef std::integral_constant<int, 1> R1;
  typedef std::integral_constant<int, 2> R2;
  if (!diag) {
    main_loop(std::false_type{}, std::false_type{}, R0{});
  } else if (ydiag) {
    if (role == 0)
      main_loop(std::true_type{}, std::true_type{}, R0{});
    else
      main_loop(std::true_type{}, std::true_type{}, R1{});
  } else {
    if (role == 0)
      main_loop(std::true_type{}, std::false_type{}, R0{});
    else
      main_loop(std::true_type{}, std::false_type{}, R2{});
  }
  if (role == 2) return;
  CVG_GLOBAL double* out = slabs + (int64_t)w.slab * K * (K + M);
  const int64_t W = K + M;
  if (role == 0) {
    const int64_t r0 = ca + wm * 64;
    const int64_t c0 = (xy_tile ? (int64_t)(w.tj - nt) * 128 : cb) + wn * 64;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const int64_t row = r0 + a * 32 + 8 * (e >> 2) + 4 * lh + (e & 3);
          const int64_t cl = c0 + b * 32 + lc;
          const double v = (double)tot[a * 2 + b][e] + (double)acc[a * 2 + b][e];
          if (row >= K) continue;
          if (!xy_tile) {
            if (cl < K) out[row * W + cl] = v;
          } else if (cl < M) {
            out[row * W + K + cl] = v;
          }
        }
  } else {
    const int64_t r0 = ca + (2 * (wm - 2) + wn) * 64;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int64_t row = r0 + a * 32 + 8 * (e >> 2) + 4 * lh + (e & 3);
        if (row < K && lc < M) out[row * W + K + lc] = (double)tot[a][e] + (double)acc[a][e];
      }
  }
}

template <int MODE>
void launch_mode(bool panel_f32, int tile, const ProbDesc* pd, const GramWork* work,
                 const int32_t* xcd, int64_t per_xcd, hipStream_t s) {
  const unsigned grid = (unsigned)(kXcds * per_xcd);
  if constexpr (MODE == CVGRAM_MODE_BF16X3) {
    if (tile == 64)
      gram_bf16_kernel<64><<<grid, kThreads, 0, s>>>(pd, work, xcd);
    else if (tile == 128)
      gram_bf16_kernel<128><<<grid, kThreads, 0, s>>>(pd, work, xcd);
    else
      gram_bf16_wide_kernel<<<grid, kThreads8, 0, s>>>(pd, work, xcd);
  } else if constexpr (MODE == CVGRAM_MODE_FP64) {
    if (panel_f32) {
      if (tile == 64)
        gram_kernel<MODE, 64, true><<<grid, kThreads, 0, s>>>(pd, work, xcd);
      else
        gram_kernel<MODE, 128, true><<<grid, kThreads, 0, s>>>(pd, work, xcd);
    } else {
      if (tile == 64)
        gram_kernel<MODE, 64, false><<<grid, kThreads, 0, s>>>(pd, work, xcd);
      else
        gram_kernel<MODE, 128, false><<<grid, kThreads, 0, s>>>(pd, work, xcd);
    }
  } else {
    if (tile == 64)
      gram_kernel<MODE, 64, false><<<grid, kThreads, 0, s>>>(pd, work, xcd);
    else
      gram_kernel<MODE, 128, false><<<grid, kThreads, 0, s>>>(pd, work, xcd);
  }
  CVG_LAUNCH_CHECK();
}

}  // namespace

void launch_gram(cvgram_mode mode, bool panel_f32, int tile, const ProbDesc* pd,
                 const GramWork* work, const int32_t* xcd, int64_t per_xcd, hipStream_t s) {
  if (per_xcd <= 0) return;
  if (mode == CVGRAM_MODE_FP64)
    launch_mode<CVGRAM_MODE_FP64>(panel_f32, tile, pd, work, xcd, per_xcd, s);
  else if (mode == CVGRAM_MODE_FP32)
    launch_mode<CVGRAM_MODE_FP32>(false, tile, pd, work, xcd, per_xcd, s);
  else
    launch_mode<CVGRAM_MODE_BF16X3>(false, tile, pd, work, xcd, per_xcd, s);
}

}  // namespace cvg
