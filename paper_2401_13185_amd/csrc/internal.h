// Internal declarations shared by the HIP translation units of libcvgram.
//
// Every device stage works on a list of problems described by ProbDesc
// records in device memory; a single cvgram_t handle is a batch of one.  The
// work of every launch is a flat list of items that name their problem, so
// problems of different N, K, M and P share one launch.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/cvgram.h"

namespace cvg {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);

struct Fail {
  cvgram_status st;
};

#define CVG_HIP(call)                                                              \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess) {                                                        \
      ::cvg::set_error(std::string(#call) + ": " + hipGetErrorString(e_));         \
      throw ::cvg::Fail{e_ == hipErrorOutOfMemory ? CVGRAM_ENOMEM : CVGRAM_EDEVICE}; \
    }                                                                              \
  } while (0)

#define CVG_LAUNCH_CHECK() CVG_HIP(hipGetLastError())

// ---------------------------------------------------------------------------
// global-memory pointers
// ---------------------------------------------------------------------------
// A pointer read from a descriptor is generic (flat) to the compiler, and a
// flat load or store also counts against the LDS wait counter: every wait for
// an LDS read would then wait for the global traffic in flight as well.
// Kernels re-type such pointers as global before use.
#define CVG_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ CVG_GLOBAL T* gmem(T* p) {
  return (CVG_GLOBAL T*)p;
}

// ---------------------------------------------------------------------------
// layout constants
// ---------------------------------------------------------------------------
// Packed row space: every fold's rows, in fold order, padded with zero rows
// to a multiple of kPanelRows.
constexpr int kPanelRows = 32;
// Packed column space: X columns [0, K), zeros up to Kp (a multiple of the
// problem's Gram tile), Y columns [Kp, Kp + M), zeros up to Wp.  X^T Y is
// computed inside diagonal tiles when M <= kYDiagCols.
constexpr int kYDiagCols = 32;
// pack pass: a workgroup packs kPackCols columns of 32-row panels of one
// chunk of at most kMaxChunkRows rows (a multiple of kPanelRows)
constexpr int kPackCols = 64;
constexpr int kMaxChunkRows = 1024;
// accelerator dies (XCDs) of the part; consecutive workgroup ids go to
// different XCDs round-robin, each XCD with its own L2
constexpr int kXcds = 8;
// Gram tile widths, one launch each: 64, 128, and 256 (BF16X3 only: a
// 256 x 128 tile, two 128-wide row blocks over one 128-wide column block)
constexpr int kWidths = 3;
constexpr int kWidth[kWidths] = {64, 128, 256};
inline int width_index(int tile) { return tile == 64 ? 0 : (tile == 128 ? 1 : 2); }
// correction tiles
constexpr int kCorrTile = 32;
// slab reduction: entries of the K x W slab per workgroup (two per thread)
constexpr int kReduceElems = 512;
// fold totals: folds per partial range
constexpr int kFoldRange = 256;

// ---------------------------------------------------------------------------
// device-side description of one problem
// ---------------------------------------------------------------------------
struct ProbDesc {
  const void* X;        // caller's X (N x K) and Y (N x M), row-major
  const void* Y;
  int64_t N, K, M, W;   // W = K + M
  int64_t Kp, Wp, Np;   // packed widths / padded row count
  int32_t P;            // folds
  int32_t tile;         // Gram tile width (64, 128 or 256)
  int32_t nt;           // Gram tile columns along X's columns (Kp / 128 for tile 256)
  int32_t xy_diag;      // X^T Y inside diagonal tiles
  int32_t ddof;
  int32_t x_vec;        // X rows 16-byte aligned and K % 4 == 0
  int32_t mode;         // cvgram_mode: element format of the packed panels
  // FP64 mode with FP32 input (and K up to 2048): the panels hold the
  // input's FP32 values as they are (padding rows: the column's pivot, an
  // FP32 value; padding columns: 0 with pivot 0), and every reader shifts
  // them in FP64, z' = (double)x - c, an exact subtraction of two FP32 values
  int32_t panel_f32;
  // Fold path.  0 (grouped): every fold padded to whole panels, one slab set
  // per fold holding G'_p.  1 (fused, for many small folds): rows packed
  // without padding between folds, the slabs hold row splits of the full
  // Gram only, and each fold's G'_p is formed inside the corrections from
  // the fold's packed rows.
  int32_t fused;
  int32_t n_slabs;
  const int32_t* perm;       // [N]
  const int64_t* offsets;    // [P+1]
  const int64_t* poff;       // [P+1] first packed row of each fold
  double* pivot;             // [W]
  void* packed;              // packed panels (FP64 / FP32 / bf16 hi)
  void* packed_lo;           // bf16 lo panel
  double* part;              // [4][n_chunks][W] per-chunk sum, sumsq, min, max
  int64_t n_chunks;
  const int32_t* chunk_begin;  // [P+1]
  double* fold;              // [4][P][W] per-fold sum, sumsq, min, max
  double* tot;               // [8][W] totals and extrema over folds
  double* tot_part;          // [R][8][W] the same per range of kFoldRange folds
  int32_t n_franges;         // R
  double* tr_sum;            // [P][W] shifted training sums
  double* tr_mean;           // [P][W] shifted training means
  double* tr_std;            // [P][W] training deviations (1 if constant)
  double* tr_mu;             // [P][W] unshifted training means
  uint8_t* tr_const;         // [P][W]
  int64_t* ntrain;           // [P]
  double* slabs;             // [S][K][W] FP64 Gram partials; fold sums in place
  const int32_t* slab_begin;  // [P+1]
  double* G;                 // [K][W]
  const int32_t* ctiles;     // correction tiles (bi, bj): X^T X first, then X^T Y
  int32_t n_ctiles_xx, n_ctiles_xy;
};

// Where the correction writes: per class a base pointer for fold p_begin
// (NULL = skip) and the element stride between consecutive folds.
struct OutDesc {
  void* xx[CVGRAM_XTX_CLASSES];
  void* xy[CVGRAM_XTY_CLASSES];
  int64_t fold_stride_xx;
  int64_t fold_stride_xy;
  int32_t p_begin;
  // leakage comparison (0: off).  1: the combination (lcx, lsx, lcy, lsy)
  // with statistics of all rows; 2: Lindgren et al.'s centred products.
  // One output pair, in xx[0] and xy[0].
  int32_t leak;
  int32_t lcx, lsx, lcy, lsy;
};

// ---------------------------------------------------------------------------
// work items
// ---------------------------------------------------------------------------
// (problem, a, b): the meaning of a and b depends on the launch
struct Item {
  int32_t prob;
  int32_t a;
  int32_t b;
};

// Packed rows [d0, d1) of one fold (whole panels); packed row d holds the
// permuted row src0 + (d - d0) when that is below src1, else zeros.  `chunk`
// is the chunk's index inside its problem (row of the partial statistics).
struct PackChunk {
  int32_t prob;
  int32_t chunk;
  int64_t d0, d1, src0, src1;
};

// One unit of the grouped Gram launch: output tile (ti, tj) of one problem,
// restricted to packed rows [r0, r1) of one fold, written to slab `slab`.
struct GramWork {
  int32_t prob;
  int32_t slab;
  int32_t ti;
  int32_t tj;
  int64_t r0;
  int64_t r1;
};

// ---------------------------------------------------------------------------
// launches (pointers are device pointers unless named *_host)
// ---------------------------------------------------------------------------
// partition.hip (one problem at a time, at plan time)
void launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
// info[0] = INT32_MAX, info[1] = INT32_MIN, info[2 .. n) = 0
void launch_count_init(int32_t* info, int64_t n, hipStream_t s);
// minimum, maximum and the counts of labels below kCountLabels (starting
// values from launch_count_init), plus the first radix pass's histogram in
// hist (radix_hist_entries(N) entries)
constexpr int kCountLabels = 4096;
void launch_label_count(const int32_t* fold, int64_t N, int32_t* info, int32_t* counts,
                        int32_t* hist, hipStream_t s);
// stable sort of the labels in [0, 2^bits); hist as left by launch_label_count
// on the same labels when hist_ready (else the first pass recounts it),
// counts = its label counts (used when bits <= 8)
void radix_partition(const int32_t* fold, int64_t N, int bits, const int32_t* counts,
                     int32_t* keys_a, int32_t* keys_b, int32_t* perm, int32_t* perm_tmp,
                     int32_t* hist, bool hist_ready, const int32_t** sorted_keys, hipStream_t s);
int64_t radix_hist_entries(int64_t N);
void launch_fold_offsets(const int32_t* sorted_keys, int64_t N, int32_t P, int64_t* offsets,
                         int32_t* flag, hipStream_t s);

// pack.hip
// items: (prob, block of 64 columns of [X | Y], -)
void launch_pivot(cvgram_dtype dt, bool round_f32, const ProbDesc* pd, const Item* items,
                  int64_t n_items, hipStream_t s);
// the same pivots for one problem from plain arguments (Y may be null when M = 0)
void launch_pivot_direct(cvgram_dtype dt, bool round_f32, const void* X, const void* Y,
                         int64_t N, int64_t K, int64_t M, double* out, hipStream_t s);
void launch_pack(cvgram_mode mode, cvgram_dtype dt, const ProbDesc* pd, const PackChunk* chunks,
                 int64_t n_chunks, int32_t max_col_blocks, hipStream_t s);

// stats.hip
// fold_items: (prob, fold, -); colblock_items: (prob, block of 64 columns, -)
void launch_stats_reduce(const ProbDesc* pd, const Item* fold_items, int64_t n_items,
                         int32_t max_col_blocks64, hipStream_t s);
// fused-path problems: per-fold sums straight from the fold's rows of X, Y;
// items (prob, first fold, end fold)
void launch_fold_sums_rows(cvgram_dtype dt, const ProbDesc* pd, const Item* fold_items,
                           int64_t n_items, int32_t max_col_blocks64, hipStream_t s);
// range_items: (prob, block of 64 columns, range of kFoldRange folds)
void launch_fold_totals(const ProbDesc* pd, const Item* range_items, int64_t n_range_items,
                        const Item* colblock_items, int64_t n_items, hipStream_t s);
void launch_train_stats(const ProbDesc* pd, const Item* fold_items, int64_t n_items,
                        int32_t max_col_blocks256, hipStream_t s);
void launch_fold_stats(const double* tr_mu, const double* tr_std, int32_t p, int64_t K,
                       int64_t M, double* mx, double* sx, double* my, double* sy, hipStream_t s);

// gram.hip
// xcd: kXcds + 1 offsets into work, the item range of each XCD; workgroup b
// runs item xcd[b % kXcds] + b / kXcds of its range (per_xcd = the largest
// range, so the grid is kXcds * per_xcd workgroups).  panel_f32: FP64 mode
// on FP32 panels (ProbDesc::panel_f32, the same for every problem).
void launch_gram(cvgram_mode mode, bool panel_f32, int tile, const ProbDesc* pd,
                 const GramWork* work, const int32_t* xcd, int64_t per_xcd, hipStream_t s);

// correct.hip
// items: (prob, block of 256 entries of K x W, -)
void launch_reduce_slabs(const ProbDesc* pd, const Item* items, int64_t n_items, hipStream_t s);
// one problem: folds [out.p_begin, out.p_begin + n_folds), all correction tiles
void launch_correct_single(const ProbDesc* pd, int32_t prob, int32_t n_tiles, const OutDesc& out,
                           int32_t n_folds, bool out_f64, hipStream_t s);
// many problems: items (prob, fold, tile); outputs per problem in outs[prob]
void launch_correct_batch(const ProbDesc* pd, const OutDesc* outs, const Item* items,
                          int64_t n_items, bool out_f64, hipStream_t s);

// solve.hip: B = (xtx_f + lambda_l I)^{-1} xty_f for every (fold f, lambda l),
// matrices p-major, into B: [n_folds n_lambda][K][M].  Workspaces, with
// Kp = ridge_padded_k(K), Ma = ridge_aug_rows(M) and Mp the multiple of 32
// at or above M: A [n_folds n_lambda][Kp + Ma][Kp] (the matrix, then R^T),
// R [n_folds n_lambda][Kp][Mp] (only where !ridge_solve_on_matrix_cores),
// Linv: n_folds n_lambda Kp 96 doubles (the 64 x 64 inverses of the diagonal
// blocks of the factor, then their 32 x 32 diagonal blocks);
// flags: [n_folds n_lambda] (set on a non-positive pivot; zeroed by the
// factorisation itself).  Up to kRidgeLambdaArgs penalties travel by value
// in lam (lambdas_dev null); more come from the device array lambdas_dev.
inline int64_t ridge_padded_k(int64_t K) { return (K + 63) / 64 * 64; }
inline int64_t ridge_aug_rows(int64_t M) { return (M + 63) / 64 * 64; }
// the backward substitution runs on the matrix cores, with the right-hand
// sides in registers, up to Kp = 512; R is read and written only beyond
inline bool ridge_solve_on_matrix_cores(int64_t Kp, int64_t M) { return M > 0 && Kp <= 512; }
constexpr int kRidgeLambdaArgs = 64;
struct RidgeLambdas {
  double v[kRidgeLambdaArgs];
};
void ridge_solve(const double* xtx, const double* xty, const RidgeLambdas& lam,
                 const double* lambdas_dev, int32_t n_folds, int32_t n_lambda, int64_t K,
                 int64_t M, double* A, double* R, double* Linv, int32_t* flags, double* B,
                 hipStream_t s);

}  // namespace cvg
