// Internal declarations shared by the HIP translation units of libcvgram.
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
// device workspace owned by a handle
// ---------------------------------------------------------------------------
struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
};

// One unit of the grouped Gram launch: an output tile (ti, tj) of
// Z'^T Z' restricted to the rows perm[r0, r1) of fold p, written to slab `slab`.
struct GramWork {
  int32_t p;
  int32_t slab;
  int32_t ti;
  int32_t tj;
  int64_t r0;
  int64_t r1;
};

// Packed row space: every fold's rows, in fold order, padded with zero rows
// to a multiple of kPanelRows.  A pack chunk covers packed rows [d0, d1) of
// one fold (a whole number of panels); packed row d holds the permuted row
// src0 + (d - d0) when that is below src1, else zeros.
constexpr int kPanelRows = 32;
struct PackChunk {
  int64_t d0;
  int64_t d1;
  int64_t src0;
  int64_t src1;
};

// Gram tiling: square output tiles of kGramTile columns; X^T Y is computed
// inside diagonal tiles when M <= kYDiagCols.
constexpr int kGramTile = 128;
constexpr int kYDiagCols = 32;

struct GramArgs {
  const void* Zp;       // packed panels (FP64 / FP32 / bf16 hi)
  const void* Zlo;      // bf16 lo panel (BF16X3 only)
  int64_t Wp, K, M, Kp;
  int32_t nt;           // tiles along X's columns (Kp / kGramTile)
  int32_t xy_diag;      // X^T Y inside diagonal tiles
  const GramWork* work;
  int64_t n_work;
  double* slabs;
};

}  // namespace cvg

struct cvgram_handle {
  int device = 0;
  hipStream_t stream = nullptr;
  int64_t N = 0, K = 0, M = 0, W = 0;  // W = K + M: columns of Z = [X | Y]
  cvgram_dtype dtype = CVGRAM_F64;
  cvgram_mode mode = CVGRAM_MODE_FP64;
  int cx = 0, sx = 0, cy = 0, sy = 0, ddof = 1;
  int32_t P = 0;
  bool scalable = false;            // every |T_p| - ddof >= 1
  std::vector<int64_t> h_offsets;   // [P+1]

  // Gram layout
  int64_t n_slabs = 0;
  int64_t n_work = 0;

  std::vector<cvg::DevBuf> bufs;    // everything below points into these

  int32_t* d_info = nullptr;        // scratch ints: label min/max, flags
  int32_t* d_keys = nullptr;        // [2][N] radix keys ping-pong
  int32_t* d_perm = nullptr;        // [N] final permutation
  int32_t* d_perm_tmp = nullptr;    // [N]
  int32_t* d_hist = nullptr;        // [256 * tiles]
  int64_t* d_offsets = nullptr;     // [P+1]
  int64_t* d_ntrain = nullptr;      // [P]
  double* d_pivot = nullptr;        // [W]
  double* d_part = nullptr;         // [4][chunks][W]  sum, sumsq, min, max
  void* d_packed = nullptr;         // packed panels (see PackChunk)
  void* d_packed_lo = nullptr;      // bf16 lo panel
  int64_t Kp = 0, Mp = 0, Wp = 0, Np = 0;
  double* d_fold = nullptr;         // [4][P][W]
  double* d_tr_sum = nullptr;       // [P][W]   shifted training sums
  double* d_tr_mean = nullptr;      // [P][W]   shifted training means
  double* d_tr_std = nullptr;       // [P][W]   training deviations (1 if constant)
  double* d_tr_mu = nullptr;        // [P][W]   unshifted training means
  double* d_scratch = nullptr;      // [2][P][W] suffix min/max
  uint8_t* d_tr_const = nullptr;    // [P][W]
  cvg::PackChunk* d_chunks = nullptr;
  int32_t* d_chunk_begin = nullptr; // [P+1]
  int64_t n_chunks = 0;
  double* d_slabs = nullptr;        // [n_slabs][K][W]
  double* d_G = nullptr;            // [K][W]
  int32_t* d_slab_begin = nullptr;  // [P+1]
  cvg::GramWork* d_work = nullptr;  // [n_work]
  int32_t* d_ctiles = nullptr;      // correction tile list: pairs (bi, bj)
  int32_t n_ctiles_xx = 0, n_ctiles_xy = 0;

  // host copies of the uploaded plans; kept until destroy so that the
  // asynchronous uploads never read freed host memory
  std::vector<std::vector<char>> host_plans;

  bool timing = false;              // stage events recorded at create
  hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
};

namespace cvg {

// ----------------------------- partition.hip -------------------------------
void launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
void launch_label_minmax(const int32_t* fold, int64_t N, int32_t* info, hipStream_t s);
// stable LSD radix sort of labels (values < 2^bits) carrying row indices;
// result: d_perm (rows by label), keys_out (sorted labels)
void radix_partition(const int32_t* fold, int64_t N, int bits, int32_t* keys_a, int32_t* keys_b,
                     int32_t* perm, int32_t* perm_tmp, int32_t* hist, const int32_t** sorted_keys,
                     hipStream_t s);
int64_t radix_hist_entries(int64_t N);
void launch_fold_offsets(const int32_t* sorted_keys, int64_t N, int32_t P, int64_t* offsets,
                         int32_t* flag, hipStream_t s);

// -------------------------------- pack.hip ---------------------------------
void launch_pivot(const void* X, const void* Y, cvgram_dtype dt, bool round_f32, int64_t N,
                  int64_t K, int64_t M, double* pivot, hipStream_t s);
void launch_pack(cvgram_mode mode, const void* X, const void* Y, cvgram_dtype dt, int64_t K,
                 int64_t M, int64_t Kp, int64_t Wp, const int32_t* perm, const PackChunk* chunks,
                 int64_t n_chunks, const double* pivot, void* packed, void* packed_lo,
                 double* part, hipStream_t s);

// ------------------------------- stats.hip ---------------------------------
void launch_stats_reduce(const double* part, int64_t n_chunks, const int32_t* chunk_begin,
                         int32_t P, int64_t W, double* fold, hipStream_t s);
void launch_train_stats(const double* fold, const int64_t* offsets, int32_t P, int64_t N,
                        int64_t W, int ddof, const double* pivot, double* scratch,
                        double* tr_sum, double* tr_mean, double* tr_std, double* tr_mu,
                        uint8_t* tr_const, int64_t* ntrain, hipStream_t s);
void launch_fold_stats(const double* tr_mu, const double* tr_std, int32_t p, int64_t K,
                       int64_t M, double* mx, double* sx, double* my, double* sy, hipStream_t s);

// -------------------------------- gram.hip ---------------------------------
void launch_gram(cvgram_mode mode, const GramArgs& g, hipStream_t s);

// ------------------------------- correct.hip -------------------------------
void launch_reduce_slabs(const double* slabs, int64_t n_slabs, int64_t elems, double* G,
                         hipStream_t s);

struct CorrectArgs {
  const double* slabs;
  const double* G;
  const int32_t* slab_begin;
  const double* pivot;
  const double* tr_sum;
  const double* tr_mean;
  const double* tr_std;
  const uint8_t* tr_const;
  const int64_t* ntrain;
  const int32_t* tiles;      // (bi, bj) pairs: XtX tiles first, then XtY tiles
  int64_t K, M, W;
  int32_t n_tiles_xx, n_tiles_xy;
  int32_t p_begin;
  void* out_xx[CVGRAM_XTX_CLASSES];   // base for fold p_begin, NULL = skip
  void* out_xy[CVGRAM_XTY_CLASSES];
  int64_t fold_stride_xx;    // elements between consecutive folds
  int64_t fold_stride_xy;
};

constexpr int kCorrTile = 32;

void launch_correct(const CorrectArgs& a, int32_t n_folds, bool out_f64, hipStream_t s);

}  // namespace cvg
