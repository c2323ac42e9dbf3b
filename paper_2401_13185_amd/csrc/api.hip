// C ABI of libcvgram: argument checks, fold bookkeeping and validation,
// planning of the grouped Gram launch, workspace ownership and dispatch of
// the per-fold correction kernels.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

namespace cvg {

static thread_local std::string g_last_error;
static std::atomic<int> g_stage_timing{0};

void set_error(const std::string& msg) { g_last_error = msg; }

namespace {

cvgram_status fail(cvgram_status st, const std::string& msg) {
  set_error(msg);
  return st;
}

// ---------------------------------------------------------------------------
// per-device workspace cache: blocks released by cvgram_destroy are reused by
// later handles when a cached block is at least as large as the request and
// at most about twice as large.
// ---------------------------------------------------------------------------
constexpr size_t kCacheCap = (size_t)32 << 30;
constexpr int kMaxDev = 64;

struct Cache {
  std::mutex mu;
  std::multimap<size_t, void*> blocks[kMaxDev];
  size_t total[kMaxDev] = {};
};
Cache& cache() {
  static Cache* c = new Cache();  // never destroyed: outlives static teardown
  return *c;
}

void cache_give(int dev, void* p, size_t bytes) {
  Cache& c = cache();
  {
    std::lock_guard<std::mutex> g(c.mu);
    if (dev >= 0 && dev < kMaxDev && c.total[dev] + bytes <= kCacheCap) {
      c.blocks[dev].insert({bytes, p});
      c.total[dev] += bytes;
      return;
    }
  }
  (void)hipFree(p);
}

void cache_trim(int dev) {
  Cache& c = cache();
  std::lock_guard<std::mutex> g(c.mu);
  if (dev < 0 || dev >= kMaxDev) return;
  for (auto& kv : c.blocks[dev]) (void)hipFree(kv.second);
  c.blocks[dev].clear();
  c.total[dev] = 0;
}

template <typename T>
T* alloc(cvgram_handle* h, int64_t count) {
  if (count <= 0) count = 1;
  const size_t want = ((size_t)count * sizeof(T) + 255) / 256 * 256;
  void* p = nullptr;
  size_t got = want;
  {
    Cache& c = cache();
    std::lock_guard<std::mutex> g(c.mu);
    if (h->device >= 0 && h->device < kMaxDev) {
      auto it = c.blocks[h->device].lower_bound(want);
      if (it != c.blocks[h->device].end() && it->first <= 2 * want + 4096) {
        p = it->second;
        got = it->first;
        c.total[h->device] -= it->first;
        c.blocks[h->device].erase(it);
      }
    }
  }
  if (!p) {
    hipError_t e = hipMalloc(&p, want);
    if (e == hipErrorOutOfMemory) {
      (void)hipGetLastError();
      cache_trim(h->device);
      e = hipMalloc(&p, want);
    }
    if (e != hipSuccess) {
      (void)hipGetLastError();
      set_error(std::string("hipMalloc(") + std::to_string(want) + "): " + hipGetErrorString(e));
      throw Fail{e == hipErrorOutOfMemory ? CVGRAM_ENOMEM : CVGRAM_EDEVICE};
    }
  }
  DevBuf b;
  b.ptr = p;
  b.bytes = got;
  h->bufs.push_back(b);
  return (T*)p;
}

void free_all(cvgram_handle* h) {
  for (auto& b : h->bufs)
    if (b.ptr) cache_give(h->device, b.ptr, b.bytes);
  h->bufs.clear();
  for (auto& e : h->ev)
    if (e) {
      (void)hipEventDestroy(e);
      e = nullptr;
    }
}

// Asynchronous upload of a host plan; the handle keeps the host bytes alive
// until it is destroyed.
template <typename T>
void upload(cvgram_handle* h, T* dst, const std::vector<T>& src, hipStream_t s) {
  if (src.empty()) return;
  const char* b = (const char*)src.data();
  h->host_plans.emplace_back(b, b + src.size() * sizeof(T));
  CVG_HIP(hipMemcpyAsync(dst, h->host_plans.back().data(), src.size() * sizeof(T),
                         hipMemcpyHostToDevice, s));
}

int bit_length(uint32_t v) {
  int b = 0;
  while (v) {
    ++b;
    v >>= 1;
  }
  return b;
}

constexpr int64_t kStatChunkRows = 1024;  // multiple of kPanelRows
constexpr int64_t kGramTargetItems = 2048;
constexpr int64_t kGramMinRows = 512;

bool out_is_f64(const cvgram_handle* h) { return h->mode == CVGRAM_MODE_FP64; }

// Runs the whole create pipeline; throws Fail on device errors.
cvgram_status build(cvgram_handle* h, const void* X, const void* Y, const int32_t* fold) {
  hipStream_t s = h->stream;
  const int64_t N = h->N, K = h->K, M = h->M, W = h->W;

  auto mark = [&](int k) {
    if (h->timing) CVG_HIP(hipEventRecord(h->ev[k], s));
  };
  if (h->timing)
    for (auto& e : h->ev) CVG_HIP(hipEventCreate(&e));
  mark(0);
  // ---- Algorithm 1: labels -> P, stable partition, offsets ---------------
  h->d_info = alloc<int32_t>(h, 64);
  launch_fill_i32(h->d_info, 1, INT32_MAX, s);
  launch_fill_i32(h->d_info + 1, 1, INT32_MIN, s);
  launch_fill_i32(h->d_info + 2, 62, 0, s);
  launch_label_minmax(fold, N, h->d_info, s);
  int32_t info[2] = {0, 0};
  CVG_HIP(hipMemcpyAsync(info, h->d_info, sizeof(info), hipMemcpyDeviceToHost, s));
  CVG_HIP(hipStreamSynchronize(s));
  if (info[0] < 0) return fail(CVGRAM_EFOLDS, "fold label < 0 (Definition 1)");
  const int64_t P = (int64_t)info[1] + 1;
  if (P < 2) return fail(CVGRAM_EFOLDS, "fewer than 2 folds (Definition 1)");
  if (P > N) return fail(CVGRAM_EFOLDS, "more folds than rows (Definition 1)");
  h->P = (int32_t)P;

  h->d_keys = alloc<int32_t>(h, 2 * N);
  h->d_perm = alloc<int32_t>(h, N);
  h->d_perm_tmp = alloc<int32_t>(h, N);
  h->d_hist = alloc<int32_t>(h, radix_hist_entries(N));
  h->d_offsets = alloc<int64_t>(h, P + 1);
  const int32_t* sorted = nullptr;
  radix_partition(fold, N, bit_length((uint32_t)(P - 1)), h->d_keys, h->d_keys + N, h->d_perm,
                  h->d_perm_tmp, h->d_hist, &sorted, s);
  launch_fold_offsets(sorted, N, (int32_t)P, h->d_offsets, h->d_info + 2, s);
  h->h_offsets.assign(P + 1, 0);
  int32_t flag = 0;
  CVG_HIP(hipMemcpyAsync(h->h_offsets.data(), h->d_offsets, (P + 1) * sizeof(int64_t),
                         hipMemcpyDeviceToHost, s));
  CVG_HIP(hipMemcpyAsync(&flag, h->d_info + 2, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  CVG_HIP(hipStreamSynchronize(s));
  if (flag) return fail(CVGRAM_EFOLDS, "a fold label in [0, P) has no rows (Definition 1)");
  int64_t max_fold = 0;
  for (int64_t p = 0; p < P; ++p)
    max_fold = std::max(max_fold, h->h_offsets[p + 1] - h->h_offsets[p]);
  h->scalable = (N - max_fold - h->ddof) >= 1;
  if ((h->sx || h->sy) && !h->scalable)
    return fail(CVGRAM_ENOTSCALABLE,
                "scaling needs |T_p| - ddof >= 1 for every fold (Definition 6)");

  // ---- plans --------------------------------------------------------------
  // packed rows: each fold padded to whole panels
  const int64_t PR = kPanelRows;
  std::vector<int64_t> poff(P + 1, 0);
  for (int64_t p = 0; p < P; ++p) {
    const int64_t n = h->h_offsets[p + 1] - h->h_offsets[p];
    poff[p + 1] = poff[p] + (n + PR - 1) / PR * PR;
  }
  h->Np = poff[P];
  // packed columns: X, zeros to Kp, Y, zeros to Wp
  h->Kp = (K + kGramTile - 1) / kGramTile * kGramTile;
  const bool xy_diag = M > 0 && M <= kYDiagCols;
  h->Mp = M == 0 ? 0 : (xy_diag ? kYDiagCols : (M + kGramTile - 1) / kGramTile * kGramTile);
  h->Wp = h->Kp + h->Mp;

  std::vector<PackChunk> chunks;
  std::vector<int32_t> chunk_begin(P + 1, 0);
  for (int64_t p = 0; p < P; ++p) {
    chunk_begin[p] = (int32_t)chunks.size();
    for (int64_t d = poff[p]; d < poff[p + 1]; d += kStatChunkRows)
      chunks.push_back({d, std::min(d + kStatChunkRows, poff[p + 1]),
                        h->h_offsets[p] + (d - poff[p]), h->h_offsets[p + 1]});
  }
  chunk_begin[P] = (int32_t)chunks.size();
  h->n_chunks = (int64_t)chunks.size();

  const int64_t nt = h->Kp / kGramTile;
  const int64_t nyt = xy_diag ? 0 : h->Mp / kGramTile;
  std::vector<std::pair<int32_t, int32_t>> gtiles;
  for (int64_t ti = 0; ti < nt; ++ti) {
    for (int64_t tj = ti; tj < nt; ++tj) gtiles.push_back({(int32_t)ti, (int32_t)tj});
    for (int64_t y = 0; y < nyt; ++y) gtiles.push_back({(int32_t)ti, (int32_t)(nt + y)});
  }
  const int64_t ntile = (int64_t)gtiles.size();
  // split folds along rows until the launch has enough items to fill the chip
  int64_t rows_per_split = (h->Np * ntile + kGramTargetItems - 1) / kGramTargetItems;
  rows_per_split = std::max(rows_per_split, kGramMinRows);
  rows_per_split = (rows_per_split + PR - 1) / PR * PR;
  std::vector<GramWork> work;
  std::vector<int32_t> slab_begin(P + 1, 0);
  int32_t slab = 0;
  for (int64_t p = 0; p < P; ++p) {
    slab_begin[p] = slab;
    const int64_t a = poff[p], b = poff[p + 1];
    const int64_t panels = (b - a) / PR;
    const int64_t splits =
        std::min(panels, std::max<int64_t>(1, (b - a + rows_per_split - 1) / rows_per_split));
    for (int64_t sp = 0; sp < splits; ++sp) {
      const int64_t r0 = a + panels * sp / splits * PR;
      const int64_t r1 = a + panels * (sp + 1) / splits * PR;
      for (auto& tt : gtiles) work.push_back({(int32_t)p, slab, tt.first, tt.second, r0, r1});
      ++slab;
    }
  }
  slab_begin[P] = slab;
  h->n_slabs = slab;
  h->n_work = (int64_t)work.size();

  std::vector<int32_t> ctiles;
  const int64_t nct = (K + kCorrTile - 1) / kCorrTile;
  for (int64_t bi = 0; bi < nct; ++bi)
    for (int64_t bj = bi; bj < nct; ++bj) {
      ctiles.push_back((int32_t)bi);
      ctiles.push_back((int32_t)bj);
    }
  h->n_ctiles_xx = (int32_t)(ctiles.size() / 2);
  const int64_t ncy = (M + kCorrTile - 1) / kCorrTile;
  for (int64_t bi = 0; bi < nct; ++bi)
    for (int64_t bj = 0; bj < ncy; ++bj) {
      ctiles.push_back((int32_t)bi);
      ctiles.push_back((int32_t)bj);
    }
  h->n_ctiles_xy = (int32_t)(ctiles.size() / 2) - h->n_ctiles_xx;

  // ---- workspace ---------------------------------------------------------
  h->d_pivot = alloc<double>(h, W);
  h->d_chunks = alloc<PackChunk>(h, h->n_chunks);
  if (h->mode == CVGRAM_MODE_FP64) {
    h->d_packed = alloc<double>(h, h->Np * h->Wp);
  } else if (h->mode == CVGRAM_MODE_FP32) {
    h->d_packed = alloc<float>(h, h->Np * h->Wp);
  } else {
    h->d_packed = alloc<uint16_t>(h, h->Np * h->Wp);
    h->d_packed_lo = alloc<uint16_t>(h, h->Np * h->Wp);
  }
  h->d_chunk_begin = alloc<int32_t>(h, P + 1);
  h->d_part = alloc<double>(h, 4 * h->n_chunks * W);
  h->d_fold = alloc<double>(h, 4 * P * W);
  h->d_scratch = alloc<double>(h, 2 * P * W);
  h->d_tr_sum = alloc<double>(h, P * W);
  h->d_tr_mean = alloc<double>(h, P * W);
  h->d_tr_std = alloc<double>(h, P * W);
  h->d_tr_mu = alloc<double>(h, P * W);
  h->d_tr_const = alloc<uint8_t>(h, P * W);
  h->d_ntrain = alloc<int64_t>(h, P);
  h->d_slabs = alloc<double>(h, h->n_slabs * K * W);
  h->d_G = alloc<double>(h, K * W);
  h->d_slab_begin = alloc<int32_t>(h, P + 1);
  h->d_work = alloc<GramWork>(h, h->n_work);
  h->d_ctiles = alloc<int32_t>(h, (int64_t)ctiles.size());
  upload(h, h->d_chunks, chunks, s);
  upload(h, h->d_chunk_begin, chunk_begin, s);
  upload(h, h->d_slab_begin, slab_begin, s);
  upload(h, h->d_work, work, s);
  upload(h, h->d_ctiles, ctiles, s);

  // ---- statistics and Gram pass -------------------------------------------
  const bool mixed = h->mode != CVGRAM_MODE_FP64;
  mark(1);
  launch_pivot(X, Y, h->dtype, mixed, N, K, M, h->d_pivot, s);
  launch_pack(h->mode, X, Y, h->dtype, K, M, h->Kp, h->Wp, h->d_perm, h->d_chunks, h->n_chunks,
              h->d_pivot, h->d_packed, h->d_packed_lo, h->d_part, s);
  launch_stats_reduce(h->d_part, h->n_chunks, h->d_chunk_begin, (int32_t)P, W, h->d_fold, s);
  launch_train_stats(h->d_fold, h->d_offsets, (int32_t)P, N, W, h->ddof, h->d_pivot,
                     h->d_scratch, h->d_tr_sum, h->d_tr_mean, h->d_tr_std, h->d_tr_mu,
                     h->d_tr_const, h->d_ntrain, s);
  mark(2);
  GramArgs ga;
  ga.Zp = h->d_packed;
  ga.Zlo = h->d_packed_lo;
  ga.Wp = h->Wp;
  ga.K = K;
  ga.M = M;
  ga.Kp = h->Kp;
  ga.nt = (int32_t)nt;
  ga.xy_diag = xy_diag ? 1 : 0;
  ga.work = h->d_work;
  ga.n_work = h->n_work;
  ga.slabs = h->d_slabs;
  launch_gram(h->mode, ga, s);
  mark(3);
  launch_reduce_slabs(h->d_slabs, h->n_slabs, K * W, h->d_G, s);
  mark(4);
  return CVGRAM_OK;
}

CorrectArgs base_args(const cvgram_handle* h) {
  CorrectArgs a;
  std::memset(&a, 0, sizeof(a));
  a.slabs = h->d_slabs;
  a.G = h->d_G;
  a.slab_begin = h->d_slab_begin;
  a.pivot = h->d_pivot;
  a.tr_sum = h->d_tr_sum;
  a.tr_mean = h->d_tr_mean;
  a.tr_std = h->d_tr_std;
  a.tr_const = h->d_tr_const;
  a.ntrain = h->d_ntrain;
  a.tiles = h->d_ctiles;
  a.K = h->K;
  a.M = h->M;
  a.W = h->W;
  a.n_tiles_xx = h->n_ctiles_xx;
  a.n_tiles_xy = h->n_ctiles_xy;
  return a;
}

bool flag01(int v) { return v == 0 || v == 1; }

}  // namespace
}  // namespace cvg

using namespace cvg;

extern "C" {

cvgram_status cvgram_create(const void* X, const void* Y, const int32_t* fold_id, int64_t N,
                            int64_t K, int64_t M, cvgram_dtype dtype, int center_x, int scale_x,
                            int center_y, int scale_y, int ddof, cvgram_mode mode, void* stream,
                            cvgram_t* out) {
  set_error("");
  if (!out) return fail(CVGRAM_EINVAL, "out is NULL");
  *out = nullptr;
  if (!X || !fold_id) return fail(CVGRAM_EINVAL, "X or fold_id is NULL");
  if (M > 0 && !Y) return fail(CVGRAM_EINVAL, "Y is NULL with M > 0");
  if (N < 2 || K < 1 || M < 0) return fail(CVGRAM_EINVAL, "need N >= 2, K >= 1, M >= 0");
  if (N > (int64_t)INT32_MAX - 1) return fail(CVGRAM_EINVAL, "N must fit in int32");
  if (dtype != CVGRAM_F32 && dtype != CVGRAM_F64) return fail(CVGRAM_EINVAL, "bad dtype");
  if (mode != CVGRAM_MODE_FP64 && mode != CVGRAM_MODE_FP32 && mode != CVGRAM_MODE_BF16X3)
    return fail(CVGRAM_EINVAL, "bad mode");
  if (!flag01(center_x) || !flag01(scale_x) || !flag01(center_y) || !flag01(scale_y))
    return fail(CVGRAM_EINVAL, "centering/scaling flags must be 0 or 1");
  if (ddof != 0 && ddof != 1) return fail(CVGRAM_EINVAL, "ddof must be 0 or 1");

  std::unique_ptr<cvgram_handle> h(new cvgram_handle());
  h->stream = (hipStream_t)stream;
  h->N = N;
  h->K = K;
  h->M = M;
  h->W = K + M;
  h->dtype = dtype;
  h->mode = mode;
  h->cx = center_x;
  h->sx = scale_x;
  h->cy = center_y;
  h->sy = scale_y;
  h->ddof = ddof;
  h->timing = g_stage_timing.load() != 0;
  cvgram_status st;
  try {
    CVG_HIP(hipGetDevice(&h->device));
    st = build(h.get(), X, Y, fold_id);
  } catch (const Fail& f) {
    st = f.st;
  }
  if (st != CVGRAM_OK) {
    (void)hipStreamSynchronize(h->stream);
    free_all(h.get());
    return st;
  }
  *out = h.release();
  return CVGRAM_OK;
}

cvgram_status cvgram_num_folds(cvgram_t h, int32_t* P) {
  if (!h || !P) return fail(CVGRAM_EINVAL, "NULL argument");
  *P = h->P;
  return CVGRAM_OK;
}

cvgram_status cvgram_partition(cvgram_t h, int32_t* perm, int64_t* offsets) {
  if (!h) return fail(CVGRAM_EINVAL, "NULL handle");
  try {
    if (perm)
      CVG_HIP(hipMemcpyAsync(perm, h->d_perm, h->N * sizeof(int32_t), hipMemcpyDeviceToDevice,
                             h->stream));
    if (offsets)
      CVG_HIP(hipMemcpyAsync(offsets, h->d_offsets, (h->P + 1) * sizeof(int64_t),
                             hipMemcpyDeviceToDevice, h->stream));
  } catch (const Fail& f) {
    return f.st;
  }
  return CVGRAM_OK;
}

static cvgram_status run_correct(cvgram_t h, int32_t p0, int32_t p1, void* const* xx,
                                 void* const* xy) {
  CorrectArgs a = base_args(h);
  a.p_begin = p0;
  for (int c = 0; c < CVGRAM_XTX_CLASSES; ++c) a.out_xx[c] = xx[c];
  for (int c = 0; c < CVGRAM_XTY_CLASSES; ++c) a.out_xy[c] = xy[c];
  a.fold_stride_xx = 0;
  a.fold_stride_xy = 0;
  try {
    launch_correct(a, p1 - p0, out_is_f64(h), h->stream);
  } catch (const Fail& f) {
    return f.st;
  }
  return CVGRAM_OK;
}

cvgram_status cvgram_fold_combo(cvgram_t h, int32_t p, int center_x, int scale_x, int center_y,
                                int scale_y, void* out_XtX, void* out_XtY) {
  if (!h) return fail(CVGRAM_EINVAL, "NULL handle");
  if (p < 0 || p >= h->P) return fail(CVGRAM_ERANGE, "fold index out of range");
  if (!flag01(center_x) || !flag01(scale_x) || !flag01(center_y) || !flag01(scale_y))
    return fail(CVGRAM_EINVAL, "centering/scaling flags must be 0 or 1");
  if ((scale_x || scale_y) && !h->scalable)
    return fail(CVGRAM_ENOTSCALABLE, "partitioning is not scalable for this ddof");
  void* xx[CVGRAM_XTX_CLASSES] = {nullptr, nullptr, nullptr, nullptr};
  void* xy[CVGRAM_XTY_CLASSES] = {nullptr, nullptr, nullptr, nullptr,
                                  nullptr, nullptr, nullptr, nullptr};
  xx[2 * center_x + scale_x] = out_XtX;
  if (h->M > 0) xy[4 * (center_x | center_y) + 2 * scale_x + scale_y] = out_XtY;
  return run_correct(h, p, p + 1, xx, xy);
}

cvgram_status cvgram_fold(cvgram_t h, int32_t p, void* out_XtX, void* out_XtY) {
  if (!h) return fail(CVGRAM_EINVAL, "NULL handle");
  return cvgram_fold_combo(h, p, h->cx, h->sx, h->cy, h->sy, out_XtX, out_XtY);
}

cvgram_status cvgram_folds_all(cvgram_t h, int32_t p_begin, int32_t p_end, void* out_XtX,
                               void* out_XtY) {
  if (!h) return fail(CVGRAM_EINVAL, "NULL handle");
  if (p_begin < 0 || p_end > h->P || p_begin > p_end)
    return fail(CVGRAM_ERANGE, "fold range out of bounds");
  if (p_begin == p_end) return CVGRAM_OK;
  CorrectArgs a = base_args(h);
  a.p_begin = p_begin;
  const size_t es = out_is_f64(h) ? sizeof(double) : sizeof(float);
  const int64_t KK = h->K * h->K, KM = h->K * h->M;
  for (int c = 0; c < CVGRAM_XTX_CLASSES; ++c) {
    const bool scaled = c & 1;
    a.out_xx[c] = (out_XtX && (h->scalable || !scaled)) ? (char*)out_XtX + c * KK * es : nullptr;
  }
  for (int c = 0; c < CVGRAM_XTY_CLASSES; ++c) {
    const bool scaled = c & 3;
    a.out_xy[c] = (out_XtY && h->M > 0 && (h->scalable || !scaled))
                      ? (char*)out_XtY + c * KM * es
                      : nullptr;
  }
  a.fold_stride_xx = CVGRAM_XTX_CLASSES * KK;
  a.fold_stride_xy = CVGRAM_XTY_CLASSES * KM;
  try {
    launch_correct(a, p_end - p_begin, out_is_f64(h), h->stream);
  } catch (const Fail& f) {
    return f.st;
  }
  return CVGRAM_OK;
}

cvgram_status cvgram_fold_stats(cvgram_t h, int32_t p, double* mean_x, double* std_x,
                                double* mean_y, double* std_y) {
  if (!h) return fail(CVGRAM_EINVAL, "NULL handle");
  if (p < 0 || p >= h->P) return fail(CVGRAM_ERANGE, "fold index out of range");
  try {
    launch_fold_stats(h->d_tr_mu, h->d_tr_std, p, h->K, h->M, mean_x, std_x, mean_y, std_y,
                      h->stream);
  } catch (const Fail& f) {
    return f.st;
  }
  return CVGRAM_OK;
}

cvgram_status cvgram_set_stage_timing(int on) {
  g_stage_timing.store(on ? 1 : 0);
  return CVGRAM_OK;
}

cvgram_status cvgram_stage_times(cvgram_t h, double* ms, int32_t n) {
  if (!h || (!ms && n > 0)) return fail(CVGRAM_EINVAL, "NULL argument");
  if (!h->timing) return fail(CVGRAM_EINVAL, "handle created without stage timing");
  try {
    CVG_HIP(hipEventSynchronize(h->ev[4]));
    for (int k = 0; k < 4 && k < n; ++k) {
      float t = 0.f;
      CVG_HIP(hipEventElapsedTime(&t, h->ev[k], h->ev[k + 1]));
      ms[k] = t;
    }
  } catch (const Fail& f) {
    return f.st;
  }
  return CVGRAM_OK;
}

cvgram_status cvgram_trim_cache(void) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(CVGRAM_EDEVICE, "hipGetDevice failed");
  cache_trim(dev);
  return CVGRAM_OK;
}

cvgram_status cvgram_set_stream(cvgram_t h, void* stream) {
  if (!h) return fail(CVGRAM_EINVAL, "NULL handle");
  h->stream = (hipStream_t)stream;
  return CVGRAM_OK;
}

cvgram_status cvgram_destroy(cvgram_t h) {
  if (!h) return CVGRAM_OK;
  hipError_t e = hipStreamSynchronize(h->stream);
  free_all(h);
  delete h;
  if (e != hipSuccess) return fail(CVGRAM_EDEVICE, hipGetErrorString(e));
  return CVGRAM_OK;
}

const char* cvgram_status_string(cvgram_status s) {
  switch (s) {
    case CVGRAM_OK: return "ok";
    case CVGRAM_EINVAL: return "invalid argument";
    case CVGRAM_EFOLDS: return "invalid partitioning (Definition 1)";
    case CVGRAM_ENOTSCALABLE: return "partitioning not scalable (Definition 6)";
    case CVGRAM_ENOMEM: return "out of memory";
    case CVGRAM_EDEVICE: return "HIP runtime error";
    case CVGRAM_ERANGE: return "fold index out of range";
  }
  return "unknown status";
}

const char* cvgram_last_error_message(void) { return g_last_error.c_str(); }

int32_t cvgram_version(void) { return 100; }

}  // extern "C"
