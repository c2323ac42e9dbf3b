// C ABI of libcvgram: argument checks, fold bookkeeping and validation,
// planning of every launch, workspace ownership, the batched pipeline and
// its HIP graph, and the autotuning table.
#include <algorithm>
#include <atomic>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <tuple>
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
// workspace caches.  Device blocks (per device) and pinned host blocks
// released by a handle are reused by later handles when a cached block is at
// least as large as the request and at most about twice as large.
//
// Release is stream-ordered: a handle released with work still queued tags
// its blocks with an event recorded on its stream at that point.  A tagged
// device block is reused at once by work on the same stream (stream order
// puts the new work behind the old); by another stream, and a pinned block by
// the host, only once the event has completed.
// ---------------------------------------------------------------------------
// device cache bound: half of the device's memory, at least 32 GiB (a
// large problem's workspace, tens of GB, then stays cached between handles)
constexpr size_t kCacheCapMin = (size_t)32 << 30;
constexpr size_t kHostCacheCap = (size_t)1 << 30;
constexpr int kMaxDev = 64;

hipEvent_t event_get(int device, bool timed);
void event_put(int device, bool timed, hipEvent_t e);

// the event of one stream-ordered release, shared by the blocks it tags;
// back to the event pool when the last of them leaves the cache
struct ReleaseMark {
  int device = 0;
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;
  ~ReleaseMark() { event_put(device, false, ev); }
};
struct Cached {
  void* ptr = nullptr;
  std::shared_ptr<ReleaseMark> mark;  // null: released with no work queued
};

struct Cache {
  std::mutex mu;
  std::multimap<size_t, Cached> dev[kMaxDev];
  size_t dev_total[kMaxDev] = {};
  size_t dev_cap[kMaxDev] = {};  // 0: not yet known
  std::multimap<size_t, Cached> host;
  size_t host_total = 0;
};
Cache& cache() {
  static Cache* c = new Cache();  // never destroyed: outlives static teardown
  return *c;
}

// true once the work before the mark has completed (no mark: nothing queued)
bool mark_done(const std::shared_ptr<ReleaseMark>& mk) {
  if (!mk) return true;
  const hipError_t e = hipEventQuery(mk->ev);
  if (e == hipSuccess) return true;
  (void)hipGetLastError();  // "not ready" is an answer, not an error to keep
  return false;
}

void cache_trim_dev(int dev) {
  std::multimap<size_t, Cached> gone;
  {
    Cache& c = cache();
    std::lock_guard<std::mutex> g(c.mu);
    if (dev < 0 || dev >= kMaxDev) return;
    gone.swap(c.dev[dev]);
    c.dev_total[dev] = 0;
  }
  for (auto& kv : gone) {
    if (kv.second.mark) (void)hipEventSynchronize(kv.second.mark->ev);
    (void)hipFree(kv.second.ptr);
  }
}

// a cached block of at least `want` bytes and at most about twice that.  A
// block that is free now (idle, or a device block last released on `stream`)
// is preferred; else the first that fits is returned with the mark the caller
// must wait for before using it.
struct Taken {
  void* p = nullptr;
  std::shared_ptr<ReleaseMark> wait;
};
Taken take(std::multimap<size_t, Cached>& m, size_t& total, size_t want, size_t* got,
           hipStream_t stream, bool host) {
  Taken r;
  auto pick = m.end(), first = m.end();
  int looked = 0;
  for (auto it = m.lower_bound(want); it != m.end() && it->first <= 2 * want + 4096 && looked < 8;
       ++it, ++looked) {
    const auto& mk = it->second.mark;
    if ((!host && mk && mk->stream == stream) || mark_done(mk)) {
      pick = it;
      break;
    }
    if (first == m.end()) first = it;
  }
  if (pick == m.end()) {
    if (first == m.end()) return r;
    pick = first;
    r.wait = pick->second.mark;
  }
  r.p = pick->second.ptr;
  *got = pick->first;
  total -= pick->first;
  m.erase(pick);
  return r;
}

// one owned block: device or pinned host
struct Block {
  void* ptr = nullptr;
  size_t bytes = 0;
  bool host = false;
};

// Fixed memory of the allocation-free entry point: device blocks are carved
// in order from the library's static scratch array (through its device
// address), host staging from a static host buffer.  Nothing is allocated,
// and giving blocks back is a no-op; a request beyond either region fails.
struct Arena {
  char* dev = nullptr;
  size_t dev_cap = 0, dev_used = 0;
  char* host = nullptr;
  size_t host_cap = 0, host_used = 0;

  void* take(bool on_host, size_t want) {
    char* base = on_host ? host : dev;
    size_t& used = on_host ? host_used : dev_used;
    const size_t cap = on_host ? host_cap : dev_cap;
    if (want > cap - used) {
      set_error(std::string("the allocation-free entry point needs more ") +
                (on_host ? "host staging" : "device workspace") + " than its fixed " +
                std::to_string(cap >> 20) + " MiB (" + std::to_string(used + want) +
                " bytes asked for): use cvgram_create for this problem");
      throw Fail{CVGRAM_EINVAL};
    }
    void* p = base + used;
    used += want;
    return p;
  }
};

struct Owned {
  int device = 0;
  hipStream_t stream = nullptr;  // the stream the owner's work runs on
  std::vector<Block> blocks;
  Arena* arena = nullptr;        // set: every block comes from it

  void* dev(size_t want) {
    want = (want + 255) / 256 * 256;
    if (want == 0) want = 256;
    if (arena) return arena->take(false, want);
    size_t got = want;
    Taken tk;
    {
      Cache& c = cache();
      std::lock_guard<std::mutex> g(c.mu);
      if (device >= 0 && device < kMaxDev)
        tk = take(c.dev[device], c.dev_total[device], want, &got, stream, false);
    }
    void* p = tk.p;
    if (tk.wait && hipEventSynchronize(tk.wait->ev) != hipSuccess) {
      (void)hipGetLastError();
      (void)hipDeviceSynchronize();
    }
    if (!p) {
      hipError_t e = hipMalloc(&p, want);
      if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        cache_trim_dev(device);
        e = hipMalloc(&p, want);
      }
      if (e != hipSuccess) {
        (void)hipGetLastError();
        set_error("hipMalloc(" + std::to_string(want) + "): " + hipGetErrorString(e));
        throw Fail{e == hipErrorOutOfMemory ? CVGRAM_ENOMEM : CVGRAM_EDEVICE};
      }
      got = want;
    }
    blocks.push_back({p, got, false});
    return p;
  }

  void* pinned(size_t want) {
    want = (want + 4095) / 4096 * 4096;
    if (want == 0) want = 4096;
    if (arena) return arena->take(true, want);
    size_t got = want;
    Taken tk;
    {
      Cache& c = cache();
      std::lock_guard<std::mutex> g(c.mu);
      tk = take(c.host, c.host_total, want, &got, stream, true);
    }
    void* p = tk.p;
    if (tk.wait && hipEventSynchronize(tk.wait->ev) != hipSuccess) {
      (void)hipGetLastError();
      (void)hipDeviceSynchronize();
    }
    if (!p) {
      hipError_t e = hipHostMalloc(&p, want, hipHostMallocDefault);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        set_error("hipHostMalloc(" + std::to_string(want) + "): " + hipGetErrorString(e));
        throw Fail{CVGRAM_ENOMEM};
      }
      got = want;
    }
    blocks.push_back({p, got, true});
    return p;
  }

  // give one block back early (scratch)
  void give_back(void* p) {
    for (size_t i = 0; i < blocks.size(); ++i)
      if (blocks[i].ptr == p) {
        release_one(blocks[i]);
        blocks.erase(blocks.begin() + (long)i);
        return;
      }
  }

  void release_one(const Block& b, const std::shared_ptr<ReleaseMark>& mark = nullptr) {
    Cache& c = cache();
    size_t cap = kCacheCapMin;
    if (!b.host && device >= 0 && device < kMaxDev) {
      {
        std::lock_guard<std::mutex> g(c.mu);
        cap = c.dev_cap[device];
      }
      if (cap == 0) {
        size_t total_b = 0;
        if (hipDeviceTotalMem(&total_b, device) != hipSuccess) {
          (void)hipGetLastError();
          total_b = 0;
        }
        cap = std::max(kCacheCapMin, total_b / 2);
        std::lock_guard<std::mutex> g(c.mu);
        c.dev_cap[device] = cap;
      }
    }
    {
      std::lock_guard<std::mutex> g(c.mu);
      if (b.host) {
        if (c.host_total + b.bytes <= kHostCacheCap) {
          c.host.insert({b.bytes, Cached{b.ptr, mark}});
          c.host_total += b.bytes;
          return;
        }
      } else if (device >= 0 && device < kMaxDev && c.dev_total[device] + b.bytes <= cap) {
        c.dev[device].insert({b.bytes, Cached{b.ptr, mark}});
        c.dev_total[device] += b.bytes;
        return;
      }
    }
    if (mark) (void)hipEventSynchronize(mark->ev);
    if (b.host)
      (void)hipHostFree(b.ptr);
    else
      (void)hipFree(b.ptr);
  }

  // every block back to the cache; no work that uses them may be queued
  void release() {
    for (auto& b : blocks) release_one(b);
    blocks.clear();
  }

  // every block back to the cache while work that uses them may still be
  // queued on `s`: they are tagged with an event recorded there now
  void release_async(hipStream_t s) {
    if (blocks.empty()) return;
    auto mark = std::make_shared<ReleaseMark>();
    mark->device = device;
    mark->stream = s;
    bool ok = false;
    try {
      mark->ev = event_get(device, false);
      ok = hipEventRecord(mark->ev, s) == hipSuccess;
    } catch (const Fail&) {
    }
    if (!ok) {
      (void)hipGetLastError();
      (void)hipStreamSynchronize(s);
      release();
      return;
    }
    for (auto& b : blocks) release_one(b, mark);
    blocks.clear();
  }
};

// ---------------------------------------------------------------------------
// launch configuration and the autotuning table
// ---------------------------------------------------------------------------
struct Config {
  int tile = 128;
  int64_t target_items = 1024;  // Gram work items to aim for
  // a tuned batch rule: 256 x 128 tiles only for K >= wide_min_k (0: every
  // problem the built-in rule gives them)
  int64_t wide_min_k = 0;
};

int log2_bucket(int64_t v) {
  int b = 0;
  while ((int64_t(1) << b) < v && b < 62) ++b;
  return b;
}

// Tuned choices, keyed by the device (architecture name and compute-unit
// count: a table written on another part is kept but not used), the mode,
// the input type and log2 buckets of K, M + 1, N and the mean fold size
// N / P (which sets how many row splits fill the chip).
using TuneKey = std::tuple<std::string, int, int, int, int, int, int>;
struct TuneTable {
  std::mutex mu;
  std::map<TuneKey, Config> t;
  std::map<int, std::string> arch;  // device ordinal -> key of its part
  bool loaded = false;
};
TuneTable& tune_table() {
  static TuneTable* t = new TuneTable();
  return *t;
}

// "<gcnArchName>/<CUs>" of the current device, with no spaces (call with the
// table's mutex held)
const std::string& device_arch_locked(TuneTable& tt) {
  static const std::string none = "none";
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return none;  // planning on a host without a device: no tuned entry applies
  }
  auto it = tt.arch.find(dev);
  if (it != tt.arch.end()) return it->second;
  hipDeviceProp_t prop;
  CVG_HIP(hipGetDeviceProperties(&prop, dev));
  std::string a = std::string(prop.gcnArchName) + "/" + std::to_string(prop.multiProcessorCount);
  for (char& ch : a)
    if (ch == ' ') ch = '_';
  return tt.arch[dev] = a;
}

TuneKey tune_key_locked(TuneTable& tt, cvgram_mode mode, cvgram_dtype dt, int64_t K, int64_t M,
                        int64_t N, int64_t P) {
  return TuneKey(device_arch_locked(tt), (int)mode, (int)dt, log2_bucket(K), log2_bucket(M + 1),
                 log2_bucket(N), log2_bucket(std::max<int64_t>(1, N / std::max<int64_t>(1, P))));
}

void tune_load_locked(TuneTable& tt) {
  if (tt.loaded) return;
  tt.loaded = true;
  const char* path = std::getenv("CVGRAM_TUNE_FILE");
  if (!path) return;
  FILE* f = std::fopen(path, "r");
  if (!f) return;
  char arch[128];
  int a, b, c, d, e, v, tile;
  long long items;
  while (std::fscanf(f, "%127s %d %d %d %d %d %d %d %lld", arch, &a, &b, &c, &d, &e, &v, &tile,
                     &items) == 9)
    if ((tile == 64 || tile == 128 || tile == 256) && items > 0)
      tt.t[TuneKey(arch, a, b, c, d, e, v)] = {tile, items};
  std::fclose(f);
}

void tune_save_locked(TuneTable& tt) {
  const char* path = std::getenv("CVGRAM_TUNE_FILE");
  if (!path) return;
  FILE* f = std::fopen(path, "w");
  if (!f) return;
  for (auto& kv : tt.t)
    std::fprintf(f, "%s %d %d %d %d %d %d %d %lld\n", std::get<0>(kv.first).c_str(),
                 std::get<1>(kv.first), std::get<2>(kv.first), std::get<3>(kv.first),
                 std::get<4>(kv.first), std::get<5>(kv.first), std::get<6>(kv.first),
                 kv.second.tile, (long long)kv.second.target_items);
  std::fclose(f);
}

// Built-in tile rule: 64 for K <= 64, else 128, and in BF16X3 mode 256 x 128
// tiles from K > 128 (half the panel bytes per product of the 128-wide
// tiles; narrower problems would pad to 256 columns).  CVGRAM_BF16_TILE
// (64, 128 or 256) overrides the BF16X3 choice.
Config default_config(cvgram_mode mode, int64_t K) {
  Config c;
  c.tile = K <= 64 ? 64 : 128;
  if (mode == CVGRAM_MODE_BF16X3) {
    if (K > 128) c.tile = 256;
    if (const char* e = std::getenv("CVGRAM_BF16_TILE")) {
      const int v = std::atoi(e);
      if (v == 64 || v == 128 || v == 256) c.tile = v;
    }
  }
  c.target_items = mode == CVGRAM_MODE_FP64 ? 1536 : 1024;
  return c;
}

// the widest tile the built-in rule gives a problem of this K (no override)
int natural_tile(cvgram_mode mode, int64_t K) {
  if (K <= 64) return 64;
  return (mode == CVGRAM_MODE_BF16X3 && K > 128) ? 256 : 128;
}

Config choose_config(cvgram_mode mode, cvgram_dtype dt, int64_t K, int64_t M, int64_t N,
                     int64_t P) {
  TuneTable& tt = tune_table();
  std::lock_guard<std::mutex> g(tt.mu);
  tune_load_locked(tt);
  auto it = tt.t.find(tune_key_locked(tt, mode, dt, K, M, N, P));
  if (it != tt.t.end()) return it->second;
  return default_config(mode, K);
}

// ---------------------------------------------------------------------------
// plans
// ---------------------------------------------------------------------------
struct ProbPlan {
  const void* X = nullptr;
  const void* Y = nullptr;
  const int32_t* fold = nullptr;
  int64_t N = 0, K = 0, M = 0, W = 0;
  void* out_xx = nullptr;
  void* out_xy = nullptr;
  int32_t P = 0;
  bool scalable = false;
  std::vector<int64_t> offsets;  // [P+1]
  Config cfg;
  bool fused = false;         // fold path (see ProbDesc::fused)
  int64_t Kp = 0, Mp = 0, Wp = 0, Np = 0;
  bool xy_diag = false;
  int32_t nt = 0;
  bool tile_groups = false;   // tile order and XCD spread (see kTileGroup)
  std::vector<int64_t> poff;  // [P+1] packed row offsets
  std::vector<int32_t> chunk_begin, slab_begin, ctiles;
  int64_t n_chunks = 0, n_slabs = 0;
  int32_t n_franges = 0;
  int32_t n_ctiles_xx = 0, n_ctiles_xy = 0;
  int32_t* d_perm = nullptr;
  double* d_pivot = nullptr;  // computed at bookkeeping time (single problems)
};

// Events of released handles, kept per device and reused by later handles
// (a handle per call is the common pattern; creating its events each time
// would sit on the host path between two steps).  An event may come back
// with its last record still pending: its next user records it again, and
// nothing waits on the old record any more.
struct EventPool {
  std::mutex mu;
  std::vector<hipEvent_t> timed[kMaxDev], plain[kMaxDev];
};
EventPool& event_pool() {
  static EventPool* e = new EventPool();  // never destroyed: outlives static teardown
  return *e;
}
hipEvent_t event_get(int device, bool timed) {
  if (device >= 0 && device < kMaxDev) {
    EventPool& ep = event_pool();
    std::lock_guard<std::mutex> g(ep.mu);
    auto& v = timed ? ep.timed[device] : ep.plain[device];
    if (!v.empty()) {
      hipEvent_t e = v.back();
      v.pop_back();
      return e;
    }
  }
  hipEvent_t e = nullptr;
  CVG_HIP(hipEventCreateWithFlags(&e, timed ? hipEventDefault : hipEventDisableTiming));
  return e;
}
void event_put(int device, bool timed, hipEvent_t e) {
  if (!e) return;
  if (device >= 0 && device < kMaxDev) {
    EventPool& ep = event_pool();
    std::lock_guard<std::mutex> g(ep.mu);
    auto& v = timed ? ep.timed[device] : ep.plain[device];
    if (v.size() < 64) {
      v.push_back(e);
      return;
    }
  }
  (void)hipEventDestroy(e);
}

// the device pipeline of a batch (a single handle is a batch of one)
struct Batch {
  int device = 0;
  hipStream_t stream = nullptr;
  cvgram_mode mode = CVGRAM_MODE_FP64;
  cvgram_dtype dtype = CVGRAM_F64;
  int ddof = 1;
  bool batched = false;           // outputs written by the pipeline itself
  bool force_cfg = false;         // autotuner candidates
  Config forced;
  std::vector<ProbPlan> pp;
  Owned mem;
  std::vector<ProbDesc> h_pd;     // host copies of the descriptors
  ProbDesc* d_pd = nullptr;
  OutDesc* d_out = nullptr;
  Item* d_pivot_items = nullptr;
  int64_t n_pivot_items = 0;
  PackChunk* d_chunks = nullptr;
  int64_t n_chunks = 0;
  int32_t max_pack_cb = 0;
  Item* d_fold_items = nullptr;
  int64_t n_fold_items = 0;
  Item* d_sr_items = nullptr;     // folds of grouped-path problems
  int64_t n_sr_items = 0;
  Item* d_fs_items = nullptr;     // folds of fused-path problems
  int64_t n_fs_items = 0;
  int32_t max_cb64 = 0, max_cb256 = 0;
  Item* d_cb_items = nullptr;
  int64_t n_cb_items = 0;
  Item* d_range_items = nullptr;
  int64_t n_range_items = 0;
  GramWork* d_work = nullptr;     // the items of the three launches, one array
  int64_t n_work[kWidths] = {};
  int32_t* d_xcd[kWidths] = {};   // per-XCD item ranges of each launch
  int64_t grid[kWidths] = {};     // largest per-XCD item count
  Item* d_red_items = nullptr;
  int64_t n_red_items = 0;
  Item* d_corr_items = nullptr;
  int64_t n_corr_items = 0;
  bool timing = false;
  hipEvent_t ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
  hipEvent_t ev_wait = nullptr;   // the host's wait for the label counts
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;

  void release() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    gexec = nullptr;
    graph = nullptr;
    for (auto& e : ev) {
      event_put(device, true, e);
      e = nullptr;
    }
    event_put(device, false, ev_wait);
    ev_wait = nullptr;
    mem.release();
  }
  // as release(), with work still queued on the stream (stream-ordered; a
  // captured graph is waited for first)
  void release_async() {
    if (gexec || graph) {
      (void)hipStreamSynchronize(stream);
      release();
      return;
    }
    for (auto& e : ev) {
      event_put(device, true, e);
      e = nullptr;
    }
    event_put(device, false, ev_wait);
    ev_wait = nullptr;
    mem.release_async(stream);
  }
};

// FP64 mode on FP32 input keeps the panels in FP32 (ProbDesc::panel_f32):
// half the pack's writes and the Gram's panel reads, for an FP64 shift per
// loaded value on the vector units beside the FP64 MFMAs (the Gram launch
// measured 4.5 % slower, at K = 1024 and K = 4096 alike).  The pack is
// linear in K, the Gram quadratic, so FP32 panels pay up to about K = 2300
// (measured: K = 1024 gains 0.9 ms of 19.9, K = 4096 loses 10 ms of 537);
// they are taken while every problem has K <= kPanelF32MaxK.
constexpr int64_t kPanelF32MaxK = 2048;
bool panel_f32(const Batch& b) {
  if (b.mode != CVGRAM_MODE_FP64 || b.dtype != CVGRAM_F32) return false;
  for (const auto& p : b.pp)
    if (p.K > kPanelF32MaxK) return false;
  return true;
}
// pivots are FP32 values in the mixed modes (the FP32 shift is then exact
// for inputs within a factor 2 of it) and with FP32 panels (a padding row
// holds the pivot and shifts to exactly 0)
bool pivot_f32(const Batch& b) { return b.mode != CVGRAM_MODE_FP64 || panel_f32(b); }

int bit_length(uint32_t v) {
  int b = 0;
  while (v) {
    ++b;
    v >>= 1;
  }
  return b;
}

constexpr int64_t kPackTargetBlocks = 4096;  // pack workgroups (one wave each) to aim for
constexpr int64_t kGramMinRows = 256;

// Algorithm 1 on the device for every problem, with the checks of
// Definition 1 and Definition 6.  Fills P, offsets, scalable and d_perm.
cvgram_status bookkeeping(Batch& b) {
  hipStream_t s = b.stream;
  int64_t sumN = 0, maxN = 0;
  for (auto& p : b.pp) {
    sumN += p.N;
    maxN = std::max(maxN, p.N);
  }
  int32_t* perm_block = (int32_t*)b.mem.dev((size_t)sumN * sizeof(int32_t));
  Owned scratch;
  scratch.device = b.device;
  scratch.stream = s;
  scratch.arena = b.mem.arena;
  // the host's wait for the label counts: an event, or (fixed memory, where
  // no event is created) the whole stream
  const bool wait_stream = b.mem.arena != nullptr;
  // info[0] min label, info[1] max label, info[2 ..) counts of labels below
  // kCountLabels, then flags: one block, one initialising launch, one copy.
  // The block stays with the batch: the sort's scan reads the counts after
  // this function returns.
  constexpr int64_t kInfo = 2 + kCountLabels + 62;
  int32_t* info = (int32_t*)b.mem.dev(kInfo * sizeof(int32_t));
  int32_t* counts = info + 2;
  int32_t* flag = info + 2 + kCountLabels;
  // buffers of the sort stay with the batch: the sort still runs after this
  // function returns (only the validation data is waited for)
  int32_t* keys = (int32_t*)b.mem.dev((size_t)2 * maxN * sizeof(int32_t));
  int32_t* perm_tmp = (int32_t*)b.mem.dev((size_t)maxN * sizeof(int32_t));
  int32_t* hist = (int32_t*)b.mem.dev((size_t)radix_hist_entries(maxN) * sizeof(int32_t));
  int64_t* offs = (int64_t*)b.mem.dev((size_t)(maxN + 1) * sizeof(int64_t));
  int32_t* hbuf = (int32_t*)scratch.pinned(kInfo * sizeof(int32_t));
  int32_t* hcounts = hbuf + 2;
  if (!b.ev_wait && !wait_stream) b.ev_wait = event_get(b.device, false);
  cvgram_status st = CVGRAM_OK;
  int64_t at = 0;
  try {
    for (size_t i = 0; i < b.pp.size() && st == CVGRAM_OK; ++i) {
      ProbPlan& p = b.pp[i];
      const std::string tag = b.pp.size() > 1 ? "problem " + std::to_string(i) + ": " : "";
      p.d_perm = perm_block + at;
      at += p.N;
      launch_count_init(info, kInfo, s);
      launch_label_count(p.fold, p.N, info, counts, hist, s);
      CVG_HIP(hipMemcpyAsync(hbuf, info, (2 + kCountLabels) * sizeof(int32_t),
                             hipMemcpyDeviceToHost, s));
      if (!wait_stream) CVG_HIP(hipEventRecord(b.ev_wait, s));
      if (!b.batched) {
        // the pivots need only X and Y: they run while the host waits for the
        // counts and plans (a batch computes them inside its graph instead)
        p.d_pivot = (double*)b.mem.dev((size_t)p.W * sizeof(double));
        launch_pivot_direct(b.dtype, pivot_f32(b), p.X, p.Y, p.N, p.K, p.M,
                            p.d_pivot, s);
      }
      // the sort starts before the wait on the guess that the labels fit in
      // one 8-bit pass (P <= 256, where its result is exact); labels that
      // turn out wider are sorted again below.  Any label values keep the
      // early pass inside its buffers (it sorts by the low 8 bits).
      const int32_t* sorted = nullptr;
      constexpr int kEarlyBits = 8;
      radix_partition(p.fold, p.N, kEarlyBits, counts, keys, keys + maxN, p.d_perm, perm_tmp,
                      hist, true, &sorted, s);
      if (wait_stream)
        CVG_HIP(hipStreamSynchronize(s));
      else
        CVG_HIP(hipEventSynchronize(b.ev_wait));
      if (hbuf[0] < 0) {
        st = fail(CVGRAM_EFOLDS, tag + "fold label < 0 (Definition 1)");
        break;
      }
      const int64_t P = (int64_t)hbuf[1] + 1;
      if (P < 2) {
        st = fail(CVGRAM_EFOLDS, tag + "fewer than 2 folds (Definition 1)");
        break;
      }
      if (P > p.N) {
        st = fail(CVGRAM_EFOLDS, tag + "more folds than rows (Definition 1)");
        break;
      }
      p.P = (int32_t)P;
      const int bits = bit_length((uint32_t)(P - 1));
      if (bits > kEarlyBits)
        // the early pass scanned the histogram in place: count it again
        radix_partition(p.fold, p.N, bits, counts, keys, keys + maxN, p.d_perm, perm_tmp, hist,
                        false, &sorted, s);
      p.offsets.assign(P + 1, 0);
      bool empty = false;
      if (P <= kCountLabels) {
        // the fold sizes came with the first wait: no second one
        for (int64_t q = 0; q < P; ++q) {
          empty |= hcounts[q] == 0;
          p.offsets[q + 1] = p.offsets[q] + hcounts[q];
        }
      } else {
        launch_fold_offsets(sorted, p.N, (int32_t)P, offs, flag, s);
        CVG_HIP(hipMemcpyAsync(p.offsets.data(), offs, (P + 1) * sizeof(int64_t),
                               hipMemcpyDeviceToHost, s));
        CVG_HIP(hipMemcpyAsync(hbuf + 2 + kCountLabels, flag, sizeof(int32_t),
                               hipMemcpyDeviceToHost, s));
        CVG_HIP(hipStreamSynchronize(s));
        empty = hbuf[2 + kCountLabels] != 0;
      }
      if (empty) {
        st = fail(CVGRAM_EFOLDS, tag + "a fold label in [0, P) has no rows (Definition 1)");
        break;
      }
      int64_t max_fold = 0;
      for (int64_t q = 0; q < P; ++q) max_fold = std::max(max_fold, p.offsets[q + 1] - p.offsets[q]);
      p.scalable = (p.N - max_fold - b.ddof) >= 1;
    }
  } catch (const Fail& f) {
    (void)hipStreamSynchronize(s);
    scratch.release();
    throw;
  }
  // On success nothing enqueued after the last wait reads the scratch
  // (label counts, validation flags); on failure wait for the sorts before
  // the batch's memory is handed back.
  if (st != CVGRAM_OK) CVG_HIP(hipStreamSynchronize(s));
  scratch.release();
  return st;
}

// Layout of every problem and the flat work lists of every launch.
struct HostLists {
  std::vector<Item> pivot_items, fold_items, sr_items, fs_items, cb_items, range_items, red_items,
      corr_items;
  std::vector<PackChunk> chunks;
  std::vector<GramWork> work[kWidths];
  // per-XCD item ranges of each Gram launch (kXcds + 1 offsets each)
  std::vector<int32_t> xcd[kWidths];
  // empty every list, keeping its memory (the lists are reused per thread:
  // no allocation or first-touch page faults on the planning path)
  void clear() {
    for (auto* v : {&pivot_items, &fold_items, &sr_items, &fs_items, &cb_items, &range_items,
                    &red_items, &corr_items})
      v->clear();
    chunks.clear();
    for (int k = 0; k < kWidths; ++k) {
      work[k].clear();
      xcd[k].clear();
    }
  }
};

// Fold path of a problem.  The grouped path pads every fold to whole panels
// and keeps at least one K x (K + M) FP64 slab per fold; the fused path (no
// padding between folds) forms each G'_p inside the corrections instead,
// re-reading the fold's rows for every output tile (a cost that does not
// shrink with the folds).  Measured on N=1e5, K=512 (create + all folds):
// grouped is faster down to folds of 33 rows (P=3000: 10.3 vs 12.5 ms), the
// fused path from folds of about 20 rows on, where padding and per-fold
// slabs dominate.  The fused path is also taken when the per-fold slabs
// would not fit a memory budget.  CVGRAM_FOLD_PATH=grouped|fused forces
// either.
constexpr int64_t kFusedMaxFoldRows = 24;
constexpr int32_t kFusedMinFolds = 64;
constexpr double kGroupedSlabBudget = 16e9;  // bytes

bool choose_fused(const ProbPlan& p) {
  const char* f = std::getenv("CVGRAM_FOLD_PATH");
  if (f && std::strcmp(f, "fused") == 0) return true;
  if (f && std::strcmp(f, "grouped") == 0) return false;
  int64_t max_fold = 0;
  for (int32_t q = 0; q < p.P; ++q) max_fold = std::max(max_fold, p.offsets[q + 1] - p.offsets[q]);
  if (p.P >= kFusedMinFolds && max_fold <= kFusedMaxFoldRows) return true;
  return (double)p.P * (double)p.K * (double)p.W * 8.0 > kGroupedSlabBudget;
}

// Order of a Gram launch's items.  The kernel maps workgroup b to item
// xcd[b % 8] + b / 8 of XCD b % 8's range.  A single problem keeps the list
// order in 8 equal ranges (its items are of similar size; the tiles of one
// fold row range are consecutive, so they run on one XCD and share its L2).
// A batch mixes items of very different sizes: a unit is one fold row range
// of one problem with all its output tiles, units are taken longest first
// and each goes to the XCD with the least work so far (LPT), and an XCD runs
// its units longest first.  Reordering is free: every item writes its own
// slab, summed later in slab order.
// Estimated cost of one Gram item: its rows (plus about two panels for the
// first stage and the tile store) times the 16 x 16 blocks each wave
// computes per row step: 16 on a full tile; on a 128-wide diagonal tile 9 of
// the triangle plus the wave's X^T Y blocks.
int64_t gram_item_cost(const GramWork& w, const std::vector<ProbPlan>& pp) {
  const ProbPlan& p = pp[w.prob];
  int64_t blocks = 16;
  if (p.cfg.tile == 128 && w.ti == w.tj && w.tj < p.nt)
    blocks = 9 + 2 * (p.xy_diag ? (p.M <= 16 ? 1 : 2) : 0);
  if (p.cfg.tile == 256) blocks = 32;  // a 128 x 64 wave tile
  return (w.r1 - w.r0 + 2 * kPanelRows) * blocks;
}

// The last items an XCD starts decide when the launch ends: the final
// kTailPercent of every XCD's range run longest first, so that the launch
// ends on short items.  The rest keep list order (the tiles of one fold row
// range stay together and share the XCD's L2).
constexpr int kTailPercent = 30;
// single problems with at least kTileGroupMinNt tile columns visit their
// tiles in square groups, each group on one XCD (ProbPlan::tile_groups).
// Below that the per-XCD ranges keep a fold row range's tiles in one L2:
// measured with groups dealt item by item round-robin over the XCDs, the
// BF16X3 launch on K = 1024 slowed from 3.8 to 4.5 ms, and the FP64 launch
// on K = 512 gained 1 % while its L2 misses doubled (served by the
// memory-side cache).
constexpr int32_t kTileGroup = 8;
constexpr int32_t kTileGroupMinNt = 16;
void order_tails(std::vector<GramWork>& wl, const std::vector<int32_t>& xcd,
                 const std::vector<ProbPlan>& pp) {
  for (int x = 0; x < kXcds; ++x) {
    const int32_t b = xcd[x], e = xcd[x + 1];
    const int32_t k = e - (e - b) * kTailPercent / 100;
    std::stable_sort(wl.begin() + k, wl.begin() + e, [&](const GramWork& u, const GramWork& v) {
      return gram_item_cost(u, pp) > gram_item_cost(v, pp);
    });
  }
}

void schedule_gram(std::vector<GramWork>& wl, std::vector<int32_t>& xcd, bool balance,
                   const std::vector<ProbPlan>& pp) {
  xcd.assign(kXcds + 1, 0);
  if (wl.empty()) return;
  const int32_t n = (int32_t)wl.size();
  if (!balance) {
    const int32_t per = (n + kXcds - 1) / kXcds;
    for (int x = 0; x <= kXcds; ++x) xcd[x] = std::min(n, x * per);
    if (pp[0].tile_groups) {
      // whole tile groups per XCD: the items of one group (one fold row
      // range, at most 2 x 8 column blocks) run together on one XCD and
      // read their column blocks through its L2 once per group instead of
      // once per item.  Groups go in list order to the XCD with the least
      // work so far, so the XCDs stay on neighbouring groups of the same
      // rows (shared through the memory-side cache).
      const ProbPlan& p = pp[0];
      const int32_t ga = p.cfg.tile == 256 ? kTileGroup / 2 : kTileGroup;
      auto same_group = [&](const GramWork& u, const GramWork& v) {
        const int32_t gu = u.tj < p.nt ? u.tj / kTileGroup : -1;
        const int32_t gv = v.tj < p.nt ? v.tj / kTileGroup : -1;
        return u.slab == v.slab && u.ti / ga == v.ti / ga && gu == gv;
      };
      thread_local std::vector<int32_t> owner_tl;
      thread_local std::vector<GramWork> out_tl;
      std::vector<int32_t>& owner = owner_tl;
      owner.assign(wl.size(), 0);
      int64_t load[kXcds] = {};
      int32_t count[kXcds] = {};
      for (int32_t i = 0; i < n;) {
        int32_t j = i + 1;
        while (j < n && same_group(wl[j], wl[i])) ++j;
        int x = 0;
        for (int y = 1; y < kXcds; ++y)
          if (load[y] < load[x]) x = y;
        for (int32_t k = i; k < j; ++k) {
          owner[k] = x;
          load[x] += gram_item_cost(wl[k], pp);
        }
        count[x] += j - i;
        i = j;
      }
      for (int x = 0; x < kXcds; ++x) xcd[x + 1] = xcd[x] + count[x];
      std::vector<GramWork>& out = out_tl;
      out.resize(wl.size());
      int32_t fill[kXcds];
      for (int x = 0; x < kXcds; ++x) fill[x] = xcd[x];
      for (int32_t i = 0; i < n; ++i) out[fill[owner[i]]++] = wl[i];
      wl.swap(out);
    }
    order_tails(wl, xcd, pp);
    return;
  }
  struct Unit {
    int64_t cost;
    int32_t begin, end;
  };
  // scratch kept per thread (no allocation once warm)
  thread_local std::vector<Unit> units_tl;
  thread_local std::vector<GramWork> out_tl;
  std::vector<Unit>& units = units_tl;
  std::vector<GramWork>& out = out_tl;
  units.clear();
  for (int32_t i = 0; i < n;) {
    int32_t j = i + 1;
    while (j < n && wl[j].prob == wl[i].prob && wl[j].slab == wl[i].slab) ++j;
    // rows x tiles, plus a per-item allowance for the first stage and the
    // tile store (about two panels)
    units.push_back({(int64_t)(j - i) * (wl[i].r1 - wl[i].r0 + 2 * kPanelRows), i, j});
    i = j;
  }
  // longest first; ties in list order (a total order: deterministic)
  std::sort(units.begin(), units.end(), [](const Unit& a, const Unit& c) {
    return a.cost != c.cost ? a.cost > c.cost : a.begin < c.begin;
  });
  int64_t load[kXcds] = {};
  int32_t count[kXcds] = {};
  for (Unit& u : units) {
    int x = 0;
    for (int y = 1; y < kXcds; ++y)
      if (load[y] < load[x]) x = y;
    load[x] += u.cost;
    count[x] += u.end - u.begin;
    u.cost = x;  // the unit's XCD from here on
  }
  for (int x = 0; x < kXcds; ++x) xcd[x + 1] = xcd[x] + count[x];
  int32_t fill[kXcds];
  for (int x = 0; x < kXcds; ++x) fill[x] = xcd[x];
  out.resize(wl.size());
  for (const Unit& u : units) {
    const int x = (int)u.cost;
    for (int32_t i = u.begin; i < u.end; ++i) out[fill[x]++] = wl[i];
  }
  wl.swap(out);
  order_tails(wl, xcd, pp);
}

void plan_layout(Batch& b, HostLists& L) {
  const int64_t PR = kPanelRows;
  int64_t pack_cols_rows = 0;  // sum over problems of Np * column blocks
  // sum over problems of Np * items per row range, per Gram launch (each
  // tile width is launched apart, so each launch is split for its own work)
  int64_t gram_rows[kWidths] = {};
  for (auto& p : b.pp) {
    if (b.force_cfg) {
      // a candidate's tile width caps each problem's own widest one
      p.cfg = b.forced;
      p.cfg.tile = std::min(b.forced.tile, natural_tile(b.mode, p.K));
      if (p.cfg.tile == 256 && p.K < b.forced.wide_min_k) p.cfg.tile = 128;
    } else {
      p.cfg = choose_config(b.mode, b.dtype, p.K, p.M, p.N, p.P);
    }
    const int T = p.cfg.tile;
    p.fused = choose_fused(p);
    p.poff.assign(p.P + 1, 0);
    for (int32_t q = 0; q < p.P; ++q) {
      const int64_t n = p.offsets[q + 1] - p.offsets[q];
      p.poff[q + 1] = p.poff[q] + (p.fused ? n : (n + PR - 1) / PR * PR);
    }
    p.Np = (p.poff[p.P] + PR - 1) / PR * PR;
    // TB: width of a B block (the tile's columns); tile 256 pairs two
    // 128-wide row blocks (A 256 columns, B 128)
    const int TB = T == 256 ? 128 : T;
    p.Kp = (p.K + T - 1) / T * T;
    p.xy_diag = p.M > 0 && p.M <= kYDiagCols;
    p.Mp = p.M == 0 ? 0 : (p.xy_diag ? kYDiagCols : (p.M + TB - 1) / TB * TB);
    p.Wp = p.Kp + p.Mp;
    p.nt = (int32_t)(p.Kp / TB);
    p.tile_groups = b.pp.size() == 1 && p.nt >= kTileGroupMinNt;
    const int64_t nyt = p.xy_diag ? 0 : p.Mp / TB;
    const int64_t na = p.Kp / T;  // A blocks
    const int64_t ntile = T == 256 ? na * p.nt - na * (na - 1) + na * nyt
                                   : (int64_t)p.nt * (p.nt + 1) / 2 + (int64_t)p.nt * nyt;
    pack_cols_rows += p.Np * ((p.Wp + kPackCols - 1) / kPackCols);
    gram_rows[width_index(T)] += p.Np * ntile;
  }
  int64_t chunk_rows = (pack_cols_rows + kPackTargetBlocks - 1) / kPackTargetBlocks;
  chunk_rows = std::min((int64_t)kMaxChunkRows, std::max(PR, (chunk_rows + PR - 1) / PR * PR));

  for (size_t i = 0; i < b.pp.size(); ++i) {
    ProbPlan& p = b.pp[i];
    const int32_t pi = (int32_t)i;
    const int T = p.cfg.tile;
    // pivots
    for (int64_t cb = 0; cb < (p.W + 63) / 64; ++cb) L.pivot_items.push_back({pi, (int32_t)cb, 0});
    // pack chunks: whole panels of one fold (grouped path), or of the whole
    // packed row space (fused path: packed row d holds permuted row d)
    p.chunk_begin.assign(p.P + 1, 0);
    int32_t nch = 0;
    if (p.fused) {
      for (int64_t d = 0; d < p.Np; d += chunk_rows)
        L.chunks.push_back({pi, nch++, d, std::min(d + chunk_rows, p.Np), d, p.N});
    } else {
      for (int32_t q = 0; q < p.P; ++q) {
        p.chunk_begin[q] = nch;
        for (int64_t d = p.poff[q]; d < p.poff[q + 1]; d += chunk_rows)
          L.chunks.push_back({pi, nch++, d, std::min(d + chunk_rows, p.poff[q + 1]),
                              p.offsets[q] + (d - p.poff[q]), p.offsets[q + 1]});
      }
      p.chunk_begin[p.P] = nch;
    }
    p.n_chunks = nch;
    b.max_pack_cb = std::max<int32_t>(b.max_pack_cb, (int32_t)((p.Wp + kPackCols - 1) / kPackCols));
    // statistics
    for (int32_t q = 0; q < p.P; ++q) {
      L.fold_items.push_back({pi, q, 0});
      if (!p.fused) L.sr_items.push_back({pi, q, 0});
    }
    if (p.fused) {
      // consecutive folds per item, up to 256 folds or 2048 rows
      for (int32_t q = 0; q < p.P;) {
        int32_t e = q + 1;
        while (e < p.P && e - q < 256 && p.offsets[e + 1] - p.offsets[q] <= 2048) ++e;
        L.fs_items.push_back({pi, q, e});
        q = e;
      }
    }
    p.n_franges = (p.P + kFoldRange - 1) / kFoldRange;
    for (int64_t cb = 0; cb < (p.W + 63) / 64; ++cb) {
      L.cb_items.push_back({pi, (int32_t)cb, 0});
      for (int32_t r = 0; r < p.n_franges; ++r) L.range_items.push_back({pi, (int32_t)cb, r});
    }
    b.max_cb64 = std::max<int32_t>(b.max_cb64, (int32_t)((p.W + 63) / 64));
    b.max_cb256 = std::max<int32_t>(b.max_cb256, (int32_t)((p.W + 255) / 256));
    // Gram work: split folds along rows so the launch this problem joins
    // has about target_items items (shared over the problems of the batch
    // with the same tile width)
    std::vector<std::pair<int32_t, int32_t>> gtiles;
    const int64_t nyt = p.xy_diag ? 0 : p.Mp / (T == 256 ? 128 : T);
    if (T == 256) {
      // (A block ti of 256 columns, B block tj of 128) for tj >= 2 ti; with
      // many tiles in groups of 4 A blocks x 8 B blocks (the same column
      // span as the 8 x 8 groups of 128-wide tiles)
      const int32_t na = (int32_t)(p.Kp / 256);
      const int32_t ga = p.tile_groups ? kTileGroup / 2 : na;
      const int32_t gb = p.tile_groups ? kTileGroup : p.nt;
      for (int32_t ba = 0; ba * ga < na; ++ba) {
        const int32_t i0 = ba * ga, i1 = std::min(na, i0 + ga);
        for (int32_t bb = 0; bb * gb < p.nt; ++bb) {
          const int32_t j0 = bb * gb, j1 = std::min(p.nt, j0 + gb);
          for (int32_t ti = i0; ti < i1; ++ti)
            for (int32_t tj = std::max(2 * ti, j0); tj < j1; ++tj) gtiles.push_back({ti, tj});
        }
        for (int64_t y = 0; y < nyt; ++y)
          for (int32_t ti = i0; ti < i1; ++ti) gtiles.push_back({ti, (int32_t)(p.nt + y)});
      }
    } else if (!p.tile_groups) {
      for (int32_t ti = 0; ti < p.nt; ++ti) {
        for (int32_t tj = ti; tj < p.nt; ++tj) gtiles.push_back({ti, tj});
        for (int64_t y = 0; y < nyt; ++y) gtiles.push_back({ti, (int32_t)(p.nt + y)});
      }
    } else {
      // many tiles per fold row range: square groups of kTileGroup x
      // kTileGroup tiles, so that the items running together read few
      // distinct column blocks (2 kTileGroup for 64 tiles)
      const int32_t ng = (p.nt + kTileGroup - 1) / kTileGroup;
      for (int32_t bi = 0; bi < ng; ++bi) {
        const int32_t i0 = bi * kTileGroup, i1 = std::min(p.nt, i0 + kTileGroup);
        for (int32_t bj = bi; bj < ng; ++bj) {
          const int32_t j0 = bj * kTileGroup, j1 = std::min(p.nt, j0 + kTileGroup);
          for (int32_t ti = i0; ti < i1; ++ti)
            for (int32_t tj = std::max(ti, j0); tj < j1; ++tj) gtiles.push_back({ti, tj});
        }
        for (int64_t y = 0; y < nyt; ++y)
          for (int32_t ti = i0; ti < i1; ++ti) gtiles.push_back({ti, (int32_t)(p.nt + y)});
      }
    }
    const int64_t grows = gram_rows[width_index(T)];
    int64_t rows_per_split = (grows + p.cfg.target_items - 1) / p.cfg.target_items;
    rows_per_split = std::max(rows_per_split, kGramMinRows);
    rows_per_split = (rows_per_split + PR - 1) / PR * PR;
    auto& wl = L.work[width_index(T)];
    {
      // room for every item up front (no regrowth while appending)
      int64_t n_splits = 0;
      auto count_splits = [&](int64_t a, int64_t e) {
        const int64_t panels = (e - a) / PR;
        n_splits += std::min(panels, std::max<int64_t>(1, (e - a + rows_per_split - 1) / rows_per_split));
      };
      if (p.fused)
        count_splits(0, p.Np);
      else
        for (int32_t q = 0; q < p.P; ++q) count_splits(p.poff[q], p.poff[q + 1]);
      wl.reserve(wl.size() + (size_t)(n_splits * (int64_t)gtiles.size()));
    }
    p.slab_begin.assign(p.P + 1, 0);
    int32_t slab = 0;
    auto split_rows = [&](int64_t a, int64_t e) {
      const int64_t panels = (e - a) / PR;
      const int64_t splits =
          std::min(panels, std::max<int64_t>(1, (e - a + rows_per_split - 1) / rows_per_split));
      for (int64_t sp = 0; sp < splits; ++sp) {
        const int64_t r0 = a + panels * sp / splits * PR;
        const int64_t r1 = a + panels * (sp + 1) / splits * PR;
        for (auto& tt : gtiles) wl.push_back({pi, slab, tt.first, tt.second, r0, r1});
        ++slab;
      }
    };
    if (p.fused) {
      split_rows(0, p.Np);  // the full Gram only
    } else {
      for (int32_t q = 0; q < p.P; ++q) {
        p.slab_begin[q] = slab;
        split_rows(p.poff[q], p.poff[q + 1]);
      }
    }
    p.slab_begin[p.P] = slab;
    p.n_slabs = slab;
    // slab reduction
    const int64_t n_red = (p.K * p.W + kReduceElems - 1) / kReduceElems;
    L.red_items.reserve(L.red_items.size() + (size_t)n_red);
    for (int64_t eb = 0; eb < n_red; ++eb) L.red_items.push_back({pi, (int32_t)eb, 0});
    // correction tiles: upper triangle of X^T X, then X^T Y
    p.ctiles.clear();
    const int64_t nct = (p.K + kCorrTile - 1) / kCorrTile;
    for (int64_t bi = 0; bi < nct; ++bi)
      for (int64_t bj = bi; bj < nct; ++bj) {
        p.ctiles.push_back((int32_t)bi);
        p.ctiles.push_back((int32_t)bj);
      }
    p.n_ctiles_xx = (int32_t)(p.ctiles.size() / 2);
    const int64_t ncy = (p.M + kCorrTile - 1) / kCorrTile;
    for (int64_t bi = 0; bi < nct; ++bi)
      for (int64_t bj = 0; bj < ncy; ++bj) {
        p.ctiles.push_back((int32_t)bi);
        p.ctiles.push_back((int32_t)bj);
      }
    p.n_ctiles_xy = (int32_t)(p.ctiles.size() / 2) - p.n_ctiles_xx;
    if (b.batched)
      for (int32_t q = 0; q < p.P; ++q)
        for (int32_t tl = 0; tl < p.n_ctiles_xx + p.n_ctiles_xy; ++tl)
          L.corr_items.push_back({pi, q, tl});
  }
  for (int k = 0; k < kWidths; ++k) schedule_gram(L.work[k], L.xcd[k], b.pp.size() > 1, b.pp);
}

// the plan blob: segments at 256-byte aligned offsets.  Laid out twice:
// once with dst == nullptr to measure it, then straight into the pinned
// upload buffer (no intermediate copy).
struct Blob {
  char* dst = nullptr;
  size_t size = 0;
  template <typename T>
  size_t put(const T* data, size_t count, bool align = true) {
    const size_t off = align ? (size + 255) / 256 * 256 : size;
    size = off + count * sizeof(T);
    if (dst && count && data) std::memcpy(dst + off, data, count * sizeof(T));
    return off;
  }
  template <typename T>
  size_t put(const std::vector<T>& v, bool align = true) {
    return put(v.data(), v.size(), align);
  }
};

// bytes of one packed panel element; FP64 mode on FP32 panels (panel_f32,
// the same decision the pack and the Gram launch take) uses 4
size_t elem_bytes(const Batch& b) {
  if (b.mode == CVGRAM_MODE_FP64) return panel_f32(b) ? 4 : 8;
  return b.mode == CVGRAM_MODE_FP32 ? 4 : 2;
}

// Workspace arena of a planned batch: byte offsets of every problem's
// buffers (256-byte aligned) and the total.
struct ArenaOff {
  size_t pivot, packed, packed_lo, part, fold, tot, tot_part, tr_sum, tr_mean, tr_std, tr_mu,
      tr_const, ntrain, slabs, G;
};
size_t arena_layout(const Batch& b, std::vector<ArenaOff>& off) {
  const size_t eb = elem_bytes(b);
  off.assign(b.pp.size(), ArenaOff{});
  size_t total = 0;
  auto take_bytes = [&](size_t bytes) {
    const size_t o = total;
    total += (bytes + 255) / 256 * 256;
    return o;
  };
  for (size_t i = 0; i < b.pp.size(); ++i) {
    const ProbPlan& p = b.pp[i];
    ArenaOff& o = off[i];
    o.pivot = p.d_pivot ? 0 : take_bytes(p.W * 8);
    o.packed = take_bytes((size_t)p.Np * p.Wp * eb);
    o.packed_lo = b.mode == CVGRAM_MODE_BF16X3 ? take_bytes((size_t)p.Np * p.Wp * eb) : 0;
    o.part = take_bytes((size_t)4 * p.n_chunks * p.W * 8);
    o.fold = take_bytes((size_t)4 * p.P * p.W * 8);
    o.tot = take_bytes((size_t)8 * p.W * 8);
    o.tot_part = take_bytes((size_t)p.n_franges * 8 * p.W * 8);
    o.tr_sum = take_bytes((size_t)p.P * p.W * 8);
    o.tr_mean = take_bytes((size_t)p.P * p.W * 8);
    o.tr_std = take_bytes((size_t)p.P * p.W * 8);
    o.tr_mu = take_bytes((size_t)p.P * p.W * 8);
    o.tr_const = take_bytes((size_t)p.P * p.W);
    o.ntrain = take_bytes((size_t)p.P * 8);
    o.slabs = take_bytes((size_t)p.n_slabs * p.K * p.W * 8);
    o.G = take_bytes((size_t)p.K * p.W * 8);
  }
  return total;
}

// Workspace arena + device descriptors + one upload of every plan.
void allocate_and_upload(Batch& b, const HostLists& L) {
  std::vector<ArenaOff> off;
  const size_t total = arena_layout(b, off);
  char* arena = (char*)b.mem.dev(total);

  // plan blob: per-problem small arrays first, then descriptors and lists
  std::vector<size_t> o_offsets(b.pp.size()), o_poff(b.pp.size()), o_cbeg(b.pp.size()),
      o_sbeg(b.pp.size()), o_ctiles(b.pp.size());
  size_t o_pd = 0, o_out = 0, o_pivot = 0, o_chunks = 0, o_fold = 0, o_sr = 0, o_fs = 0,
         o_cb = 0, o_range = 0, o_work = 0, o_red = 0, o_corr = 0;
  size_t o_xcd[kWidths] = {};
  auto layout = [&](Blob& blob) {
    for (size_t i = 0; i < b.pp.size(); ++i) {
      o_offsets[i] = blob.put(b.pp[i].offsets);
      o_poff[i] = blob.put(b.pp[i].poff);
      o_cbeg[i] = blob.put(b.pp[i].chunk_begin);
      o_sbeg[i] = blob.put(b.pp[i].slab_begin);
      o_ctiles[i] = blob.put(b.pp[i].ctiles);
    }
    o_pd = blob.put((const ProbDesc*)nullptr, b.pp.size());
    o_out = blob.put((const OutDesc*)nullptr, b.pp.size());
    o_pivot = blob.put(L.pivot_items);
    o_chunks = blob.put(L.chunks);
    o_fold = blob.put(L.fold_items);
    o_sr = blob.put(L.sr_items);
    o_fs = blob.put(L.fs_items);
    o_cb = blob.put(L.cb_items);
    o_range = blob.put(L.range_items);
    o_work = blob.put(L.work[0]);
    for (int k = 1; k < kWidths; ++k) blob.put(L.work[k], false);  // one array
    o_red = blob.put(L.red_items);
    o_corr = blob.put(L.corr_items);
    for (int k = 0; k < kWidths; ++k) o_xcd[k] = blob.put(L.xcd[k]);
  };
  Blob measure;
  layout(measure);
  const size_t blob_bytes = measure.size;
  char* dblob = (char*)b.mem.dev(blob_bytes);
  // pinned upload buffer (kept until the batch is freed), written in place
  char* hb = (char*)b.mem.pinned(blob_bytes);
  Blob blob;
  blob.dst = hb;
  layout(blob);

  b.h_pd.assign(b.pp.size(), ProbDesc{});
  std::vector<OutDesc> outs(b.pp.size());
  for (size_t i = 0; i < b.pp.size(); ++i) {
    const ProbPlan& p = b.pp[i];
    const ArenaOff& o = off[i];
    ProbDesc& d = b.h_pd[i];
    std::memset(&d, 0, sizeof(d));
    d.X = p.X;
    d.Y = p.Y;
    d.N = p.N;
    d.K = p.K;
    d.M = p.M;
    d.W = p.W;
    d.Kp = p.Kp;
    d.Wp = p.Wp;
    d.Np = p.Np;
    d.P = p.P;
    d.tile = p.cfg.tile;
    d.nt = p.nt;
    d.xy_diag = p.xy_diag ? 1 : 0;
    d.ddof = b.ddof;
    d.x_vec = (p.K % 4 == 0) && ((uintptr_t)p.X % 16 == 0) ? 1 : 0;
    d.mode = (int32_t)b.mode;
    d.panel_f32 = panel_f32(b) ? 1 : 0;
    d.fused = p.fused ? 1 : 0;
    d.n_slabs = (int32_t)p.n_slabs;
    d.perm = p.d_perm;
    d.offsets = (const int64_t*)(dblob + o_offsets[i]);
    d.poff = (const int64_t*)(dblob + o_poff[i]);
    d.pivot = p.d_pivot ? p.d_pivot : (double*)(arena + o.pivot);
    d.packed = arena + o.packed;
    d.packed_lo = b.mode == CVGRAM_MODE_BF16X3 ? arena + o.packed_lo : nullptr;
    d.part = (double*)(arena + o.part);
    d.n_chunks = p.n_chunks;
    d.chunk_begin = (const int32_t*)(dblob + o_cbeg[i]);
    d.fold = (double*)(arena + o.fold);
    d.tot = (double*)(arena + o.tot);
    d.tot_part = (double*)(arena + o.tot_part);
    d.n_franges = p.n_franges;
    d.tr_sum = (double*)(arena + o.tr_sum);
    d.tr_mean = (double*)(arena + o.tr_mean);
    d.tr_std = (double*)(arena + o.tr_std);
    d.tr_mu = (double*)(arena + o.tr_mu);
    d.tr_const = (uint8_t*)(arena + o.tr_const);
    d.ntrain = (int64_t*)(arena + o.ntrain);
    d.slabs = (double*)(arena + o.slabs);
    d.slab_begin = (const int32_t*)(dblob + o_sbeg[i]);
    d.G = (double*)(arena + o.G);
    d.ctiles = (const int32_t*)(dblob + o_ctiles[i]);
    d.n_ctiles_xx = p.n_ctiles_xx;
    d.n_ctiles_xy = p.n_ctiles_xy;
    // batched outputs: every fold, all 12 classes
    OutDesc& od = outs[i];
    std::memset(&od, 0, sizeof(od));
    const size_t ob = b.mode == CVGRAM_MODE_FP64 ? 8 : 4;
    const int64_t KK = p.K * p.K, KM = p.K * p.M;
    // every class is written; a fold whose |T_p| - ddof < 1 has NaN
    // deviations, so its scaled classes come out NaN
    for (int c = 0; c < CVGRAM_XTX_CLASSES; ++c)
      od.xx[c] = p.out_xx ? (char*)p.out_xx + c * KK * ob : nullptr;
    for (int c = 0; c < CVGRAM_XTY_CLASSES; ++c)
      od.xy[c] = (p.out_xy && p.M > 0) ? (char*)p.out_xy + c * KM * ob : nullptr;
    od.fold_stride_xx = CVGRAM_XTX_CLASSES * KK;
    od.fold_stride_xy = CVGRAM_XTY_CLASSES * KM;
    od.p_begin = 0;
  }
  std::memcpy(hb + o_pd, b.h_pd.data(), b.h_pd.size() * sizeof(ProbDesc));
  std::memcpy(hb + o_out, outs.data(), outs.size() * sizeof(OutDesc));

  b.d_pd = (ProbDesc*)(dblob + o_pd);
  b.d_out = (OutDesc*)(dblob + o_out);
  b.d_pivot_items = (Item*)(dblob + o_pivot);
  b.n_pivot_items = (int64_t)L.pivot_items.size();
  b.d_chunks = (PackChunk*)(dblob + o_chunks);
  b.n_chunks = (int64_t)L.chunks.size();
  b.d_fold_items = (Item*)(dblob + o_fold);
  b.n_fold_items = (int64_t)L.fold_items.size();
  b.d_sr_items = (Item*)(dblob + o_sr);
  b.n_sr_items = (int64_t)L.sr_items.size();
  b.d_fs_items = (Item*)(dblob + o_fs);
  b.n_fs_items = (int64_t)L.fs_items.size();
  b.d_cb_items = (Item*)(dblob + o_cb);
  b.n_cb_items = (int64_t)L.cb_items.size();
  b.d_range_items = (Item*)(dblob + o_range);
  b.n_range_items = (int64_t)L.range_items.size();
  b.d_work = (GramWork*)(dblob + o_work);
  for (int k = 0; k < kWidths; ++k) {
    b.n_work[k] = (int64_t)L.work[k].size();
    b.d_xcd[k] = (int32_t*)(dblob + o_xcd[k]);
  }
  auto widest = [](const std::vector<int32_t>& x) {
    int64_t m = 0;
    for (size_t i = 0; i + 1 < x.size(); ++i) m = std::max<int64_t>(m, x[i + 1] - x[i]);
    return m;
  };
  for (int k = 0; k < kWidths; ++k) b.grid[k] = widest(L.xcd[k]);
  b.d_red_items = (Item*)(dblob + o_red);
  b.n_red_items = (int64_t)L.red_items.size();
  b.d_corr_items = (Item*)(dblob + o_corr);
  b.n_corr_items = (int64_t)L.corr_items.size();

  // one asynchronous upload from pinned memory
  CVG_HIP(hipMemcpyAsync(dblob, hb, blob_bytes, hipMemcpyHostToDevice, b.stream));
}

// The device pipeline (Algorithm 7 steps 3-4, 8, 10, 17, 19 and, for a
// batch, steps 9, 11-16, 18, 20-27 for every fold and class).
void run_pipeline(Batch& b, bool with_events) {
  hipStream_t s = b.stream;
  auto mark = [&](int k) {
    if (with_events && b.timing) CVG_HIP(hipEventRecord(b.ev[k], s));
  };
  mark(1);
  if (b.batched) launch_pivot(b.dtype, pivot_f32(b), b.d_pd, b.d_pivot_items, b.n_pivot_items, s);
  launch_pack(b.mode, b.dtype, b.d_pd, b.d_chunks, b.n_chunks, b.max_pack_cb, s);
  launch_stats_reduce(b.d_pd, b.d_sr_items, b.n_sr_items, b.max_cb64, s);
  launch_fold_sums_rows(b.dtype, b.d_pd, b.d_fs_items, b.n_fs_items, b.max_cb64, s);
  launch_fold_totals(b.d_pd, b.d_range_items, b.n_range_items, b.d_cb_items, b.n_cb_items, s);
  launch_train_stats(b.d_pd, b.d_fold_items, b.n_fold_items, b.max_cb256, s);
  mark(2);
  int64_t first = 0;
  for (int k = 0; k < kWidths; ++k) {
    launch_gram(b.mode, panel_f32(b), kWidth[k], b.d_pd, b.d_work + first, b.d_xcd[k], b.grid[k],
                s);
    first += b.n_work[k];
  }
  mark(3);
  launch_reduce_slabs(b.d_pd, b.d_red_items, b.n_red_items, s);
  if (b.batched)
    launch_correct_batch(b.d_pd, b.d_out, b.d_corr_items, b.n_corr_items,
                         b.mode == CVGRAM_MODE_FP64, s);
  mark(4);
}

// bookkeeping + plan + workspace for a batch whose problems are filled in
cvgram_status prepare(Batch& b) {
  if (b.timing)
    for (auto& e : b.ev)
      if (!e) e = event_get(b.device, true);
  if (b.timing) CVG_HIP(hipEventRecord(b.ev[0], b.stream));
  b.mem.device = b.device;
  b.mem.stream = b.stream;
  cvgram_status st = bookkeeping(b);
  if (st != CVGRAM_OK) return st;
  thread_local HostLists L;
  L.clear();
  plan_layout(b, L);
  allocate_and_upload(b, L);
  return CVGRAM_OK;
}

bool flag01(int v) { return v == 0 || v == 1; }

cvgram_status check_shape(int64_t N, int64_t K, int64_t M) {
  if (N < 2 || K < 1 || M < 0) return fail(CVGRAM_EINVAL, "need N >= 2, K >= 1, M >= 0");
  if (N > (int64_t)INT32_MAX - 1) return fail(CVGRAM_EINVAL, "N must fit in int32");
  if (K > (int64_t)1 << 24 || M > (int64_t)1 << 24) return fail(CVGRAM_EINVAL, "K or M too large");
  return CVGRAM_OK;
}

cvgram_status check_problem(const void* X, const void* Y, const int32_t* fold, int64_t N,
                            int64_t K, int64_t M) {
  if (!X || !fold) return fail(CVGRAM_EINVAL, "X or fold_id is NULL");
  if (M > 0 && !Y) return fail(CVGRAM_EINVAL, "Y is NULL with M > 0");
  if (N < 2 || K < 1 || M < 0) return fail(CVGRAM_EINVAL, "need N >= 2, K >= 1, M >= 0");
  if (N > (int64_t)INT32_MAX - 1) return fail(CVGRAM_EINVAL, "N must fit in int32");
  if (K > (int64_t)1 << 24 || M > (int64_t)1 << 24) return fail(CVGRAM_EINVAL, "K or M too large");
  return CVGRAM_OK;
}

}  // namespace
}  // namespace cvg

using namespace cvg;

// a single problem: a batch of one, plus the combination asked for at create
struct cvgram_handle {
  Batch b;
  int cx = 0, sx = 0, cy = 0, sy = 0;
};

struct cvgram_batch {
  Batch b;
};

namespace {

bool out_is_f64(const Batch& b) { return b.mode == CVGRAM_MODE_FP64; }

cvgram_status correct_single(const Batch& b, int32_t p0, int32_t p1, const OutDesc& od) {
  const ProbDesc& d = b.h_pd[0];
  try {
    launch_correct_single(b.d_pd, 0, d.n_ctiles_xx + d.n_ctiles_xy, od, p1 - p0,
                          out_is_f64(b), b.stream);
  } catch (const Fail& f) {
    return f.st;
  }
  return CVGRAM_OK;
}
cvgram_status correct_single(cvgram_t h, int32_t p0, int32_t p1, const OutDesc& od) {
  return correct_single(h->b, p0, p1, od);
}

// outputs of every class of folds p_begin, p_begin + 1, ...:
// [fold][class][K][K] and [fold][class][K][M]; scaled classes of folds with
// |T_p| - ddof < 1 come out NaN
OutDesc all_classes_out(const Batch& b, int32_t p_begin, void* out_XtX, void* out_XtY) {
  const ProbPlan& pp = b.pp[0];
  OutDesc od;
  std::memset(&od, 0, sizeof(od));
  const size_t es = out_is_f64(b) ? sizeof(double) : sizeof(float);
  const int64_t KK = pp.K * pp.K, KM = pp.K * pp.M;
  for (int c = 0; c < CVGRAM_XTX_CLASSES; ++c)
    od.xx[c] = out_XtX ? (char*)out_XtX + c * KK * es : nullptr;
  for (int c = 0; c < CVGRAM_XTY_CLASSES; ++c)
    od.xy[c] = (out_XtY && pp.M > 0) ? (char*)out_XtY + c * KM * es : nullptr;
  od.fold_stride_xx = CVGRAM_XTX_CLASSES * KK;
  od.fold_stride_xy = CVGRAM_XTY_CLASSES * KM;
  od.p_begin = p_begin;
  return od;
}

}  // namespace

// C++ exceptions never cross the C ABI: the body of every entry point that
// returns a status is a function-try-block ending in these handlers (a
// failure inside the library's own try blocks is reported there first).
#define CVG_ABI_CATCH                                                           \
  catch (const Fail& f) {                                                       \
    return f.st;                                                                \
  }                                                                             \
  catch (const std::bad_alloc&) {                                               \
    return fail(CVGRAM_ENOMEM, "host memory allocation failed");               \
  }                                                                             \
  catch (const std::exception& e) {                                             \
    return fail(CVGRAM_EINVAL, std::string("internal error: ") + e.what());    \
  }

extern "C" {

cvgram_status cvgram_create(const void* X, const void* Y, const int32_t* fold_id, int64_t N,
                            int64_t K, int64_t M, cvgram_dtype dtype, int center_x, int scale_x,
                            int center_y, int scale_y, int ddof, cvgram_mode mode, void* stream,
                            cvgram_t* out) try {
  set_error("");
  if (!out) return fail(CVGRAM_EINVAL, "out is NULL");
  *out = nullptr;
  cvgram_status st = check_problem(X, Y, fold_id, N, K, M);
  if (st != CVGRAM_OK) return st;
  if (dtype != CVGRAM_F32 && dtype != CVGRAM_F64) return fail(CVGRAM_EINVAL, "bad dtype");
  if (mode != CVGRAM_MODE_FP64 && mode != CVGRAM_MODE_FP32 && mode != CVGRAM_MODE_BF16X3)
    return fail(CVGRAM_EINVAL, "bad mode");
  if (!flag01(center_x) || !flag01(scale_x) || !flag01(center_y) || !flag01(scale_y))
    return fail(CVGRAM_EINVAL, "centering/scaling flags must be 0 or 1");
  if (ddof != 0 && ddof != 1) return fail(CVGRAM_EINVAL, "ddof must be 0 or 1");

  std::unique_ptr<cvgram_handle> h(new cvgram_handle());
  Batch& b = h->b;
  b.stream = (hipStream_t)stream;
  b.mode = mode;
  b.dtype = dtype;
  b.ddof = ddof;
  b.batched = false;
  b.timing = g_stage_timing.load() != 0;
  h->cx = center_x;
  h->sx = scale_x;
  h->cy = center_y;
  h->sy = scale_y;
  ProbPlan p;
  p.X = X;
  p.Y = M > 0 ? Y : nullptr;
  p.fold = fold_id;
  p.N = N;
  p.K = K;
  p.M = M;
  p.W = K + M;
  b.pp.push_back(p);
  try {
    CVG_HIP(hipGetDevice(&b.device));
    st = prepare(b);
    if (st == CVGRAM_OK && (scale_x || scale_y) && !b.pp[0].scalable)
      st = fail(CVGRAM_ENOTSCALABLE,
                "scaling needs |T_p| - ddof >= 1 for every fold (Definition 6)");
    if (st == CVGRAM_OK) run_pipeline(b, true);
  } catch (const Fail& f) {
    st = f.st;
  }
  if (st != CVGRAM_OK) {
    (void)hipStreamSynchronize(b.stream);
    b.release();
    return st;
  }
  *out = h.release();
  return CVGRAM_OK;
} CVG_ABI_CATCH

int32_t cvgram_num_folds(cvgram_t h) {
  if (!h) {
    set_error("NULL handle");
    return -1;
  }
  return h->b.pp[0].P;
}

cvgram_status cvgram_partition(cvgram_t h, int32_t* perm, int64_t* offsets) try {
  if (!h) return fail(CVGRAM_EINVAL, "NULL handle");
  const ProbPlan& p = h->b.pp[0];
  try {
    if (perm)
      CVG_HIP(hipMemcpyAsync(perm, p.d_perm, p.N * sizeof(int32_t), hipMemcpyDeviceToDevice,
                             h->b.stream));
    if (offsets)
      CVG_HIP(hipMemcpyAsync(offsets, h->b.h_pd[0].offsets, (p.P + 1) * sizeof(int64_t),
                             hipMemcpyDeviceToDevice, h->b.stream));
  } catch (const Fail& f) {
    return f.st;
  }
  return CVGRAM_OK;
} CVG_ABI_CATCH

cvgram_status cvgram_fold_combo(cvgram_t h, int32_t p, int center_x, int scale_x, int center_y,
                                int scale_y, void* out_XtX, void* out_XtY) try {
  if (!h) return fail(CVGRAM_EINVAL, "NULL handle");
  const ProbPlan& pp = h->b.pp[0];
  if (p < 0 || p >= pp.P) return fail(CVGRAM_ERANGE, "fold index out of range");
  if (!flag01(center_x) || !flag01(scale_x) || !flag01(center_y) || !flag01(scale_y))
    return fail(CVGRAM_EINVAL, "centering/scaling flags must be 0 or 1");
  if ((scale_x || scale_y) && !pp.scalable)
    return fail(CVGRAM_ENOTSCALABLE, "partitioning is not scalable for this ddof");
  OutDesc od;
  std::memset(&od, 0, sizeof(od));
  od.xx[2 * center_x + scale_x] = out_XtX;
  if (pp.M > 0) od.xy[4 * (center_x | center_y) + 2 * scale_x + scale_y] = out_XtY;
  od.p_begin = p;
  return correct_single(h, p, p + 1, od);
} CVG_ABI_CATCH

cvgram_status cvgram_fold_leaky(cvgram_t h, int32_t p, int kind, void* out_XtX, void* out_XtY) try {
  if (!h) return fail(CVGRAM_EINVAL, "NULL handle");
  const ProbPlan& pp = h->b.pp[0];
  if (p < 0 || p >= pp.P) return fail(CVGRAM_ERANGE, "fold index out of range");
  if (kind != CVGRAM_LEAK_GLOBAL && kind != CVGRAM_LEAK_LINDGREN)
    return fail(CVGRAM_EINVAL, "unknown leakage comparison kind");
  if (kind == CVGRAM_LEAK_LINDGREN && !(h->cx && !h->sx && h->cy && !h->sy))
    return fail(CVGRAM_EINVAL,
                "the Lindgren comparison needs the handle's combination center_x = center_y = 1, "
                "no scaling");
  OutDesc od;
  std::memset(&od, 0, sizeof(od));
  od.xx[0] = out_XtX;
  if (pp.M > 0) od.xy[0] = out_XtY;
  od.p_begin = p;
  od.leak = kind;
  od.lcx = h->cx;
  od.lsx = h->sx;
  od.lcy = h->cy;
  od.lsy = h->sy;
  return correct_single(h, p, p + 1, od);
} CVG_ABI_CATCH

cvgram_status cvgram_ridge(cvgram_t h, int32_t p0, int32_t p1, const double* lambdas,
                           int32_t n_lambda, double* out_B) try {
  if (!h) return fail(CVGRAM_EINVAL, "NULL handle");
  const ProbPlan& pp = h->b.pp[0];
  if (p0 < 0 || p1 > pp.P || p0 >= p1) return fail(CVGRAM_ERANGE, "fold range out of range");
  if (pp.M <= 0) return fail(CVGRAM_EINVAL, "ridge regression needs M > 0");
  if (!lambdas || !out_B || n_lambda < 1) return fail(CVGRAM_EINVAL, "lambdas / out_B / n_lambda");
  for (int32_t l = 0; l < n_lambda; ++l)
    if (!(lambdas[l] >= 0.0) || !std::isfinite(lambdas[l]))
      return fail(CVGRAM_EINVAL, "lambda must be finite and >= 0");
  if ((h->sx || h->sy) && !pp.scalable)
    return fail(CVGRAM_ENOTSCALABLE, "partitioning is not scalable for this ddof");
  const int32_t nf = p1 - p0;
  const int64_t K = pp.K, M = pp.M, nmat = (int64_t)nf * n_lambda;
  const int64_t Kp = ridge_padded_k(K), Mp = (M + 31) / 32 * 32;
  hipStream_t s = h->b.stream;
  Owned ws;
  ws.device = h->b.device;
  ws.stream = h->b.stream;
  cvgram_status st = CVGRAM_OK;
  try {
    double* xtx = (double*)ws.dev((size_t)nf * K * K * 8);
    double* xty = (double*)ws.dev((size_t)nf * K * M * 8);
    double* A = (double*)ws.dev((size_t)nmat * (Kp + ridge_aug_rows(M)) * Kp * 8);
    double* R = ridge_solve_on_matrix_cores(Kp, M) ? nullptr
                                                    : (double*)ws.dev((size_t)nmat * Kp * Mp * 8);
    double* Linv = (double*)ws.dev((size_t)nmat * Kp * 96 * 8);
    int32_t* flags = (int32_t*)ws.dev((size_t)nmat * 4);  // zeroed by the factorisation
    int32_t* hflags = (int32_t*)ws.pinned((size_t)nmat * 4);
    // the penalties by value in the kernel arguments, or (many) copied over
    RidgeLambdas lv;
    std::memset(&lv, 0, sizeof(lv));
    double* dl = nullptr;
    if (n_lambda <= kRidgeLambdaArgs) {
      std::memcpy(lv.v, lambdas, (size_t)n_lambda * 8);
    } else {
      dl = (double*)ws.dev((size_t)n_lambda * 8);
      double* hl = (double*)ws.pinned((size_t)n_lambda * 8);
      std::memcpy(hl, lambdas, (size_t)n_lambda * 8);
      CVG_HIP(hipMemcpyAsync(dl, hl, (size_t)n_lambda * 8, hipMemcpyHostToDevice, s));
    }
    // the handle's combination of folds [p0, p1) in FP64, fold-major
    OutDesc od;
    std::memset(&od, 0, sizeof(od));
    od.xx[2 * h->cx + h->sx] = xtx;
    od.xy[4 * (h->cx | h->cy) + 2 * h->sx + h->sy] = xty;
    od.fold_stride_xx = K * K;
    od.fold_stride_xy = K * M;
    od.p_begin = p0;
    const ProbDesc& d = h->b.h_pd[0];
    launch_correct_single(h->b.d_pd, 0, d.n_ctiles_xx + d.n_ctiles_xy, od, nf, true, s);
    ridge_solve(xtx, xty, lv, dl, nf, n_lambda, K, M, A, R, Linv, flags, out_B, s);
    CVG_HIP(hipMemcpyAsync(hflags, flags, (size_t)nmat * 4, hipMemcpyDeviceToHost, s));
    CVG_HIP(hipStreamSynchronize(s));
    for (int64_t m = 0; m < nmat; ++m)
      if (hflags[m]) {
        st = fail(CVGRAM_ESINGULAR, "fold " + std::to_string(p0 + m / n_lambda) + ", lambda " +
                                        std::to_string(lambdas[m % n_lambda]) +
                                        ": X^T X_T + lambda I is not positive definite");
        break;
      }
  } catch (const Fail& f) {
    (void)hipStreamSynchronize(s);
    ws.release();
    return f.st;
  }
  ws.release();
  return st;
} CVG_ABI_CATCH

cvgram_status cvgram_fold(cvgram_t h, int32_t p, void* out_XtX, void* out_XtY) try {
  if (!h) return fail(CVGRAM_EINVAL, "NULL handle");
  return cvgram_fold_combo(h, p, h->cx, h->sx, h->cy, h->sy, out_XtX, out_XtY);
} CVG_ABI_CATCH

cvgram_status cvgram_folds_all(cvgram_t h, int32_t p_begin, int32_t p_end, void* out_XtX,
                               void* out_XtY) try {
  if (!h) return fail(CVGRAM_EINVAL, "NULL handle");
  const ProbPlan& pp = h->b.pp[0];
  if (p_begin < 0 || p_end > pp.P || p_begin > p_end)
    return fail(CVGRAM_ERANGE, "fold range out of bounds");
  if (p_begin == p_end) return CVGRAM_OK;
  return correct_single(h->b, p_begin, p_end, all_classes_out(h->b, p_begin, out_XtX, out_XtY));
} CVG_ABI_CATCH

cvgram_status cvgram_fold_stats(cvgram_t h, int32_t p, double* mean_x, double* std_x,
                                double* mean_y, double* std_y) try {
  if (!h) return fail(CVGRAM_EINVAL, "NULL handle");
  const ProbDesc& d = h->b.h_pd[0];
  if (p < 0 || p >= d.P) return fail(CVGRAM_ERANGE, "fold index out of range");
  try {
    launch_fold_stats(d.tr_mu, d.tr_std, p, d.K, d.M, mean_x, std_x, mean_y, std_y, h->b.stream);
  } catch (const Fail& f) {
    return f.st;
  }
  return CVGRAM_OK;
} CVG_ABI_CATCH

cvgram_status cvgram_set_stage_timing(int on) try {
  g_stage_timing.store(on ? 1 : 0);
  return CVGRAM_OK;
} CVG_ABI_CATCH

cvgram_status cvgram_stage_times(cvgram_t h, double* ms, int32_t n) try {
  if (!h || (!ms && n > 0)) return fail(CVGRAM_EINVAL, "NULL argument");
  if (!h->b.timing) return fail(CVGRAM_EINVAL, "handle created without stage timing");
  try {
    CVG_HIP(hipEventSynchronize(h->b.ev[4]));
    for (int k = 0; k < 4 && k < n; ++k) {
      float t = 0.f;
      CVG_HIP(hipEventElapsedTime(&t, h->b.ev[k], h->b.ev[k + 1]));
      ms[k] = t;
    }
  } catch (const Fail& f) {
    return f.st;
  }
  return CVGRAM_OK;
} CVG_ABI_CATCH

cvgram_status cvgram_trim_cache(void) try {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(CVGRAM_EDEVICE, "hipGetDevice failed");
  cache_trim_dev(dev);
  return CVGRAM_OK;
} CVG_ABI_CATCH

cvgram_status cvgram_plan_info(cvgram_t h, int64_t* info, int32_t n) try {
  if (!h || (!info && n > 0)) return fail(CVGRAM_EINVAL, "NULL argument");
  const Batch& b = h->b;
  const ProbPlan& p = b.pp[0];
  const int64_t v[5] = {p.cfg.tile, b.n_work[0] + b.n_work[1] + b.n_work[2], p.n_slabs,
                        p.fused ? 1 : 0, (int64_t)elem_bytes(b)};
  for (int32_t k = 0; k < n && k < 5; ++k) info[k] = v[k];
  return CVGRAM_OK;
} CVG_ABI_CATCH

cvgram_status cvgram_plan_query(int64_t N, int64_t K, int64_t M, const int64_t* fold_sizes,
                                int32_t P, cvgram_dtype dtype, cvgram_mode mode, int64_t* info,
                                int32_t n) try {
  set_error("");
  if (!info && n > 0) return fail(CVGRAM_EINVAL, "NULL info");
  cvgram_status st = check_shape(N, K, M);
  if (st != CVGRAM_OK) return st;
  if (dtype != CVGRAM_F32 && dtype != CVGRAM_F64) return fail(CVGRAM_EINVAL, "bad dtype");
  if (mode != CVGRAM_MODE_FP64 && mode != CVGRAM_MODE_FP32 && mode != CVGRAM_MODE_BF16X3)
    return fail(CVGRAM_EINVAL, "bad mode");
  if (!fold_sizes || P < 1) return fail(CVGRAM_EINVAL, "need fold sizes and P >= 1");
  Batch b;
  b.mode = mode;
  b.dtype = dtype;
  b.ddof = 1;
  ProbPlan p;
  p.N = N;
  p.K = K;
  p.M = M;
  p.W = K + M;
  p.P = P;
  p.offsets.assign((size_t)P + 1, 0);
  for (int32_t q = 0; q < P; ++q) {
    if (fold_sizes[q] < 1)
      return fail(CVGRAM_EFOLDS, "fold " + std::to_string(q) + " is empty (Definition 1)");
    p.offsets[q + 1] = p.offsets[q] + fold_sizes[q];
  }
  if (p.offsets[P] != N) return fail(CVGRAM_EINVAL, "fold sizes do not sum to N");
  b.pp.push_back(std::move(p));
  try {
    HostLists L;
    L.clear();
    plan_layout(b, L);
    std::vector<ArenaOff> off;
    const size_t bytes = arena_layout(b, off);
    int64_t items = 0, most = -1, xmax = 0, xmin = 0;
    for (int k = 0; k < kWidths; ++k) {
      const int64_t nk = (int64_t)L.work[k].size();
      items += nk;
      if (nk > most && (int)L.xcd[k].size() == kXcds + 1) {
        most = nk;
        xmax = 0;
        xmin = INT64_MAX;
        for (int x = 0; x < kXcds; ++x) {
          const int64_t c = L.xcd[k][x + 1] - L.xcd[k][x];
          xmax = std::max(xmax, c);
          xmin = std::min(xmin, c);
        }
      }
    }
    const ProbPlan& q = b.pp[0];
    const int64_t v[8] = {q.cfg.tile, items, q.n_slabs, q.fused ? 1 : 0, (int64_t)elem_bytes(b),
                          (int64_t)bytes, xmax, xmin};
    for (int32_t k = 0; k < n && k < 8; ++k) info[k] = v[k];
  } catch (const Fail& f) {
    return f.st;
  }
  return CVGRAM_OK;
} CVG_ABI_CATCH

cvgram_status cvgram_set_stream(cvgram_t h, void* stream) try {
  if (!h) return fail(CVGRAM_EINVAL, "NULL handle");
  hipStream_t ns = (hipStream_t)stream;
  if (ns != h->b.stream) {
    // later work on the new stream (and the stream-ordered release at
    // destroy) comes after everything queued on the old one
    try {
      hipEvent_t e = event_get(h->b.device, false);
      const hipError_t r1 = hipEventRecord(e, h->b.stream);
      const hipError_t r2 = r1 == hipSuccess ? hipStreamWaitEvent(ns, e, 0) : r1;
      event_put(h->b.device, false, e);
      if (r2 != hipSuccess) return fail(CVGRAM_EDEVICE, hipGetErrorString(r2));
    } catch (const Fail& f) {
      return f.st;
    }
    h->b.stream = ns;
    h->b.mem.stream = ns;
  }
  return CVGRAM_OK;
} CVG_ABI_CATCH

cvgram_status cvgram_destroy(cvgram_t h) try {
  if (!h) return CVGRAM_OK;
  h->b.release_async();
  delete h;
  return CVGRAM_OK;
} CVG_ABI_CATCH

// ---------------------------------------------------------------------------
// batched form
// ---------------------------------------------------------------------------
cvgram_status cvgram_batch_create(const cvgram_problem* problems, int32_t n, cvgram_dtype dtype,
                                  int ddof, cvgram_mode mode, void* stream, cvgram_batch_t* out) try {
  set_error("");
  if (!out) return fail(CVGRAM_EINVAL, "out is NULL");
  *out = nullptr;
  if (!problems || n < 1) return fail(CVGRAM_EINVAL, "need at least one problem");
  if (dtype != CVGRAM_F32 && dtype != CVGRAM_F64) return fail(CVGRAM_EINVAL, "bad dtype");
  if (mode != CVGRAM_MODE_FP64 && mode != CVGRAM_MODE_FP32 && mode != CVGRAM_MODE_BF16X3)
    return fail(CVGRAM_EINVAL, "bad mode");
  if (ddof != 0 && ddof != 1) return fail(CVGRAM_EINVAL, "ddof must be 0 or 1");
  for (int32_t i = 0; i < n; ++i) {
    const cvgram_problem& q = problems[i];
    cvgram_status st = check_problem(q.X, q.Y, q.fold_id, q.N, q.K, q.M);
    if (st != CVGRAM_OK) return fail(st, "problem " + std::to_string(i) + ": " + g_last_error);
  }
  std::unique_ptr<cvgram_batch> bb(new cvgram_batch());
  Batch& b = bb->b;
  b.stream = (hipStream_t)stream;
  b.mode = mode;
  b.dtype = dtype;
  b.ddof = ddof;
  b.batched = true;
  for (int32_t i = 0; i < n; ++i) {
    const cvgram_problem& q = problems[i];
    ProbPlan p;
    p.X = q.X;
    p.Y = q.M > 0 ? q.Y : nullptr;
    p.fold = q.fold_id;
    p.N = q.N;
    p.K = q.K;
    p.M = q.M;
    p.W = q.K + q.M;
    p.out_xx = q.out_XtX;
    p.out_xy = q.out_XtY;
    b.pp.push_back(p);
  }
  cvgram_status st = CVGRAM_OK;
  try {
    CVG_HIP(hipGetDevice(&b.device));
    st = prepare(b);
    if (st == CVGRAM_OK) {
      // The caller's stream may be the legacy null stream, which cannot be
      // captured: capture on a private stream (default priority) and replay
      // on the caller's stream.
      CVG_HIP(hipStreamSynchronize(b.stream));  // the plan upload precedes capture
      hipStream_t user = b.stream, cap = nullptr;
      CVG_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
      b.stream = cap;
      hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess) {
        try {
          run_pipeline(b, false);
          e = hipStreamEndCapture(cap, &b.graph);
        } catch (const Fail&) {
          hipGraph_t g = nullptr;
          (void)hipStreamEndCapture(cap, &g);
          if (g) (void)hipGraphDestroy(g);
          b.stream = user;
          (void)hipStreamDestroy(cap);
          throw;
        }
      }
      b.stream = user;
      (void)hipStreamDestroy(cap);
      CVG_HIP(e);
      CVG_HIP(hipGraphInstantiate(&b.gexec, b.graph, nullptr, nullptr, 0));
    }
  } catch (const Fail& f) {
    st = f.st;
  }
  if (st != CVGRAM_OK) {
    (void)hipStreamSynchronize(b.stream);
    b.release();
    return st;
  }
  *out = bb.release();
  return CVGRAM_OK;
} CVG_ABI_CATCH

cvgram_status cvgram_batch_run(cvgram_batch_t bb) try {
  if (!bb) return fail(CVGRAM_EINVAL, "NULL batch");
  hipError_t e = hipGraphLaunch(bb->b.gexec, bb->b.stream);
  if (e != hipSuccess) return fail(CVGRAM_EDEVICE, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
  return CVGRAM_OK;
} CVG_ABI_CATCH

cvgram_status cvgram_batch_run_eager(cvgram_batch_t bb) try {
  if (!bb) return fail(CVGRAM_EINVAL, "NULL batch");
  try {
    run_pipeline(bb->b, false);
  } catch (const Fail& f) {
    return f.st;
  }
  return CVGRAM_OK;
} CVG_ABI_CATCH

cvgram_status cvgram_batch_problem_info(cvgram_batch_t bb, int32_t i, int32_t* P,
                                        int32_t* scalable) try {
  if (!bb) return fail(CVGRAM_EINVAL, "NULL batch");
  if (i < 0 || i >= (int32_t)bb->b.pp.size()) return fail(CVGRAM_ERANGE, "problem index out of range");
  if (P) *P = bb->b.pp[i].P;
  if (scalable) *scalable = bb->b.pp[i].scalable ? 1 : 0;
  return CVGRAM_OK;
} CVG_ABI_CATCH

cvgram_status cvgram_batch_destroy(cvgram_batch_t bb) try {
  if (!bb) return CVGRAM_OK;
  hipError_t e = hipStreamSynchronize(bb->b.stream);
  bb->b.release();
  delete bb;
  if (e != hipSuccess) return fail(CVGRAM_EDEVICE, hipGetErrorString(e));
  return CVGRAM_OK;
} CVG_ABI_CATCH

// ---------------------------------------------------------------------------
// autotuner
// ---------------------------------------------------------------------------
}  // extern "C"

namespace {

// Gram-stage time (pack through slab reduction, the best of three eager
// runs after a warm one) of the problems `pp` planned with the forced
// configuration `cfg` (each problem's tile capped by its own widest).  The
// candidate's workspace goes back to the cache on every path.
double time_candidate(const std::vector<ProbPlan>& pp, cvgram_dtype dtype, cvgram_mode mode,
                      hipStream_t stream, const Config& cfg, cvgram_status& st,
                      std::vector<int32_t>* folds = nullptr) {
  Batch b;
  struct Releaser {
    Batch& b;
    ~Releaser() {
      (void)hipStreamSynchronize(b.stream);
      b.release();
    }
  } releaser{b};
  b.stream = stream;
  b.mode = mode;
  b.dtype = dtype;
  b.ddof = 1;
  b.timing = true;
  b.force_cfg = true;
  b.forced = cfg;
  b.pp = pp;
  CVG_HIP(hipGetDevice(&b.device));
  st = prepare(b);
  if (st != CVGRAM_OK) return 1e300;
  if (folds) {
    folds->clear();
    for (const ProbPlan& q : b.pp) folds->push_back(q.P);
  }
  run_pipeline(b, true);  // warm
  double ms = 1e300;
  for (int rep = 0; rep < 3; ++rep) {
    run_pipeline(b, true);
    CVG_HIP(hipEventSynchronize(b.ev[4]));
    float t = 0.f;
    CVG_HIP(hipEventElapsedTime(&t, b.ev[1], b.ev[4]));
    ms = std::min(ms, (double)t);
  }
  return ms;
}

const int kTuneTiles[3] = {64, 128, 256};
const int64_t kTuneItems[6] = {512, 1024, 2048, 4096, 8192, 16384};
// a batch also tries 256 x 128 tiles for its widest problems only
const int64_t kTuneWideMinK[2] = {0, 512};

}  // namespace

extern "C" {

cvgram_status cvgram_autotune(const void* X, const void* Y, const int32_t* fold_id, int64_t N,
                              int64_t K, int64_t M, cvgram_dtype dtype, cvgram_mode mode,
                              void* stream, int32_t* tile, int32_t* target_items) try {
  set_error("");
  cvgram_status st = check_problem(X, Y, fold_id, N, K, M);
  if (st != CVGRAM_OK) return st;
  if (dtype != CVGRAM_F32 && dtype != CVGRAM_F64) return fail(CVGRAM_EINVAL, "bad dtype");
  if (mode != CVGRAM_MODE_FP64 && mode != CVGRAM_MODE_FP32 && mode != CVGRAM_MODE_BF16X3)
    return fail(CVGRAM_EINVAL, "bad mode");
  ProbPlan p;
  p.X = X;
  p.Y = M > 0 ? Y : nullptr;
  p.fold = fold_id;
  p.N = N;
  p.K = K;
  p.M = M;
  p.W = K + M;
  const std::vector<ProbPlan> pp{p};
  Config best;
  double best_ms = 1e300;
  std::vector<int32_t> folds;
  try {
    for (int t : kTuneTiles) {
      if (t == 64 && K > 1024) continue;   // too many tiles to pay off
      if (t > natural_tile(mode, K)) continue;  // wider than the problem takes
      for (int64_t it : kTuneItems) {
        Config c;
        c.tile = t;
        c.target_items = it;
        const double ms = time_candidate(pp, dtype, mode, (hipStream_t)stream, c, st, &folds);
        if (st != CVGRAM_OK) return st;
        if (ms < best_ms) {
          best_ms = ms;
          best = c;
        }
      }
    }
  } catch (const Fail& f) {
    return f.st;
  }
  {
    TuneTable& tt = tune_table();
    std::lock_guard<std::mutex> g(tt.mu);
    tune_load_locked(tt);
    tt.t[tune_key_locked(tt, mode, dtype, K, M, N, folds.empty() ? 1 : folds[0])] = best;
    tune_save_locked(tt);
  }
  if (tile) *tile = best.tile;
  if (target_items) *target_items = (int32_t)best.target_items;
  return CVGRAM_OK;
} CVG_ABI_CATCH

cvgram_status cvgram_batch_autotune(const cvgram_problem* problems, int32_t n, cvgram_dtype dtype,
                                    cvgram_mode mode, void* stream, int32_t* max_tile,
                                    int32_t* wide_min_k, int32_t* target_items, double* gram_ms) try {
  set_error("");
  if (!problems || n < 1) return fail(CVGRAM_EINVAL, "need at least one problem");
  if (dtype != CVGRAM_F32 && dtype != CVGRAM_F64) return fail(CVGRAM_EINVAL, "bad dtype");
  if (mode != CVGRAM_MODE_FP64 && mode != CVGRAM_MODE_FP32 && mode != CVGRAM_MODE_BF16X3)
    return fail(CVGRAM_EINVAL, "bad mode");
  std::vector<ProbPlan> pp;
  int widest = 64;
  for (int32_t i = 0; i < n; ++i) {
    const cvgram_problem& q = problems[i];
    cvgram_status st = check_problem(q.X, q.Y, q.fold_id, q.N, q.K, q.M);
    if (st != CVGRAM_OK) return fail(st, "problem " + std::to_string(i) + ": " + g_last_error);
    ProbPlan p;
    p.X = q.X;
    p.Y = q.M > 0 ? q.Y : nullptr;
    p.fold = q.fold_id;
    p.N = q.N;
    p.K = q.K;
    p.M = q.M;
    p.W = q.K + q.M;
    pp.push_back(p);
    widest = std::max(widest, natural_tile(mode, q.K));
  }
  Config best;
  double best_ms = 1e300;
  std::vector<int32_t> folds;
  cvgram_status st = CVGRAM_OK;
  try {
    for (int t : kTuneTiles) {
      if (t > widest) continue;
      for (int64_t wk : kTuneWideMinK) {
        if (wk > 0 && t != 256) continue;
        for (int64_t it : kTuneItems) {
          Config c;
          c.tile = t;
          c.target_items = it;
          c.wide_min_k = wk;
          const double ms = time_candidate(pp, dtype, mode, (hipStream_t)stream, c, st, &folds);
          if (st != CVGRAM_OK) return st;
          if (ms < best_ms) {
            best_ms = ms;
            best = c;
          }
        }
      }
    }
  } catch (const Fail& f) {
    return f.st;
  }
  {
    // every problem's bucket takes the batch's choice (its tile capped by
    // the problem's widest)
    TuneTable& tt = tune_table();
    std::lock_guard<std::mutex> g(tt.mu);
    tune_load_locked(tt);
    for (size_t i = 0; i < pp.size(); ++i) {
      const ProbPlan& p = pp[i];
      Config c = best;
      c.tile = std::min(best.tile, natural_tile(mode, p.K));
      if (c.tile == 256 && p.K < best.wide_min_k) c.tile = 128;
      c.wide_min_k = 0;
      tt.t[tune_key_locked(tt, mode, dtype, p.K, p.M, p.N, i < folds.size() ? folds[i] : 1)] = c;
    }
    tune_save_locked(tt);
  }
  if (max_tile) *max_tile = best.tile;
  if (wide_min_k) *wide_min_k = (int32_t)best.wide_min_k;
  if (target_items) *target_items = (int32_t)best.target_items;
  if (gram_ms) *gram_ms = best_ms;
  return CVGRAM_OK;
} CVG_ABI_CATCH

}  // extern "C"

// ---------------------------------------------------------------------------
// allocation-free form: fixed device scratch and host staging
// ---------------------------------------------------------------------------
// The device scratch is a file-scope array: each device the library runs on
// holds its own copy from module load until the process ends.  In host code
// its name is only a stand-in; its device address comes from
// hipGetSymbolAddress, taken once per device with that device current.
static __device__ __align__(256) unsigned char scratch[CVGRAM_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr size_t kNoallocHostBytes = (size_t)16 << 20;
alignas(4096) unsigned char g_noalloc_host[kNoallocHostBytes];
// one call at a time uses the host staging (device work of calls on one
// device still races unless stream-ordered; see the header)
std::mutex g_noalloc_mu;
void* g_scratch_ptr[kMaxDev] = {};

// device address of this device's scratch array (device current)
void* scratch_address(int device) {
  if (device < 0 || device >= kMaxDev) {
    set_error("device index out of range");
    throw Fail{CVGRAM_EDEVICE};
  }
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      throw Fail{CVGRAM_EDEVICE};
    }
    g_scratch_ptr[device] = ptr;
  }
  return g_scratch_ptr[device];
}

}  // namespace

extern "C" {

cvgram_status cvgram_folds_all_noalloc(const void* X, const void* Y, const int32_t* fold_id,
                                       int64_t N, int64_t K, int64_t M, cvgram_dtype dtype,
                                       int ddof, cvgram_mode mode, int32_t P, void* stream,
                                       void* out_XtX, void* out_XtY) try {
  set_error("");
  cvgram_status st = check_problem(X, Y, fold_id, N, K, M);
  if (st != CVGRAM_OK) return st;
  if (dtype != CVGRAM_F32 && dtype != CVGRAM_F64) return fail(CVGRAM_EINVAL, "bad dtype");
  if (mode != CVGRAM_MODE_FP64 && mode != CVGRAM_MODE_FP32 && mode != CVGRAM_MODE_BF16X3)
    return fail(CVGRAM_EINVAL, "bad mode");
  if (ddof != 0 && ddof != 1) return fail(CVGRAM_EINVAL, "ddof must be 0 or 1");
  if (P < 2 || P > N) return fail(CVGRAM_EINVAL, "need 2 <= P <= N");
  std::lock_guard<std::mutex> g(g_noalloc_mu);
  Arena arena;
  Batch b;
  b.stream = (hipStream_t)stream;
  b.mode = mode;
  b.dtype = dtype;
  b.ddof = ddof;
  b.batched = false;
  b.timing = false;
  b.mem.arena = &arena;
  ProbPlan p;
  p.X = X;
  p.Y = M > 0 ? Y : nullptr;
  p.fold = fold_id;
  p.N = N;
  p.K = K;
  p.M = M;
  p.W = K + M;
  b.pp.push_back(p);
  try {
    CVG_HIP(hipGetDevice(&b.device));
    arena.dev = (char*)scratch_address(b.device);
    arena.dev_cap = CVGRAM_NOALLOC_SCRATCH_BYTES;
    arena.host = (char*)g_noalloc_host;
    arena.host_cap = kNoallocHostBytes;
    st = prepare(b);
    if (st == CVGRAM_OK && b.pp[0].P != P)
      st = fail(CVGRAM_EFOLDS, "the labels give " + std::to_string(b.pp[0].P) +
                                   " folds, not the P passed");
    if (st == CVGRAM_OK) {
      run_pipeline(b, false);
      st = correct_single(b, 0, P, all_classes_out(b, 0, out_XtX, out_XtY));
    }
  } catch (const Fail& f) {
    st = f.st;
  }
  // the staging buffer is reused by the next call: every copy that reads it
  // has been consumed (pageable uploads are staged before the call
  // returns); on an error the device work is waited for
  if (st != CVGRAM_OK) (void)hipStreamSynchronize(b.stream);
  b.release();
  return st;
} CVG_ABI_CATCH

const char* cvgram_status_string(cvgram_status s) {
  switch (s) {
    case CVGRAM_OK: return "ok";
    case CVGRAM_EINVAL: return "invalid argument";
    case CVGRAM_EFOLDS: return "invalid partitioning (Definition 1)";
    case CVGRAM_ENOTSCALABLE: return "partitioning not scalable (Definition 6)";
    case CVGRAM_ENOMEM: return "out of memory";
    case CVGRAM_EDEVICE: return "HIP runtime error";
    case CVGRAM_ERANGE: return "fold index out of range";
    case CVGRAM_ESINGULAR: return "a regularised system is not positive definite";
  }
  return "unknown status";
}

const char* cvgram_last_error_message(void) { return g_last_error.c_str(); }

int32_t cvgram_version(void) { return 200; }

}  // extern "C"
