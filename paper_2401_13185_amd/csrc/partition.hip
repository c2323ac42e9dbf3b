// Fold bookkeeping on the device: Algorithm 1 (validation partitions) as a
// stable sort of the rows by fold label.  Rows inside a fold stay in
// ascending order, which is the order in which Algorithm 1 visits them, so
// the output is unique and compared bit for bit.
//
// The sort is least-significant-digit radix with 8-bit digits and only as
// many passes as the largest label needs (one pass for P <= 256).  Each pass
// is: per-tile digit histogram -> exclusive scan of the digit-major
// histogram -> stable scatter, where ranks inside a tile come from wave-wide
// ballots (no atomics on the output, so the result is deterministic).  The
// first pass's histogram comes with the label counts (same tiles), and a
// single-pass sort scans it in one launch: the digit of a label below 256 is
// the label itself, so the counts give every digit's base offset.
#include <climits>

#include "internal.h"

namespace cvg {
namespace {

constexpr int kThreads = 256;
constexpr int kItems = 8;
constexpr int kTileElems = kThreads * kItems;  // rows per radix tile
constexpr int kWaves = kThreads / 64;

__global__ void fill_i32_kernel(int32_t* p, int64_t n, int32_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}

__device__ inline int wave_min(int v) {
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ inline int wave_max(int v) {
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

// info[0] = INT_MAX, info[1] = INT_MIN, info[2 ..) = 0: the starting values
// of the label validation and counts (one launch for the whole block).
__global__ void count_init_kernel(int32_t* info, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) info[i] = i == 0 ? INT_MAX : (i == 1 ? INT_MIN : 0);
}

// Label counts for labels in [0, kCountLabels), with the minimum and maximum
// (all integer, so the result does not depend on the order of the atomics):
// one pass that gives the host the fold sizes together with the validation
// data.  Workgroup t reads radix tile t, counts into LDS, adds its non-zero
// bins, and stores the tile's histogram of the low 8 bits of the labels
// (the first radix pass's digit) at hist[d * tiles + t].
__global__ __launch_bounds__(kThreads) void label_count_kernel(const int32_t* __restrict__ f,
                                                               int64_t n, int32_t* info,
                                                               int32_t* counts,
                                                               int32_t* __restrict__ hist,
                                                               int64_t tiles) {
  __shared__ int h[kCountLabels];
  __shared__ int dh[256];
  for (int b = threadIdx.x; b < kCountLabels; b += kThreads) h[b] = 0;
  dh[threadIdx.x] = 0;
  __syncthreads();
  int lo = INT_MAX, hi = INT_MIN;
  const int64_t base = (int64_t)blockIdx.x * kTileElems;
  int v[kItems];
#pragma unroll
  for (int it = 0; it < kItems; ++it) {
    const int64_t idx = base + it * kThreads + threadIdx.x;
    v[it] = idx < n ? f[idx] : -1;
  }
#pragma unroll
  for (int it = 0; it < kItems; ++it) {
    if (base + it * kThreads + threadIdx.x >= n) continue;
    lo = min(lo, v[it]);
    hi = max(hi, v[it]);
    if (v[it] >= 0) {
      if (v[it] < kCountLabels) atomicAdd(&h[v[it]], 1);
      atomicAdd(&dh[v[it] & 255], 1);
    }
  }
  lo = wave_min(lo);
  hi = wave_max(hi);
  __shared__ int slo[kWaves], shi[kWaves];
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    slo[w] = lo;
    shi[w] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < kWaves; ++k) {
      lo = min(lo, slo[k]);
      hi = max(hi, shi[k]);
    }
    atomicMin(&info[0], lo);
    atomicMax(&info[1], hi);
  }
  for (int b = threadIdx.x; b < kCountLabels; b += kThreads)
    if (h[b]) atomicAdd(&counts[b], h[b]);
  hist[(int64_t)threadIdx.x * tiles + blockIdx.x] = dh[threadIdx.x];
}

// hist is digit-major: hist[d * tiles + t]
__global__ __launch_bounds__(kThreads) void radix_hist_kernel(const int32_t* __restrict__ keys,
                                                              int64_t n, int shift,
                                                              int32_t* __restrict__ hist,
                                                              int64_t tiles) {
  __shared__ int h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kTileElems;
#pragma unroll
  for (int it = 0; it < kItems; ++it) {
    int64_t idx = base + it * kThreads + threadIdx.x;
    if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & 255], 1);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * tiles + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of n int32 counts (sum < 2^31): per-block totals, a scan of
// the totals by one workgroup, then a per-block scan with the block offsets.
// Each thread owns kScanItems consecutive elements (coalesced per wave).
constexpr int kScanItems = 8;
constexpr int kScanBlock = kThreads * kScanItems;

__device__ inline int wave_incl_scan(int v, int lane) {
  for (int o = 1; o < 64; o <<= 1) {
    const int u = __shfl_up(v, o, 64);
    if (lane >= o) v += u;
  }
  return v;
}

__global__ __launch_bounds__(kThreads) void scan_block_sums_kernel(const int32_t* __restrict__ a,
                                                                   int64_t n,
                                                                   int32_t* __restrict__ sums) {
  __shared__ int ws[kWaves];
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + threadIdx.x * kScanItems;
  int s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i)
    if (base + i < n) s += a[base + i];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < kWaves; ++w) t += ws[w];
    sums[blockIdx.x] = t;
  }
}

// exclusive scan of the block totals in place (one workgroup, serial chunks)
__global__ __launch_bounds__(kThreads) void scan_sums_kernel(int32_t* sums, int64_t nb) {
  __shared__ int ws[kWaves];
  __shared__ int carry;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t b0 = 0; b0 < nb; b0 += kThreads) {
    const int64_t i = b0 + threadIdx.x;
    const int v = i < nb ? sums[i] : 0;
    const int inc = wave_incl_scan(v, lane);
    if (lane == 63) ws[w] = inc;
    __syncthreads();
    int off = carry;
    for (int k = 0; k < w; ++k) off += ws[k];
    if (i < nb) sums[i] = off + inc - v;
    __syncthreads();
    if (threadIdx.x == kThreads - 1) carry = off + inc;
    __syncthreads();
  }
}

__global__ __launch_bounds__(kThreads) void scan_apply_kernel(int32_t* __restrict__ a, int64_t n,
                                                              const int32_t* __restrict__ sums) {
  __shared__ int ws[kWaves];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + threadIdx.x * kScanItems;
  int v[kScanItems];
  int t = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = base + i < n ? a[base + i] : 0;
    t += v[i];
  }
  const int inc = wave_incl_scan(t, lane);
  if (lane == 63) ws[w] = inc;
  __syncthreads();
  int off = sums[blockIdx.x] + inc - t;
  for (int k = 0; k < w; ++k) off += ws[k];
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < n) a[base + i] = off;
    off += v[i];
  }
}

// Single-pass sort (labels below 256): workgroup d turns row d of the
// digit-major histogram into scatter offsets, base(d) + the exclusive prefix
// over tiles, where base(d) = counts[0] + ... + counts[d - 1].
__global__ __launch_bounds__(kThreads) void digit_scan_kernel(int32_t* __restrict__ hist,
                                                              int64_t tiles,
                                                              const int32_t* __restrict__ counts) {
  __shared__ int ws[kWaves];
  __shared__ int carry;
  const int d = blockIdx.x;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int b = threadIdx.x < d ? counts[threadIdx.x] : 0;
  for (int o = 32; o > 0; o >>= 1) b += __shfl_xor(b, o, 64);
  if (lane == 0) ws[w] = b;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int k = 0; k < kWaves; ++k) t += ws[k];
    carry = t;
  }
  __syncthreads();
  int32_t* row = hist + (int64_t)d * tiles;
  for (int64_t t0 = 0; t0 < tiles; t0 += kThreads) {
    const int64_t i = t0 + threadIdx.x;
    const int v = i < tiles ? row[i] : 0;
    const int inc = wave_incl_scan(v, lane);
    if (lane == 63) ws[w] = inc;
    __syncthreads();
    int off = carry;
    for (int k = 0; k < w; ++k) off += ws[k];
    if (i < tiles) row[i] = off + inc - v;
    __syncthreads();
    if (threadIdx.x == kThreads - 1) carry = off + inc;
    __syncthreads();
  }
}

__global__ __launch_bounds__(kThreads) void radix_scatter_kernel(
    const int32_t* __restrict__ keys_in, const int32_t* __restrict__ vals_in,
    int32_t* __restrict__ keys_out, int32_t* __restrict__ vals_out, int64_t n, int shift,
    const int32_t* __restrict__ scanned, int64_t tiles) {
  __shared__ int run[256];
  __shared__ int wcnt[kWaves][256];
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int w = t >> 6;
  run[t] = scanned[(int64_t)t * tiles + blockIdx.x];
#pragma unroll
  for (int k = 0; k < kWaves; ++k) wcnt[k][t] = 0;
  __syncthreads();
  const unsigned long long lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
  const int64_t base = (int64_t)blockIdx.x * kTileElems;
  for (int it = 0; it < kItems; ++it) {
    const int64_t idx = base + it * kThreads + t;
    const bool valid = idx < n;
    const int32_t key = valid ? keys_in[idx] : 0;
    const int32_t val = valid ? (vals_in ? vals_in[idx] : (int32_t)idx) : 0;
    const int d = (key >> shift) & 255;
    unsigned long long peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1;
      const unsigned long long bal = __ballot(bit);
      peers &= bit ? bal : ~bal;
    }
    const int rank = __popcll(peers & lt);
    if (valid && rank == 0) wcnt[w][d] = __popcll(peers);
    __syncthreads();
    if (valid) {
      int pos = run[d] + rank;
      for (int k = 0; k < w; ++k) pos += wcnt[k][d];
      keys_out[pos] = key;
      vals_out[pos] = val;
    }
    __syncthreads();
    int add = 0;
#pragma unroll
    for (int k = 0; k < kWaves; ++k) {
      add += wcnt[k][t];
      wcnt[k][t] = 0;
    }
    run[t] += add;
    __syncthreads();
  }
}

// offsets[p] = first sorted position whose label is >= p; flag[0] |= 1 when
// some label in [0, P) has no row.
__global__ void fold_offsets_kernel(const int32_t* __restrict__ sk, int64_t n, int32_t P,
                                    int64_t* __restrict__ offsets, int32_t* flag) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t k = sk[i];
  const int32_t prev = i ? sk[i - 1] : -1;
  if (k != prev) {
    for (int32_t l = prev + 1; l <= k && l <= P; ++l) offsets[l] = i;
    if (k - prev > 1) atomicOr(flag, 1);
  }
  if (i == n - 1) {
    for (int32_t l = k + 1; l <= P; ++l) offsets[l] = n;
    if (k != P - 1) atomicOr(flag, 1);
  }
}

}  // namespace

void launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
  if (n <= 0) return;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  fill_i32_kernel<<<(unsigned)blocks, 256, 0, s>>>(p, n, v);
  CVG_LAUNCH_CHECK();
}

void launch_count_init(int32_t* info, int64_t n, hipStream_t s) {
  count_init_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(info, n);
  CVG_LAUNCH_CHECK();
}

void launch_label_count(const int32_t* fold, int64_t N, int32_t* info, int32_t* counts,
                        int32_t* hist, hipStream_t s) {
  const int64_t tiles = (N + kTileElems - 1) / kTileElems;
  label_count_kernel<<<(unsigned)tiles, kThreads, 0, s>>>(fold, N, info, counts, hist, tiles);
  CVG_LAUNCH_CHECK();
}

// hist holds 256 * tiles counts followed by the scan's block totals
int64_t radix_hist_entries(int64_t N) {
  const int64_t n = 256 * ((N + kTileElems - 1) / kTileElems);
  return n + (n + kScanBlock - 1) / kScanBlock;
}

void scan_exclusive(int32_t* a, int64_t n, int32_t* sums, hipStream_t s) {
  const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
  scan_block_sums_kernel<<<(unsigned)nb, kThreads, 0, s>>>(a, n, sums);
  CVG_LAUNCH_CHECK();
  scan_sums_kernel<<<1, kThreads, 0, s>>>(sums, nb);
  CVG_LAUNCH_CHECK();
  scan_apply_kernel<<<(unsigned)nb, kThreads, 0, s>>>(a, n, sums);
  CVG_LAUNCH_CHECK();
}

void radix_partition(const int32_t* fold, int64_t N, int bits, const int32_t* counts,
                     int32_t* keys_a, int32_t* keys_b, int32_t* perm, int32_t* perm_tmp,
                     int32_t* hist, bool hist_ready, const int32_t** sorted_keys,
                     hipStream_t s) {
  const int64_t tiles = (N + kTileElems - 1) / kTileElems;
  int passes = (bits + 7) / 8;
  if (passes < 1) passes = 1;
  // ping-pong so that the last pass writes the payload into `perm`
  const int32_t* kin = fold;
  const int32_t* vin = nullptr;  // identity payload on the first pass
  for (int pass = 0; pass < passes; ++pass) {
    int32_t* kout = (pass & 1) ? keys_b : keys_a;
    int32_t* vout = ((passes - 1 - pass) & 1) ? perm_tmp : perm;
    const int shift = 8 * pass;
    if (pass > 0 || !hist_ready) {
      radix_hist_kernel<<<(unsigned)tiles, kThreads, 0, s>>>(kin, N, shift, hist, tiles);
      CVG_LAUNCH_CHECK();
    }
    if (passes == 1) {
      // labels in [0, 2^bits) with bits <= 8: one workgroup per label
      digit_scan_kernel<<<1u << bits, kThreads, 0, s>>>(hist, tiles, counts);
      CVG_LAUNCH_CHECK();
    } else {
      scan_exclusive(hist, 256 * tiles, hist + 256 * tiles, s);
    }
    radix_scatter_kernel<<<(unsigned)tiles, kThreads, 0, s>>>(kin, vin, kout, vout, N, shift,
                                                              hist, tiles);
    CVG_LAUNCH_CHECK();
    kin = kout;
    vin = vout;
  }
  *sorted_keys = kin;
}

void launch_fold_offsets(const int32_t* sorted_keys, int64_t N, int32_t P, int64_t* offsets,
                         int32_t* flag, hipStream_t s) {
  fold_offsets_kernel<<<(unsigned)((N + 255) / 256), 256, 0, s>>>(sorted_keys, N, P, offsets,
                                                                   flag);
  CVG_LAUNCH_CHECK();
}

}  // namespace cvg
