// libkbatch: batch SHA-3 on gfx950 -- kernels, scheduler and the C ABI.
//
// Pipeline of keccak_batch (persistent form), all enqueued on the caller's
// stream with no host synchronisation:
//   k_reset     clear histogram, cursors and control words
//   k_count     block count nb = floor(L/R) + 1 per message, histogram of
//               nb (bins 1..4094 exact, 4095 = "4095 or more"), and the cost
//               of arrival order (sum over 64-message waves of 64 * max nb)
//   k_plan      one workgroup: if arrival order wastes <= 2 % of the lane
//               slots it is kept; otherwise bucket starts in descending nb
//               (longest first).  Cuts the work into queue items of about
//               `steps_per_item` permutations per lane.
//   k_scatter   counting-sort scatter of message indices into `order`
//               (skipped when arrival order is kept)
//   k_persistent  a grid sized to the resident capacity pops items from an
//               atomic counter; each lane hashes one message per step.
// The plain form is one k_plain launch in arrival order; the per-bucket form
// runs k_count/k_plan/k_scatter, reads the histogram back, and launches
// k_plain once per non-empty bucket.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "kbatch.h"
#include "sponge_device.h"

using kb::kMixed;
using kb::Lane;
using kb::SpongeShape;

namespace {

constexpr int kBlock = 256;         // threads per workgroup of the hashing kernels
constexpr uint32_t kKeyBins = 4096;  // block-count buckets
constexpr int kPlanThreads = 1024;
constexpr int kScatterTile = 4096;  // messages per scatter workgroup

// control words (uint32 indices into the ctl area)
enum : int {
  CTL_QUEUE = 0,     // persistent queue counter
  CTL_NITEMS = 1,    // number of queue items
  CTL_IDENTITY = 2,  // 1: arrival order kept, order[] unused
  CTL_MAXKEY = 3,    // largest block-count key seen
  CTL_SUM_NB = 4,    // uint64: sum of nb (words 4, 5)
  CTL_SUM_WAVE = 6,  // uint64: sum over arrival-order waves of 64 * max nb (words 6, 7)
  CTL_WORDS = 64
};

struct WorkItem {
  uint32_t begin, end;  // positions in order[] (message indices in arrival order)
};

template <int V>
constexpr int out_stride() {
  return V == kMixed ? 64 : kb::digest_bytes_of(V);
}

template <int V>
__device__ __forceinline__ int rate_of(int var) {
  return V == kMixed ? kb::rate_bytes_rt(var) : kb::rate_bytes_of(V);
}

template <int V>
__device__ __forceinline__ uint64_t blocks_of(uint64_t len, int var) {
  if (V == kMixed && var > 3) return 1;  // no work: the slot is zeroed
  return len / static_cast<uint64_t>(rate_of<V>(var)) + 1u;
}

__device__ __forceinline__ uint32_t key_of(uint64_t nb) {
  return nb >= kKeyBins - 1 ? kKeyBins - 1 : static_cast<uint32_t>(nb);
}

// Hash message i into its output slot.
template <int V>
__device__ __forceinline__ void hash_message(const uint8_t* __restrict__ data,
                                             const uint64_t* __restrict__ offs,
                                             const uint64_t* __restrict__ lens,
                                             const uint8_t* __restrict__ vars, uint64_t i,
                                             uint8_t* __restrict__ out, uint32_t* row) {
  int var = V;
  if constexpr (V == kMixed) var = vars[i];
  uint8_t* o = out + i * static_cast<uint64_t>(out_stride<V>());
  if (V == kMixed && var > 3) {
    uint32_t* o32 = reinterpret_cast<uint32_t*>(o);
#pragma unroll
    for (int k = 0; k < 16; ++k) o32[k] = 0u;
    return;
  }
  Lane A[25];
  kb::sponge_hash<V>(A, data + offs[i], lens[i], var, row);
  kb::store_digest<V>(o, A, var);
}

// ---------------------------------------------------------------------------
// Hashing kernels
// ---------------------------------------------------------------------------

// One thread per message (Section 4.1).  With `order`, thread p hashes
// message order[first + p]; otherwise message first + p.
template <int V>
__global__ __launch_bounds__(kBlock) void k_plain(const uint8_t* __restrict__ data,
                                                  const uint64_t* __restrict__ offs,
                                                  const uint64_t* __restrict__ lens,
                                                  const uint8_t* __restrict__ vars,
                                                  const uint32_t* __restrict__ order,
                                                  uint64_t first, uint64_t count,
                                                  uint8_t* __restrict__ out) {
  using S = SpongeShape<V>;
  __shared__ __align__(16) uint32_t lds[kBlock * S::kRowDw];
  const uint64_t p = static_cast<uint64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (p >= count) return;
  const uint64_t i = order ? order[first + p] : first + p;
  hash_message<V>(data, offs, lens, vars, i, out, lds + threadIdx.x * S::kRowDw);
}

// Persistent form: waves pop queue items until the queue is drained.  Every
// wave leaves the loop once the counter passes the item count, so the grid
// always drains.
template <int V>
__global__ __launch_bounds__(kBlock) void k_persistent(
    const uint8_t* __restrict__ data, const uint64_t* __restrict__ offs,
    const uint64_t* __restrict__ lens, const uint8_t* __restrict__ vars,
    const uint32_t* __restrict__ order, const WorkItem* __restrict__ items,
    uint32_t* __restrict__ ctl, uint8_t* __restrict__ out) {
  using S = SpongeShape<V>;
  __shared__ __align__(16) uint32_t lds[kBlock * S::kRowDw];
  uint32_t* row = lds + threadIdx.x * S::kRowDw;
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t n_items = ctl[CTL_NITEMS];
  const uint32_t* ord = ctl[CTL_IDENTITY] ? nullptr : order;
  for (;;) {
    uint32_t t = 0;
    if (lane == 0)
      t = __hip_atomic_fetch_add(&ctl[CTL_QUEUE], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    t = __shfl(t, 0);
    if (t >= n_items) break;
    const WorkItem it = items[t];
    for (uint32_t pos = it.begin + lane; pos < it.end; pos += 64u) {
      const uint64_t i = ord ? ord[pos] : pos;
      hash_message<V>(data, offs, lens, vars, i, out, row);
    }
  }
}

// Strided messages for tree mode: message i is the min(msg_len, total - i *
// stride) bytes at base + i * stride; its digest goes to out + i * D.
template <int V>
__global__ __launch_bounds__(kBlock) void k_strided(const uint8_t* __restrict__ base,
                                                    uint64_t stride, uint64_t msg_len,
                                                    uint64_t total, uint64_t count,
                                                    uint8_t* __restrict__ out) {
  using S = SpongeShape<V>;
  __shared__ __align__(16) uint32_t lds[kBlock * S::kRowDw];
  const uint64_t i = static_cast<uint64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (i >= count) return;
  const uint64_t off = i * stride;
  const uint64_t len = total - off < msg_len ? total - off : msg_len;
  Lane A[25];
  kb::sponge_hash<V>(A, base + off, len, V, lds + threadIdx.x * S::kRowDw);
  kb::store_digest<V>(out + i * static_cast<uint64_t>(kb::digest_bytes_of(V)), A, V);
}

// ---------------------------------------------------------------------------
// Scheduler kernels
// ---------------------------------------------------------------------------

__global__ void k_reset(uint32_t* __restrict__ meta, uint32_t words) {
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < words; k += gridDim.x * blockDim.x)
    meta[k] = 0u;
}

// Active lanes holding the same key as this lane (a software match-any):
// one pass per distinct key in the wave.
__device__ __forceinline__ uint64_t same_key_lanes(uint32_t key) {
  uint64_t remaining = __ballot(1);
  uint64_t mine = 0;
  while (remaining) {
    const int leader = __ffsll(static_cast<unsigned long long>(remaining)) - 1;
    const uint32_t k0 = __shfl(key, leader);
    const uint64_t m = __ballot(key == k0) & remaining;
    if (key == k0) mine = m;
    remaining &= ~m;
  }
  return mine;
}

__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint64_t below = lane ? (~0ull >> (64u - lane)) : 0ull;
  return static_cast<uint32_t>(__popcll(mask & below));
}

template <int V>
__global__ __launch_bounds__(kBlock) void k_count(const uint64_t* __restrict__ lens,
                                                  const uint8_t* __restrict__ vars, uint64_t n,
                                                  uint32_t* __restrict__ hist,
                                                  uint32_t* __restrict__ ctl) {
  __shared__ uint32_t lhist[kKeyBins];
  __shared__ unsigned long long lsum_nb, lsum_wave;
  __shared__ uint32_t lmax;
  for (uint32_t k = threadIdx.x; k < kKeyBins; k += kBlock) lhist[k] = 0u;
  if (threadIdx.x == 0) {
    lsum_nb = 0ull;
    lsum_wave = 0ull;
    lmax = 0u;
  }
  __syncthreads();
  const uint32_t lane = threadIdx.x & 63u;
  const uint64_t waves = static_cast<uint64_t>(gridDim.x) * (kBlock / 64);
  const uint64_t wave_id = static_cast<uint64_t>(blockIdx.x) * (kBlock / 64) + threadIdx.x / 64;
  uint64_t acc_nb = 0, acc_wave = 0;
  uint32_t acc_max = 0;
  for (uint64_t c = wave_id; c * 64u < n; c += waves) {
    const uint64_t i = c * 64u + lane;
    uint64_t nb = 0;
    if (i < n) nb = blocks_of<V>(lens[i], V == kMixed ? vars[i] : V);
    // 64 * max nb over the wave, and the sum of nb
    uint64_t mx = nb, sm = nb;
    for (int d = 32; d >= 1; d >>= 1) {
      const uint64_t omx = __shfl_xor(mx, d);
      const uint64_t osm = __shfl_xor(sm, d);
      mx = omx > mx ? omx : mx;
      sm += osm;
    }
    acc_nb += sm;
    acc_wave += 64u * mx;
    if (i < n) {
      const uint32_t key = key_of(nb);
      acc_max = key > acc_max ? key : acc_max;
      const uint64_t peers = same_key_lanes(key);
      if (lanes_below(peers) == 0) atomicAdd(&lhist[key], static_cast<uint32_t>(__popcll(peers)));
    }
  }
  if (lane == 0) {
    atomicAdd(&lsum_nb, static_cast<unsigned long long>(acc_nb));
    atomicAdd(&lsum_wave, static_cast<unsigned long long>(acc_wave));
  }
  atomicMax(&lmax, acc_max);
  __syncthreads();
  for (uint32_t k = threadIdx.x; k < kKeyBins; k += kBlock)
    if (lhist[k]) atomicAdd(&hist[k], lhist[k]);
  if (threadIdx.x == 0) {
    atomicAdd(reinterpret_cast<unsigned long long*>(&ctl[CTL_SUM_NB]), lsum_nb);
    atomicAdd(reinterpret_cast<unsigned long long*>(&ctl[CTL_SUM_WAVE]), lsum_wave);
    atomicMax(&ctl[CTL_MAXKEY], lmax);
  }
}

// Block-wide exclusive scan of one value per thread (kPlanThreads threads).
__device__ uint64_t block_exclusive_scan(uint64_t v, uint64_t* scratch, uint64_t* total) {
  const uint32_t t = threadIdx.x;
  scratch[t] = v;
  __syncthreads();
  for (uint32_t d = 1; d < kPlanThreads; d <<= 1) {
    const uint64_t add = t >= d ? scratch[t - d] : 0ull;
    __syncthreads();
    scratch[t] += add;
    __syncthreads();
  }
  const uint64_t incl = scratch[t];
  *total = scratch[kPlanThreads - 1];
  __syncthreads();
  return incl - v;
}

// One workgroup of kPlanThreads threads.  Thread t owns the four bins of
// descending-key rank 4t .. 4t+3 (rank r is key kKeyBins - 1 - r).
__global__ __launch_bounds__(kPlanThreads) void k_plan(uint32_t* __restrict__ hist,
                                                       uint32_t* __restrict__ start,
                                                       uint32_t* __restrict__ ctl,
                                                       WorkItem* __restrict__ items, uint64_t n,
                                                       uint32_t steps_per_item,
                                                       int allow_identity, int force_sort) {
  __shared__ uint64_t scratch[kPlanThreads];
  __shared__ uint32_t identity;
  const uint32_t t = threadIdx.x;
  if (t == 0) {
    const uint64_t sum_nb = *reinterpret_cast<unsigned long long*>(&ctl[CTL_SUM_NB]);
    const uint64_t sum_wave = *reinterpret_cast<unsigned long long*>(&ctl[CTL_SUM_WAVE]);
    // arrival order is kept when its waves waste at most 2 % of lane slots
    identity = (!force_sort && allow_identity && sum_wave * 50u <= sum_nb * 51u) ? 1u : 0u;
    ctl[CTL_IDENTITY] = identity;
  }
  __syncthreads();
  if (identity) {
    const uint64_t sum_nb = *reinterpret_cast<unsigned long long*>(&ctl[CTL_SUM_NB]);
    const uint64_t avg = sum_nb / (n ? n : 1);
    const uint64_t g = avg >= steps_per_item ? 1u : steps_per_item / (avg ? avg : 1);
    const uint64_t per = 64u * g;
    const uint64_t m = (n + per - 1) / per;
    for (uint64_t k = t; k < m; k += kPlanThreads) {
      const uint64_t b = k * per, e = b + per < n ? b + per : n;
      items[k] = WorkItem{static_cast<uint32_t>(b), static_cast<uint32_t>(e)};
    }
    if (t == 0) ctl[CTL_NITEMS] = static_cast<uint32_t>(m);
    return;
  }
  uint32_t cnt[4], per[4];
  uint64_t c_sum = 0, it_sum = 0;
  for (int q = 0; q < 4; ++q) {
    const uint32_t key = kKeyBins - 1u - (4u * t + q);
    cnt[q] = key ? hist[key] : 0u;
    const uint32_t g = key >= steps_per_item ? 1u : steps_per_item / (key ? key : 1u);
    per[q] = 64u * g;
    c_sum += cnt[q];
    it_sum += (cnt[q] + per[q] - 1u) / per[q];
  }
  uint64_t total;
  uint64_t c_base = block_exclusive_scan(c_sum, scratch, &total);
  uint64_t it_base = block_exclusive_scan(it_sum, scratch, &total);
  if (t == 0) ctl[CTL_NITEMS] = static_cast<uint32_t>(total);
  for (int q = 0; q < 4; ++q) {
    const uint32_t key = kKeyBins - 1u - (4u * t + q);
    start[key] = static_cast<uint32_t>(c_base);
    for (uint32_t b = 0; b < cnt[q]; b += per[q]) {
      const uint32_t e = b + per[q] < cnt[q] ? b + per[q] : cnt[q];
      items[it_base++] = WorkItem{static_cast<uint32_t>(c_base + b), static_cast<uint32_t>(c_base + e)};
    }
    c_base += cnt[q];
  }
}

// Counting-sort scatter: workgroup w handles messages [w * tile, (w+1) * tile)
// and reserves one range per non-empty bin with a single global atomic.
template <int V>
__global__ __launch_bounds__(kBlock) void k_scatter(const uint64_t* __restrict__ lens,
                                                    const uint8_t* __restrict__ vars, uint64_t n,
                                                    const uint32_t* __restrict__ start,
                                                    uint32_t* __restrict__ cursor,
                                                    const uint32_t* __restrict__ ctl,
                                                    uint32_t* __restrict__ order) {
  if (ctl[CTL_IDENTITY]) return;
  __shared__ uint32_t lcount[kKeyBins];
  __shared__ uint32_t lbase[kKeyBins];
  for (uint32_t k = threadIdx.x; k < kKeyBins; k += kBlock) lcount[k] = 0u;
  __syncthreads();
  const uint64_t first = static_cast<uint64_t>(blockIdx.x) * kScatterTile;
  const uint64_t last = first + kScatterTile < n ? first + kScatterTile : n;
  for (uint64_t i0 = first; i0 < last; i0 += kBlock) {
    const uint64_t i = i0 + threadIdx.x;
    if (i < last) {
      const uint32_t key = key_of(blocks_of<V>(lens[i], V == kMixed ? vars[i] : V));
      const uint64_t peers = same_key_lanes(key);
      if (lanes_below(peers) == 0) atomicAdd(&lcount[key], static_cast<uint32_t>(__popcll(peers)));
    }
  }
  __syncthreads();
  for (uint32_t k = threadIdx.x; k < kKeyBins; k += kBlock) {
    const uint32_t c = lcount[k];
    lbase[k] = c ? start[k] + atomicAdd(&cursor[k], c) : 0u;
    lcount[k] = 0u;
  }
  __syncthreads();
  for (uint64_t i0 = first; i0 < last; i0 += kBlock) {
    const uint64_t i = i0 + threadIdx.x;
    if (i < last) {
      const uint32_t key = key_of(blocks_of<V>(lens[i], V == kMixed ? vars[i] : V));
      const uint64_t peers = same_key_lanes(key);
      const uint32_t rank = lanes_below(peers);
      uint32_t base = 0;
      if (rank == 0) base = atomicAdd(&lcount[key], static_cast<uint32_t>(__popcll(peers)));
      const int leader = __ffsll(static_cast<unsigned long long>(peers)) - 1;
      base = __shfl(base, leader);
      order[lbase[key] + base + rank] = static_cast<uint32_t>(i);
    }
  }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define KB_HIP(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) return fail(KB_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

struct Workspace {
  uint32_t* meta = nullptr;  // hist | start | cursor | ctl
  uint32_t* order = nullptr;
  uint64_t order_cap = 0;
  WorkItem* items = nullptr;
  uint64_t items_cap = 0;
  uint8_t* tree = nullptr;
  uint64_t tree_cap = 0;
  uint32_t* host_hist = nullptr;  // pinned, for the per-bucket form
};

constexpr uint32_t kMetaWords = 3 * kKeyBins + CTL_WORDS;

// Measurement hook state (keccak_timing_*): event pairs around kernel launches.
struct Timing {
  bool on = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
  size_t used = 0;
};
std::mutex g_tmu;
Timing g_timing;

// Brackets one kernel launch with events when timing is enabled.
struct TimedLaunch {
  hipEvent_t stop = nullptr;
  hipStream_t s;
  explicit TimedLaunch(hipStream_t st) : s(st) {
    std::lock_guard<std::mutex> lk(g_tmu);
    if (!g_timing.on) return;
    if (g_timing.used == g_timing.pool.size()) {
      std::pair<hipEvent_t, hipEvent_t> e{nullptr, nullptr};
      if (hipEventCreate(&e.first) != hipSuccess || hipEventCreate(&e.second) != hipSuccess) {
        (void)hipGetLastError();
        return;
      }
      g_timing.pool.push_back(e);
    }
    auto& e = g_timing.pool[g_timing.used++];
    (void)hipEventRecord(e.first, s);
    stop = e.second;
  }
  ~TimedLaunch() {
    if (stop) (void)hipEventRecord(stop, s);
  }
};

std::mutex g_mu;
std::map<std::pair<int, hipStream_t>, Workspace> g_ws;
std::map<int, int> g_cus;

int cu_count(int dev, int* cus) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_cus.find(dev);
  if (it == g_cus.end()) {
    int c = 0;
    KB_HIP(hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev));
    it = g_cus.emplace(dev, c).first;
  }
  *cus = it->second;
  return KB_OK;
}

// Grow `ptr` (device) to at least `need` bytes.  Work already enqueued on
// `stream` may still read the old buffer, so wait for it before freeing.
int grow(void** ptr, uint64_t* cap, uint64_t need, hipStream_t stream) {
  if (*cap >= need && *ptr) return KB_OK;
  if (*ptr) {
    KB_HIP(hipStreamSynchronize(stream));
    KB_HIP(hipFree(*ptr));
    *ptr = nullptr;
    *cap = 0;
  }
  const uint64_t bytes = need < 256 ? 256 : need;
  if (hipMalloc(ptr, bytes) != hipSuccess) {
    (void)hipGetLastError();
    *ptr = nullptr;
    return fail(KB_ENOMEM, "hipMalloc of %llu bytes of workspace failed",
                static_cast<unsigned long long>(bytes));
  }
  *cap = bytes;
  return KB_OK;
}

int get_ws(hipStream_t stream, uint64_t msgs, uint64_t tree_bytes, Workspace** out) {
  int dev = 0;
  KB_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_mu);
  Workspace& w = g_ws[std::make_pair(dev, stream)];
  if (!w.meta) {
    uint64_t cap = 0;
    int rc = grow(reinterpret_cast<void**>(&w.meta), &cap, kMetaWords * 4ull, stream);
    if (rc) return rc;
  }
  if (msgs) {
    int rc = grow(reinterpret_cast<void**>(&w.order), &w.order_cap, msgs * 4ull, stream);
    if (rc) return rc;
    const uint64_t items = msgs / 64 + kKeyBins + 1;
    rc = grow(reinterpret_cast<void**>(&w.items), &w.items_cap, items * sizeof(WorkItem), stream);
    if (rc) return rc;
  }
  if (tree_bytes) {
    int rc = grow(reinterpret_cast<void**>(&w.tree), &w.tree_cap, tree_bytes, stream);
    if (rc) return rc;
  }
  *out = &w;
  return KB_OK;
}

struct Batch {
  int variant;  // 0..3, or kMixed
  const uint8_t* vars;
  const uint8_t* data;
  const uint64_t* offs;
  const uint64_t* lens;
  uint64_t n;
  uint8_t* out;
};

template <int V>
int launch_plain(const Batch& b, const uint32_t* order, uint64_t first, uint64_t count,
                 hipStream_t s) {
  if (!count) return KB_OK;
  const uint64_t blocks = (count + kBlock - 1) / kBlock;
  if (blocks > 0x7FFFFFFFull) return fail(KB_EINVAL, "batch too large for one launch");
  {
    TimedLaunch tl(s);
    hipLaunchKernelGGL(k_plain<V>, dim3(static_cast<uint32_t>(blocks)), dim3(kBlock), 0, s,
                       b.data, b.offs, b.lens, b.vars, order, first, count, b.out);
  }
  KB_HIP(hipGetLastError());
  return KB_OK;
}

template <int V>
int run_schedule(const Batch& b, Workspace& w, uint32_t steps, int force_sort, hipStream_t s) {
  uint32_t* hist = w.meta;
  uint32_t* start = w.meta + kKeyBins;
  uint32_t* cursor = w.meta + 2 * kKeyBins;
  uint32_t* ctl = w.meta + 3 * kKeyBins;
  hipLaunchKernelGGL(k_reset, dim3(16), dim3(256), 0, s, w.meta, kMetaWords);
  KB_HIP(hipGetLastError());
  uint64_t cblocks = (b.n + 64 * 16 - 1) / (64 * 16);  // >= 16 waves of work per block
  if (cblocks > 2048) cblocks = 2048;
  if (cblocks < 1) cblocks = 1;
  hipLaunchKernelGGL(k_count<V>, dim3(static_cast<uint32_t>(cblocks)), dim3(kBlock), 0, s, b.lens,
                     b.vars, b.n, hist, ctl);
  KB_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_plan, dim3(1), dim3(kPlanThreads), 0, s, hist, start, ctl, w.items, b.n,
                     steps, force_sort ? 0 : 1, force_sort);
  KB_HIP(hipGetLastError());
  const uint64_t sblocks = (b.n + kScatterTile - 1) / kScatterTile;
  hipLaunchKernelGGL(k_scatter<V>, dim3(static_cast<uint32_t>(sblocks)), dim3(kBlock), 0, s,
                     b.lens, b.vars, b.n, start, cursor, ctl, w.order);
  KB_HIP(hipGetLastError());
  return KB_OK;
}

template <int V>
int run_batch(const Batch& b, int mode, const kb_tile* tile, hipStream_t s) {
  if (mode == KB_MODE_PLAIN) return launch_plain<V>(b, nullptr, 0, b.n, s);
  if (b.n >= 0xFFFFFFFFull) return launch_plain<V>(b, nullptr, 0, b.n, s);  // 32-bit order[]
  Workspace* w = nullptr;
  int rc = get_ws(s, b.n, 0, &w);
  if (rc) return rc;
  uint32_t steps = tile && tile->steps_per_item > 0 ? static_cast<uint32_t>(tile->steps_per_item) : 8u;
  if (mode == KB_MODE_PER_BUCKET) {
    rc = run_schedule<V>(b, *w, steps, 1, s);
    if (rc) return rc;
    if (!w->host_hist) KB_HIP(hipHostMalloc(reinterpret_cast<void**>(&w->host_hist), kKeyBins * 4, 0));
    KB_HIP(hipMemcpyAsync(w->host_hist, w->meta, kKeyBins * 4, hipMemcpyDeviceToHost, s));
    KB_HIP(hipStreamSynchronize(s));
    uint64_t first = 0;
    for (int key = static_cast<int>(kKeyBins) - 1; key >= 1; --key) {
      const uint32_t c = w->host_hist[key];
      if (!c) continue;
      rc = launch_plain<V>(b, w->order, first, c, s);
      if (rc) return rc;
      first += c;
    }
    return KB_OK;
  }
  rc = run_schedule<V>(b, *w, steps, 0, s);
  if (rc) return rc;
  int dev = 0, cus = 0;
  KB_HIP(hipGetDevice(&dev));
  rc = cu_count(dev, &cus);
  if (rc) return rc;
  int per_cu = 0;
  KB_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_persistent<V>, kBlock, 0));
  if (per_cu < 1) per_cu = 1;
  if (tile && tile->waves_per_simd > 0) {
    const int want = tile->waves_per_simd * 4 / (kBlock / 64);
    if (want >= 1 && want < per_cu) per_cu = want;
  }
  const uint32_t grid = static_cast<uint32_t>(per_cu * cus);
  {
    TimedLaunch tl(s);
    hipLaunchKernelGGL(k_persistent<V>, dim3(grid), dim3(kBlock), 0, s, b.data, b.offs, b.lens,
                       b.vars, w->order, w->items, w->meta + 3 * kKeyBins, b.out);
  }
  KB_HIP(hipGetLastError());
  return KB_OK;
}

int dispatch(const Batch& b, int mode, const kb_tile* tile, hipStream_t s) {
  switch (b.variant) {
    case 0: return run_batch<0>(b, mode, tile, s);
    case 1: return run_batch<1>(b, mode, tile, s);
    case 2: return run_batch<2>(b, mode, tile, s);
    case 3: return run_batch<3>(b, mode, tile, s);
    default: return run_batch<kMixed>(b, mode, tile, s);
  }
}

int check_batch(const Batch& b, int mode) {
  if (b.variant != kMixed && (b.variant < 0 || b.variant > 3))
    return fail(KB_EINVAL, "variant %d is not a SHA-3 variant (0..3)", b.variant);
  if (mode < KB_MODE_PERSISTENT || mode > KB_MODE_PER_BUCKET)
    return fail(KB_EINVAL, "unknown scheduling mode %d", mode);
  if (b.n == 0) return KB_OK;
  if (!b.data || !b.offs || !b.lens || !b.out || (b.variant == kMixed && !b.vars))
    return fail(KB_EINVAL, "NULL pointer with n > 0");
  if (reinterpret_cast<uintptr_t>(b.offs) % 8 || reinterpret_cast<uintptr_t>(b.lens) % 8)
    return fail(KB_EINVAL, "d_offsets and d_lengths must be 8-byte aligned");
  if (reinterpret_cast<uintptr_t>(b.out) % 4) return fail(KB_EINVAL, "d_digests must be 4-byte aligned");
  return KB_OK;
}

int batch_entry(int variant, const uint8_t* vars, const uint8_t* data, const uint64_t* offs,
                const uint64_t* lens, uint64_t n, uint8_t* out, int mode, const kb_tile* tile,
                hipStream_t s) {
  g_err.clear();
  Batch b{variant, vars, data, offs, lens, n, out};
  int rc = check_batch(b, mode);
  if (rc || n == 0) return rc;
  return dispatch(b, mode, tile, s);
}

template <int V>
int merkle_impl(const uint8_t* data, uint64_t total, uint64_t leaf, uint8_t* root, hipStream_t s) {
  constexpr uint64_t D = kb::digest_bytes_of(V);
  const uint64_t n = total ? (total + leaf - 1) / leaf : 1;
  const uint64_t half = (n + 1) / 2;
  Workspace* w = nullptr;
  int rc = get_ws(s, 0, (n + half) * D, &w);
  if (rc) return rc;
  uint8_t* a = w->tree;
  uint8_t* c = w->tree + n * D;
  uint64_t blocks = (n + kBlock - 1) / kBlock;
  {
    TimedLaunch tl(s);
    hipLaunchKernelGGL(k_strided<V>, dim3(static_cast<uint32_t>(blocks)), dim3(kBlock), 0, s, data,
                       leaf, leaf, total, n, a);
  }
  KB_HIP(hipGetLastError());
  for (uint64_t m = n; m > 1; m = (m + 1) / 2) {
    const uint64_t pairs = m / 2;
    blocks = (pairs + kBlock - 1) / kBlock;
    {
      TimedLaunch tl(s);
      hipLaunchKernelGGL(k_strided<V>, dim3(static_cast<uint32_t>(blocks)), dim3(kBlock), 0, s, a,
                         2 * D, 2 * D, pairs * 2 * D, pairs, c);
    }
    KB_HIP(hipGetLastError());
    if (m & 1) KB_HIP(hipMemcpyAsync(c + pairs * D, a + (m - 1) * D, D, hipMemcpyDeviceToDevice, s));
    uint8_t* t = a;
    a = c;
    c = t;
  }
  KB_HIP(hipMemcpyAsync(root, a, D, hipMemcpyDeviceToDevice, s));
  return KB_OK;
}

}  // namespace

extern "C" {

int keccak_batch(int variant, const uint8_t* d_data, const uint64_t* d_offsets,
                 const uint64_t* d_lengths, uint64_t n, uint8_t* d_digests, hipStream_t stream) {
  if (variant < 0 || variant > 3) {
    g_err.clear();
    return fail(KB_EINVAL, "variant %d is not a SHA-3 variant (0..3)", variant);
  }
  return batch_entry(variant, nullptr, d_data, d_offsets, d_lengths, n, d_digests,
                     KB_MODE_PERSISTENT, nullptr, stream);
}

int keccak_batch_mixed(const uint8_t* d_variants, const uint8_t* d_data,
                       const uint64_t* d_offsets, const uint64_t* d_lengths, uint64_t n,
                       uint8_t* d_digests, hipStream_t stream) {
  return batch_entry(kMixed, d_variants, d_data, d_offsets, d_lengths, n, d_digests,
                     KB_MODE_PERSISTENT, nullptr, stream);
}

int keccak_batch_ex(int variant, const uint8_t* d_variants, const uint8_t* d_data,
                    const uint64_t* d_offsets, const uint64_t* d_lengths, uint64_t n,
                    uint8_t* d_digests, int mode, const kb_tile* tile, hipStream_t stream) {
  if (variant != -1 && (variant < 0 || variant > 3)) {
    g_err.clear();
    return fail(KB_EINVAL, "variant %d is neither -1 (mixed) nor a SHA-3 variant", variant);
  }
  return batch_entry(variant == -1 ? kMixed : variant, d_variants, d_data, d_offsets, d_lengths,
                     n, d_digests, mode, tile, stream);
}

int merkle_root(int variant, const uint8_t* d_data, uint64_t total_len, uint64_t leaf_size,
                uint8_t* d_root, hipStream_t stream) {
  g_err.clear();
  if (variant < 0 || variant > 3) return fail(KB_EINVAL, "variant %d is not a SHA-3 variant", variant);
  if (leaf_size == 0) return fail(KB_EINVAL, "leaf_size must be positive");
  if (!d_root || (total_len && !d_data)) return fail(KB_EINVAL, "NULL pointer");
  switch (variant) {
    case 0: return merkle_impl<0>(d_data, total_len, leaf_size, d_root, stream);
    case 1: return merkle_impl<1>(d_data, total_len, leaf_size, d_root, stream);
    case 2: return merkle_impl<2>(d_data, total_len, leaf_size, d_root, stream);
    default: return merkle_impl<3>(d_data, total_len, leaf_size, d_root, stream);
  }
}

int keccak_digest_bytes(int variant) {
  return variant >= 0 && variant <= 3 ? kb::digest_bytes_of(variant) : -1;
}

int keccak_rate_bytes(int variant) {
  return variant >= 0 && variant <= 3 ? kb::rate_bytes_of(variant) : -1;
}

int keccak_reserve(uint64_t max_msgs, uint64_t max_leaves, hipStream_t stream) {
  g_err.clear();
  Workspace* w = nullptr;
  const uint64_t tree = max_leaves ? (max_leaves + (max_leaves + 1) / 2) * 64ull : 0ull;
  return get_ws(stream, max_msgs, tree, &w);
}

int keccak_release(void) {
  g_err.clear();
  std::lock_guard<std::mutex> lk(g_mu);
  int rc = KB_OK;
  for (auto& kv : g_ws) {
    Workspace& w = kv.second;
    int prev = -1;
    if (hipGetDevice(&prev) == hipSuccess && hipSetDevice(kv.first.first) == hipSuccess) {
      if (hipDeviceSynchronize() != hipSuccess) rc = KB_EHIP;
      if (w.meta) (void)hipFree(w.meta);
      if (w.order) (void)hipFree(w.order);
      if (w.items) (void)hipFree(w.items);
      if (w.tree) (void)hipFree(w.tree);
      if (w.host_hist) (void)hipHostFree(w.host_hist);
      (void)hipSetDevice(prev);
    } else {
      rc = KB_EHIP;
    }
  }
  g_ws.clear();
  if (rc) fail(rc, "keccak_release: a device could not be synchronised");
  return rc;
}

int keccak_timing_enable(int on) {
  g_err.clear();
  std::lock_guard<std::mutex> lk(g_tmu);
  g_timing.on = on != 0;
  g_timing.used = 0;
  return KB_OK;
}

int keccak_timing_read(double* total_ms, uint64_t* launches) {
  g_err.clear();
  if (!total_ms || !launches) return fail(KB_EINVAL, "NULL output pointer");
  std::lock_guard<std::mutex> lk(g_tmu);
  double sum = 0.0;
  for (size_t k = 0; k < g_timing.used; ++k) {
    auto& e = g_timing.pool[k];
    KB_HIP(hipEventSynchronize(e.second));
    float ms = 0.f;
    KB_HIP(hipEventElapsedTime(&ms, e.first, e.second));
    sum += ms;
  }
  *total_ms = sum;
  *launches = g_timing.used;
  return KB_OK;
}

const char* keccak_last_error(void) { return g_err.c_str(); }

const char* keccak_version(void) { return "kbatch 0.1 (gfx950)"; }

}  // extern "C"
