// libkbatch: batch SHA-3 on gfx950 -- kernels, scheduler and the C ABI.
//
// Pipeline of keccak_batch (persistent form), all enqueued on the caller's
// stream with no host synchronisation:
//   k_reset     clear histogram, cursors and control words
//   k_count     block count nb = floor(L/R) + 1 per message and its histogram
//               (bins 1..4094 exact, 4095 = "4095 or more"); per 64-message
//               wave of arrival order, the lane-slots a wave would idle
//   k_plan      one workgroup: keep arrival order if it idles <= 2 % of the
//               lane slots, else bucket starts in descending nb (longest
//               first) and queue-item counts per bucket (about
//               `steps_per_item` permutations per lane each)
//   k_fill      one thread per queue item: its message range and bucket;
//               in the same launch, the counting-sort scatter of message
//               indices into `order` (skipped when arrival order is kept)
//   k_persistent  a grid sized to the resident capacity pops items from an
//               atomic counter; each lane hashes one message per step.  The
//               longest items run at raised wave priority so that the long
//               absorb chains, which bound the makespan, are not slowed by
//               round-robin issue with shorter work.
// The plain form is one k_plain launch in arrival order; the per-bucket form
// runs the same scheduling kernels, reads the histogram back, and launches
// k_plain once per non-empty bucket.
//
// Tree mode: k_tree hashes 256 leaves per workgroup and reduces them eight
// levels in place (pairs of child digests, an unpaired last node carried up);
// further k_tree launches reduce 256 nodes per workgroup until one is left.
// Every level is written to its own region, so no workgroup reads a node
// another one may overwrite.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "kb_error.h"
#include "kbatch.h"
#include "sponge_device.h"
#include "split_device.h"

using kb::kMixed;
using kb::kShake128;
using kb::kShake256;
using kb::Lane;
using kb::SpongeShape;

namespace {

constexpr int kBlock = 256;         // threads per workgroup of the hashing kernels
constexpr int kTreeTop = 1024;      // nodes the workgroup that reduces a tree's last levels takes
constexpr int kTreeTopThreads = 512;  // its threads: two nodes (one pair) each at its first level
constexpr uint32_t kKeyBins = 4096;  // block-count buckets
constexpr int kScatterTile = 4096;  // messages per scatter workgroup

// control words (uint32 indices into the ctl area)
enum : int {
  CTL_NITEMS = 2,    // number of queue items
  CTL_IDENTITY = 3,  // 1: arrival order kept, order[] unused
  CTL_MAXKEY = 4,    // largest block-count key seen
  CTL_ID_PER = 5,    // arrival order: messages per queue item
  CTL_USEFUL = 6,    // uint64 (words 6, 7): sum of (clamped) block counts
  CTL_IDLE = 8,      // uint64 (words 8, 9): lane-slots arrival-order waves would idle
  CTL_PRIO_KEY = 10, // front waves raise their priority on items of at least this many blocks
  CTL_SPLIT_N = 11,  // bucketed order positions [0, CTL_SPLIT_N) are hashed in the split form
  CTL_WORDS = 64
};

// One flag per SIMD of the chip, indexed from the wave's hardware id
// (XCC, shader engine, shader array, CU, SIMD); the first wave to claim its
// SIMD's flag takes queue items from the front.
constexpr uint32_t kSimdSlots = 8 * 8 * 2 * 16 * 4;

// The queue is dealt round-robin into kQueues sub-queues (item t goes to
// sub-queue t mod kQueues, so each keeps the longest-first order); a wave
// starts on the sub-queue of its XCD.  Each sub-queue is one uint64 counter
// (items taken from the front | taken from the back << 32) on its own
// 256-byte line.
constexpr uint32_t kQueues = 8;
constexpr uint32_t kQueueStrideDw = 64;
// the sub-queues, then the counter of split items on a line of its own
constexpr uint32_t kQueueAreaDw = (kQueues + 1) * kQueueStrideDw;

// k_count accumulates into kCopies partial histograms and control sums (copy
// = workgroup index mod 8, which is its XCD), so that the workgroups' closing
// atomics spread over eight addresses instead of one; k_plan folds them.
constexpr uint32_t kCopies = 8;
constexpr uint32_t kPartialWords = 8;  // per copy: useful (u64), idle (u64), max key
enum : uint32_t { P_USEFUL = 0, P_IDLE = 2, P_MAXKEY = 4 };
// Workspace metadata layout (uint32 words): hist | start | cursor | iend |
// ctl | queues | SIMD flags | hist copies 1..7 | partials.
constexpr uint32_t kHistCopiesOff = 4 * kKeyBins + CTL_WORDS + kQueueAreaDw + kSimdSlots;
constexpr uint32_t kPartialsOff = kHistCopiesOff + (kCopies - 1) * kKeyBins;

struct WorkItem {
  uint32_t begin, end;  // positions in order[] (message indices in arrival order)
  uint32_t key;         // block-count bucket of the item (0 in arrival order)
  uint32_t pad;
};

template <int V>
__device__ __forceinline__ int rate_of(int var) {
  return V == kMixed ? kb::rate_bytes_rt(var) : SpongeShape<V>::kMaxRate;
}

template <int V>
__device__ __forceinline__ uint64_t blocks_of(uint64_t len, int var) {
  if (V == kMixed && var > 3) return 1;  // no work: the slot is zeroed
  return len / static_cast<uint64_t>(rate_of<V>(var)) + 1u;
}

__device__ __forceinline__ uint32_t key_of(uint64_t nb) {
  return nb >= kKeyBins - 1 ? kKeyBins - 1 : static_cast<uint32_t>(nb);
}

// Hash message i (`len` bytes at data + off, variant `var` in the mixed
// form) into its output slot of `stride` bytes (the digest size, 64 in the
// mixed form, the output length for the XOFs).
template <int V>
__device__ __forceinline__ void hash_one(const uint8_t* __restrict__ data, uint64_t off,
                                         uint64_t len, int var, uint64_t i,
                                         uint8_t* __restrict__ out, uint64_t stride, uint32_t* row) {
  uint8_t* o = out + i * stride;
  if constexpr (V >= kShake128) {
    Lane A[25];
    kb::sponge_hash<V>(A, data + off, len, var, row);
    kb::squeeze_xof<V>(A, o, stride);
    return;
  }
  if (V == kMixed && var > 3) {
    uint32_t* o32 = reinterpret_cast<uint32_t*>(o);
#pragma unroll
    for (int k = 0; k < 16; ++k) o32[k] = 0u;
    return;
  }
  Lane A[25];
  kb::sponge_hash<V>(A, data + off, len, var, row);
  kb::store_digest<V>(o, A, var);
}

template <int V>
__device__ __forceinline__ void hash_message(const uint8_t* __restrict__ data,
                                             const uint64_t* __restrict__ offs,
                                             const uint64_t* __restrict__ lens,
                                             const uint8_t* __restrict__ vars, uint64_t i,
                                             uint8_t* __restrict__ out, uint64_t stride,
                                             uint32_t* row) {
  hash_one<V>(data, offs[i], lens[i], V == kMixed ? vars[i] : V, i, out, stride, row);
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
                                                  uint8_t* __restrict__ out, uint64_t stride) {
  using S = SpongeShape<V>;
  __shared__ __align__(16) uint32_t lds[kBlock * S::kRowDw];
  const uint64_t p = static_cast<uint64_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (p >= count) return;
  const uint64_t i = order ? order[first + p] : first + p;
  hash_message<V>(data, offs, lens, vars, i, out, stride, lds + threadIdx.x * S::kRowDw);
}

// One message hashed by a group of eight lanes in the split form (`len`
// bytes at msg, variant `var`); the digest's dwords go to o[0 .. slot_dw),
// zero past the digest.  With PF the next block's words are loaded before
// the current block's permutation (for long messages); without, each block
// is loaded when it is absorbed (fewer registers, for one- and two-block
// tree nodes).
template <int V, bool PF>
__device__ __forceinline__ void split_absorb(Lane (&a)[5], const uint8_t* msg, uint64_t len,
                                             int var, const kb::split::SplitLane& L) {
  namespace sp = kb::split;
  using S = SpongeShape<V>;
#pragma unroll
  for (int j = 0; j < 5; ++j) a[j] = Lane{0u, 0u};
  const int R = rate_of<V>(var);
  const uint32_t sh = static_cast<uint32_t>(reinterpret_cast<uintptr_t>(msg) & 3u);
  const uint64_t nb = len / static_cast<uint64_t>(R) + 1u;
  sp::BlockWords bw;
  if (PF) sp::load_words(bw, msg, sh, len, 0, R, L);
  for (uint64_t b = 0; b < nb; ++b) {
    const uint64_t boff = b * static_cast<uint64_t>(R);
    const bool fin = b + 1 == nb;
    if (!PF) sp::load_words(bw, msg, sh, len, boff, R, L);
    sp::absorb_words(a, bw, sh, R, fin, fin ? static_cast<uint32_t>(len - boff) : 0u,
                     S::kPadByte, L);
    if (PF && !fin) sp::load_words(bw, msg, sh, len, boff + R, R, L);
    sp::split_permute(a, L);
  }
}

template <int V, bool PF = true>
__device__ __forceinline__ void split_hash(const uint8_t* msg, uint64_t len, int var, uint32_t* o,
                                           int slot_dw, const kb::split::SplitLane& L) {
  Lane a[5];
  split_absorb<V, PF>(a, msg, len, var, L);
  const int dw = V == kMixed ? kb::digest_bytes_rt(var) / 4 : kb::digest_bytes_of(V) / 4;
  kb::split::store_words(o, a, dw, slot_dw, L);
}

// XOF squeeze in the lane-split form (Section 3.2): each lane writes its words
// that lie in the rate, r bits of output per permutation, until out_len
// bytes are out; the permutation between reads involves all eight lanes of
// the group, which all take the same number of turns (out_len is the batch's).
// Bytes are stored one by one unless out_len is a multiple of 4 and `out` is
// 4-byte aligned.
template <int V>
__device__ __forceinline__ void split_xof(Lane (&a)[5], uint8_t* out, uint64_t out_len,
                                          const kb::split::SplitLane& L) {
  constexpr uint32_t R = SpongeShape<V>::kMaxRate;
  const bool words = (out_len & 3u) == 0 && (reinterpret_cast<uintptr_t>(out) & 3u) == 0;
  for (uint64_t done = 0;;) {
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      const uint32_t li = L.li[j];
      if (8u * li < R) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const uint32_t v = h ? a[j].hi : a[j].lo;
          const uint64_t at = done + 8u * li + 4u * h;
          if (at < out_len) {
            if (words) {
              *reinterpret_cast<uint32_t*>(out + at) = v;
            } else {
              for (uint32_t q = 0; q < 4u && at + q < out_len; ++q)
                out[at + q] = static_cast<uint8_t>(v >> (8u * q));
            }
          }
        }
      }
    }
    done += R;
    if (done >= out_len) break;
    kb::split::split_permute(a, L);
  }
}

// Lane-split form: each group of eight lanes hashes one message at a time,
// message order[first + p] (or first + p) for p = group, group + groups, ...
// One wave per workgroup, so a handful of messages spreads over SIMDs.
constexpr int kSplitBlock = 64;
constexpr int kSplitGroups = kSplitBlock / kb::split::kGroupLanes;

template <int V>
__global__ __launch_bounds__(kSplitBlock) void k_split(const uint8_t* __restrict__ data,
                                                       const uint64_t* __restrict__ offs,
                                                       const uint64_t* __restrict__ lens,
                                                       const uint8_t* __restrict__ vars,
                                                       const uint32_t* __restrict__ order,
                                                       uint64_t first, uint64_t count,
                                                       uint8_t* __restrict__ out, uint64_t stride) {
  namespace sp = kb::split;
  __shared__ uint64_t lds[kSplitGroups * sp::kGroupSlots + 1];
  const uint32_t g = threadIdx.x / sp::kGroupLanes, t = threadIdx.x % sp::kGroupLanes;
  uint64_t* zero = lds + kSplitGroups * sp::kGroupSlots;
  if (threadIdx.x == 0) *zero = 0;
  __syncthreads();
  sp::SplitLane L;
  sp::setup(L, t, lds + g * sp::kGroupSlots, zero);
  const uint64_t groups = static_cast<uint64_t>(gridDim.x) * kSplitGroups;
  const int slot_dw = V == kMixed ? 16 : kb::digest_bytes_of(V) / 4;
  for (uint64_t p = static_cast<uint64_t>(blockIdx.x) * kSplitGroups + g; p < count; p += groups) {
    const uint64_t i = order ? order[first + p] : first + p;
    if constexpr (V >= kShake128) {
      Lane a[5];
      split_absorb<V, true>(a, data + offs[i], lens[i], V, L);
      split_xof<V>(a, out + i * stride, stride, L);
      continue;
    }
    const int var = V == kMixed ? vars[i] : V;
    uint32_t* o = reinterpret_cast<uint32_t*>(out + i * stride);
    if (V == kMixed && var > 3) {  // no such variant: the slot is zeroed
      Lane z[5];
#pragma unroll
      for (int j = 0; j < 5; ++j) z[j] = Lane{0u, 0u};
      sp::store_words(o, z, 0, slot_dw, L);
      continue;
    }
    split_hash<V>(data + offs[i], lens[i], var, o, slot_dw, L);
  }
}

// Persistent form: waves pop queue items until the queue is drained.  Every
// wave leaves the loop once the counter passes the item count, so the grid
// always drains.
// Index of the SIMD this wave runs on, from the HW_ID register (SIMD [5:4],
// CU [11:8], SH [12], SE [15:13]) and XCC_ID [3:0].  Used only to spread the
// front-of-queue waves one per SIMD; a wrong index costs balance, never
// correctness.
__device__ __forceinline__ uint32_t simd_slot() {
  const uint32_t hw = __builtin_amdgcn_s_getreg((31 << 11) | 4);
  const uint32_t xcc = __builtin_amdgcn_s_getreg((3 << 11) | 20) & 7u;
  const uint32_t simd = (hw >> 4) & 3u, cu = (hw >> 8) & 15u, sh = (hw >> 12) & 1u,
                 se = (hw >> 13) & 7u;
  return ((((xcc * 8u + se) * 2u + sh) * 16u + cu) * 4u) + simd;
}

// Persistent form.  Queue items are ordered longest first.  On each SIMD one
// wave (the first to claim the SIMD's flag) takes items from the front at
// raised issue priority while they are long, so the long absorb chains that
// bound the makespan run back to back at full rate; the other resident waves
// take the shortest items from the back and fill the issue slots the front
// wave leaves idle.  Both ends of a sub-queue advance one packed 64-bit
// counter, so no item is taken twice.  A wave drains the sub-queue of its own
// XCD first and then the others in turn, so every item is taken whatever the
// mapping of waves to XCDs, and every wave leaves once all sub-queues are
// empty, so the grid always drains.  In arrival order (uniform work) every
// wave takes from the front at normal priority.
template <int V>
__global__ __launch_bounds__(kBlock) void k_persistent(
    const uint8_t* __restrict__ data, const uint64_t* __restrict__ offs,
    const uint64_t* __restrict__ lens, const uint8_t* __restrict__ vars,
    const uint32_t* __restrict__ order, const WorkItem* __restrict__ items,
    const uint32_t* __restrict__ ctl, unsigned long long* __restrict__ queues,
    uint32_t* __restrict__ simd_flags, uint8_t* __restrict__ out, uint64_t stride) {
  using S = SpongeShape<V>;
  __shared__ __align__(16) uint32_t lds[kBlock * S::kRowDw];
  static_assert(2 * (kSplitGroups * kb::split::kGroupSlots + 1) <= 64 * S::kRowDw,
                "a wave's staging rows hold its split exchange area");
  uint32_t* row = lds + threadIdx.x * S::kRowDw;
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t n_items = ctl[CTL_NITEMS];
  const bool sorted = ctl[CTL_IDENTITY] == 0u;
  const uint32_t prio_key = ctl[CTL_PRIO_KEY];
  const uint32_t* ord = sorted ? order : nullptr;
  uint32_t claim = 0;
  if (sorted && lane == 0) claim = atomicCAS(&simd_flags[simd_slot()], 0u, 1u) == 0u ? 1u : 0u;
  const bool front = !sorted || __builtin_amdgcn_readfirstlane(__shfl(claim, 0)) != 0u;
  const unsigned long long step = 1ull << (front ? 0 : 32);
  const uint32_t home = __builtin_amdgcn_s_getreg((3 << 11) | 20) & (kQueues - 1u);
  // Split items first: the front waves hash the longest messages (bucketed
  // positions [0, split_n)) eight at a time, one per 8-lane group, in the
  // lane-split form, whose chain of permutations runs about twice as fast.
  // The exchange area is this wave's own staging rows.
  // (compiled into the mixed-variant kernel only: in the fixed-variant ones
  // the extra code alone slowed the one-block uniform batch by 8 %)
  const uint32_t split_n = sorted && V == kMixed ? ctl[CTL_SPLIT_N] : 0u;
  if constexpr (V == kMixed) {
    if (front && split_n) {
      namespace sp = kb::split;
      uint64_t* area = reinterpret_cast<uint64_t*>(lds + (threadIdx.x & ~63u) * S::kRowDw);
      uint64_t* zero = area + kSplitGroups * sp::kGroupSlots;
      if (lane == 0) *zero = 0;
      __asm__ volatile("" ::: "memory");
      sp::SplitLane L;
      sp::setup(L, lane % sp::kGroupLanes, area + (lane / sp::kGroupLanes) * sp::kGroupSlots, zero);
      const int slot_dw = V == kMixed ? 16 : kb::digest_bytes_of(V) / 4;
      uint32_t* split_ctr = reinterpret_cast<uint32_t*>(queues + kQueues * (kQueueStrideDw / 2));
      __builtin_amdgcn_s_setprio(3);
      for (;;) {
        uint32_t d = 0;
        if (lane == 0)
          d = __hip_atomic_fetch_add(split_ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        d = __builtin_amdgcn_readfirstlane(__shfl(d, 0));
        if (d >= (split_n + kSplitGroups - 1u) / kSplitGroups) break;
        const uint32_t pos = d * kSplitGroups + lane / sp::kGroupLanes;
        if (pos < split_n) {
          const uint32_t i = order[pos];
          const int var = V == kMixed ? vars[i] : V;
          uint32_t* o = reinterpret_cast<uint32_t*>(out + static_cast<uint64_t>(i) * stride);
          if (V == kMixed && var > 3) {
            Lane z[5];
#pragma unroll
            for (int j = 0; j < 5; ++j) z[j] = Lane{0u, 0u};
            sp::store_words(o, z, 0, slot_dw, L);
          } else {
            split_hash<V>(data + offs[i], lens[i], var, o, slot_dw, L);
          }
        }
      }
      __builtin_amdgcn_s_setprio(0);
    }
  }
  uint32_t qi = 0;  // sub-queues tried so far (bucketed order)
  for (;;) {
    // choose the next item; the hashing below appears once in the kernel
    uint32_t t = 0xFFFFFFFFu;
    if (!sorted) {
      uint32_t d = 0;
      if (lane == 0)
        d = __hip_atomic_fetch_add(reinterpret_cast<uint32_t*>(queues), 1u, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
      d = __builtin_amdgcn_readfirstlane(__shfl(d, 0));
      if (d < n_items) t = d;
    } else {
      while (qi < kQueues) {
        const uint32_t x = (home + qi) & (kQueues - 1u);
        const uint32_t m = n_items > x ? (n_items - x + kQueues - 1u) / kQueues : 0u;
        unsigned long long old = 0;
        if (lane == 0)
          old = __hip_atomic_fetch_add(queues + x * (kQueueStrideDw / 2), step, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t head = __builtin_amdgcn_readfirstlane(__shfl(static_cast<uint32_t>(old), 0));
        const uint32_t tail =
            __builtin_amdgcn_readfirstlane(__shfl(static_cast<uint32_t>(old >> 32), 0));
        if (static_cast<uint64_t>(head) + tail < m) {
          t = x + kQueues * (front ? head : m - 1u - tail);
          break;
        }
        ++qi;
      }
    }
    if (t == 0xFFFFFFFFu) break;
    const WorkItem it = items[t];
    if (sorted && front && it.key >= prio_key)
      __builtin_amdgcn_s_setprio(3);
    else
      __builtin_amdgcn_s_setprio(0);
    // the next message's index and metadata are loaded while this one hashes
    uint32_t pos = it.begin + lane;
    uint64_t i = 0, off = 0, len = 0;
    int var = V;
    if (pos < it.end) {
      i = ord ? ord[pos] : pos;
      off = offs[i];
      len = lens[i];
      if constexpr (V == kMixed) var = vars[i];
    }
    while (pos < it.end) {
      const uint32_t pn = pos + 64u;
      uint64_t in = 0, offn = 0, lenn = 0;
      int varn = V;
      if (pn < it.end) {
        in = ord ? ord[pn] : pn;
        offn = offs[in];
        lenn = lens[in];
        if constexpr (V == kMixed) varn = vars[in];
      }
      hash_one<V>(data, off, len, var, i, out, stride, row);
      pos = pn;
      i = in;
      off = offn;
      len = lenn;
      var = varn;
    }
  }
  __builtin_amdgcn_s_setprio(0);
}

// Tree mode.  Level l has m[l] nodes stored from byte offset off[l] of
// `nodes` (level 0 = leaf digests).  Node j of level l+1 is H(node 2j ||
// node 2j+1) of level l, or node 2j itself when it is the unpaired last one.
struct TreeLevels {
  uint64_t m[64];
  uint64_t off[64];
};

// Workgroup w owns nodes [T w, T w + T) of level `first` and reduces them
// `levels` levels.  first == 0: it also hashes those leaves (leaf i is
// min(leaf_size, total - i * leaf_size) bytes at data + i * leaf_size).  Each
// level is separated by a workgroup barrier, which also orders the global
// node writes of one level before the reads of the next.  The node of level
// `top` (the root) is written to `root`.
//
// A level with more pairs per workgroup than the workgroup has 8-lane groups
// hashes one pair per thread; the narrower levels at the top of each
// workgroup's subtree, where one thread per pair would leave a wave's worth
// of permutation latency for a handful of lanes, hash one pair per group in
// the lane-split form (five lanes per state, about twice as fast per
// permutation).  The split form's exchange area reuses the staging rows,
// which no level uses after the first split one.
//
// A workgroup owns NODES nodes of level `first`: T for the leaf and middle
// launches (one leaf or node per thread), 2T for the last workgroup, whose
// first level is then one pair per thread (a 512-thread workgroup keeps the
// 256-VGPR limit, where 1024 threads would cap it at 128 and spill).
//
// With W8 every message the kernel hashes is whole 8-byte words at an
// 8-byte-aligned address (the host checks the leaves; node pairs always are):
// blocks go from HBM into a per-wave LDS area with the loads that write LDS
// directly, the next block's while the current one is permuted, and come back
// as whole words (no byte realignment, no registers holding bytes in flight).
template <int V, int T, bool PF, bool W8, int NODES = T>
__global__ __launch_bounds__(T) void k_tree(const uint8_t* __restrict__ data, uint64_t total,
                                            uint64_t leaf_size, uint8_t* __restrict__ nodes,
                                            uint8_t* __restrict__ root, int first, int levels,
                                            int top, TreeLevels lv) {
  namespace sp = kb::split;
  using S = SpongeShape<V>;
  constexpr uint64_t D = kb::digest_bytes_of(V);
  constexpr int kGroups = T / sp::kGroupLanes;
  // SHA3-512's leaf kernel fits four waves per SIMD (125 VGPRs) only without
  // the split path (148), and its leaves are the long chains, so there the
  // in-workgroup levels stay one pair per thread.
  constexpr bool kSplitLevels = !(V == 3 && T == kBlock);
  constexpr int kSplitDw = 2 * (kGroups * sp::kGroupSlots + 1);
  constexpr int kWordsDw = (T / 64) * kb::WordArea<V>::kDw;
  constexpr int kStageDw = W8 ? kWordsDw : T * S::kRowDw;
  __shared__ __align__(16) uint32_t lds[kStageDw > kSplitDw ? kStageDw : kSplitDw];
  static_assert(kSplitDw <= T * S::kRowDw, "the split exchange area fits in the staging rows");
  uint32_t* row = lds + (W8 ? 0u : threadIdx.x * S::kRowDw);
  // one message of whole words (W8: through this wave's LDS area) or of any
  // bytes (staged through this thread's row)
  auto hash = [&](Lane (&A)[25], const uint8_t* msg, uint64_t len) {
    if constexpr (W8)
      kb::sponge_hash_words<V, PF>(
          A, msg, len,
          (__attribute__((address_space(3))) uint32_t*)(lds) +
              __builtin_amdgcn_readfirstlane(threadIdx.x / 64u) * kb::WordArea<V>::kDw,
          threadIdx.x & 63u);
    else
      kb::sponge_hash<V, PF>(A, msg, len, V, row);
  };
  const uint64_t w = blockIdx.x;
  auto dst_of = [&](int level, uint64_t j) -> uint8_t* {
    return level == top ? root : nodes + lv.off[level] + j * D;
  };
  static_assert(NODES == T || NODES == 2 * T, "one or two nodes per thread");
  if (NODES == T && first == 0) {  // leaves: only launches with one node per thread take level 0
    const uint64_t i = w * T + threadIdx.x;
    if (i < lv.m[0]) {
      const uint64_t off = i * leaf_size;
      const uint64_t len = total - off < leaf_size ? total - off : leaf_size;
      Lane A[25];
      hash(A, data + off, len);
      kb::store_digest<V>(dst_of(0, i), A, V);
    }
  }
  for (int k = 0; k < levels; ++k) {
    const int l = first + k;  // reading level l, writing level l + 1
    __syncthreads();
    const uint64_t span = static_cast<uint64_t>(NODES) >> (k + 1);  // pairs of this workgroup
    if (!kSplitLevels || span > static_cast<uint64_t>(kGroups)) {
      const uint64_t j = w * span + threadIdx.x;
      if (threadIdx.x < span && j < lv.m[l + 1]) {
        const uint8_t* src = nodes + lv.off[l] + 2 * j * D;
        uint8_t* dst = dst_of(l + 1, j);
        if (2 * j + 1 < lv.m[l]) {
          Lane A[25];
          hash(A, src, 2 * D);
          kb::store_digest<V>(dst, A, V);
        } else {
          const uint32_t* s32 = reinterpret_cast<const uint32_t*>(src);
          uint32_t* d32 = reinterpret_cast<uint32_t*>(dst);
#pragma unroll
          for (int q = 0; q < static_cast<int>(D / 4); ++q) d32[q] = s32[q];
        }
      }
    } else {
      uint64_t* area = reinterpret_cast<uint64_t*>(lds);
      uint64_t* zero = area + kGroups * sp::kGroupSlots;
      if (threadIdx.x == 0) *zero = 0;
      __syncthreads();
      const uint32_t g = threadIdx.x / sp::kGroupLanes, t = threadIdx.x % sp::kGroupLanes;
      const uint64_t j = w * span + g;
      if (g < span && j < lv.m[l + 1]) {
        const uint8_t* src = nodes + lv.off[l] + 2 * j * D;
        uint32_t* d32 = reinterpret_cast<uint32_t*>(dst_of(l + 1, j));
        if (2 * j + 1 < lv.m[l]) {
          sp::SplitLane L;
          sp::setup(L, t, area + g * sp::kGroupSlots, zero);
          split_hash<V, false>(src, 2 * D, V, d32, static_cast<int>(D / 4), L);
        } else {
          const uint32_t* s32 = reinterpret_cast<const uint32_t*>(src);
          for (uint32_t q = t; q < D / 4; q += sp::kGroupLanes) d32[q] = s32[q];
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Scheduler kernels
// ---------------------------------------------------------------------------

__global__ void k_reset(uint32_t* __restrict__ meta, uint32_t words) {
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < words; k += gridDim.x * blockDim.x)
    meta[k] = 0u;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d);
  return v;
}

__device__ __forceinline__ uint32_t wave_max(uint32_t v) {
  for (int d = 32; d >= 1; d >>= 1) {
    const uint32_t o = __shfl_xor(v, d);
    v = o > v ? o : v;
  }
  return v;
}

template <int V>
__device__ __forceinline__ uint32_t key_at(const uint64_t* __restrict__ lens,
                                           const uint8_t* __restrict__ vars, uint64_t i) {
  return key_of(blocks_of<V>(lens[i], V == kMixed ? vars[i] : V));
}

// One 64-message chunk of arrival order (lane 0 always holds a message,
// `cnt` of the 64 lanes do).  When every message of the chunk has the same
// length and variant (the common case for uniform batches) the block count
// is worked out once and one LDS atomic records the chunk; otherwise every
// lane adds its own key and the chunk's idle lane-slots (cnt * max - sum)
// are accumulated.  `useful` and `idle` stay wave-uniform.
template <int V>
__device__ __forceinline__ void count_chunk(uint64_t len, int var, bool valid, uint32_t cnt,
                                            uint32_t lane, uint32_t* lhist, uint64_t& useful,
                                            uint64_t& idle, uint32_t& kmax) {
  const uint32_t lo0 = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(len));
  const uint32_t hi0 = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(len >> 32));
  const uint64_t len0 = (static_cast<uint64_t>(hi0) << 32) | lo0;
  const int var0 = V == kMixed ? __builtin_amdgcn_readfirstlane(var) : V;
  if (__ballot(valid && (len != len0 || var != var0)) == 0) {
    const uint32_t key = key_of(blocks_of<V>(len0, var0));
    if (lane == 0) atomicAdd(&lhist[key], cnt);
    useful += static_cast<uint64_t>(key) * cnt;
    kmax = key > kmax ? key : kmax;
  } else {
    const uint32_t key = valid ? key_of(blocks_of<V>(len, var)) : 0u;
    kmax = key > kmax ? key : kmax;
    if (valid) atomicAdd(&lhist[key], 1u);
    const uint32_t sm = wave_sum(key), mx = wave_max(key);
    useful += sm;
    idle += static_cast<uint64_t>(mx) * cnt - sm;
  }
}

// Inclusive prefix sum over the kBlock threads of a workgroup.
__device__ uint32_t block_inclusive_scan(uint32_t v, uint32_t* scratch) {
  const uint32_t t = threadIdx.x;
  scratch[t] = v;
  __syncthreads();
  for (uint32_t d = 1; d < kBlock; d <<= 1) {
    const uint32_t add = t >= d ? scratch[t - d] : 0u;
    __syncthreads();
    scratch[t] += add;
    __syncthreads();
  }
  const uint32_t r = scratch[t];
  __syncthreads();
  return r;
}

// Messages per queue item in a bucket of `key` blocks: 64 lanes times enough
// messages that one item is about `steps` permutations per lane.
__device__ __forceinline__ uint32_t item_msgs(uint32_t key, uint32_t steps) {
  const uint32_t g = key >= steps ? 1u : steps / (key ? key : 1u);
  return 64u * g;
}

// The plan: keep
// arrival order if it idles at most 2 % of the lane slots (and no sort is
// forced), else bucket starts in descending block count.  Bucket rank
// r = kKeyBins - 1 - key orders buckets longest first; thread t owns ranks
// 16t .. 16t+15.  Writes the bucket starts (start[key]), the inclusive prefix
// of queue items per rank (iend[r]) and the queue size.
constexpr uint32_t kRanksPerThread = kKeyBins / kBlock;

// The first CTL_SPLIT_N positions of the bucketed order (the longest
// messages) go to the split form: the messages of at least
// max(kSplitMinKey, 4 x the mean, 2 x the blocks per resident lane) blocks,
// at most `split_cap` of them.  Below the last bound the batch's throughput,
// not its longest chain, sets the time, and a split item (eight messages per
// wave) costs throughput.
constexpr uint32_t kSplitMinKey = 32;

__device__ void make_plan(uint32_t* __restrict__ hist, const uint32_t* __restrict__ hist_copies,
                          const uint32_t* __restrict__ partials, uint32_t* __restrict__ start,
                          uint32_t* __restrict__ iend, uint32_t* __restrict__ ctl, uint64_t n,
                          uint32_t steps, int force_sort, uint32_t split_cap, uint64_t lanes,
                          uint32_t* scratch) {
  __shared__ uint32_t identity, split_n;
  const uint32_t t = threadIdx.x;
  uint64_t useful = 0, idle = 0;
  uint32_t maxkey = 0;
#pragma unroll
  for (uint32_t c = 0; c < kCopies; ++c) {
    const uint32_t* pc = partials + c * kPartialWords;
    useful += *reinterpret_cast<const unsigned long long*>(pc + P_USEFUL);
    idle += *reinterpret_cast<const unsigned long long*>(pc + P_IDLE);
    maxkey = pc[P_MAXKEY] > maxkey ? pc[P_MAXKEY] : maxkey;
  }
  if (t == 0) {
    *reinterpret_cast<unsigned long long*>(&ctl[CTL_USEFUL]) = useful;
    *reinterpret_cast<unsigned long long*>(&ctl[CTL_IDLE]) = idle;
    ctl[CTL_MAXKEY] = maxkey;
  }
  const uint64_t avg = useful / (n ? n : 1);
  if (t == 0) {
    identity = (!force_sort && idle * 50u <= useful) ? 1u : 0u;
    ctl[CTL_IDENTITY] = identity;
    ctl[CTL_PRIO_KEY] = static_cast<uint32_t>(2u * avg + 2u);
    if (identity) {
      const uint32_t per = item_msgs(avg > 0xFFFFu ? 0xFFFFu : static_cast<uint32_t>(avg), 8u);
      ctl[CTL_ID_PER] = per;
      ctl[CTL_NITEMS] = static_cast<uint32_t>((n + per - 1) / per);
    }
  }
  __syncthreads();
  if (identity) return;
  // This thread's ranks are the 16 consecutive keys lo .. lo + 15 (64-byte
  // aligned): fold the copies with 16-byte loads, all issued before use.
  static_assert(kRanksPerThread == 16, "four 16-byte loads per copy");
  const uint32_t lo = kKeyBins - kRanksPerThread * (t + 1u);
  uint4 part[kCopies][4];
#pragma unroll
  for (uint32_t k = 0; k < kCopies; ++k) {
    const uint4* src = reinterpret_cast<const uint4*>((k ? hist_copies + (k - 1) * kKeyBins : hist) + lo);
#pragma unroll
    for (int v = 0; v < 4; ++v) part[k][v] = src[v];
  }
  uint32_t byk[kRanksPerThread];  // folded count of key lo + i
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    uint4 a = part[0][v];
#pragma unroll
    for (uint32_t k = 1; k < kCopies; ++k) {
      a.x += part[k][v].x;
      a.y += part[k][v].y;
      a.z += part[k][v].z;
      a.w += part[k][v].w;
    }
    byk[4 * v] = a.x;
    byk[4 * v + 1] = a.y;
    byk[4 * v + 2] = a.z;
    byk[4 * v + 3] = a.w;
    // the folded histogram, read by k_fill and the per-bucket form
    reinterpret_cast<uint4*>(hist + lo)[v] = a;
  }
  uint32_t cnt[kRanksPerThread], st[kRanksPerThread], c_sum = 0;
#pragma unroll
  for (uint32_t q = 0; q < kRanksPerThread; ++q) {
    const uint32_t key = kKeyBins - 1u - (kRanksPerThread * t + q);  // = lo + 15 - q
    cnt[q] = key ? byk[kRanksPerThread - 1u - q] : 0u;
    c_sum += cnt[q];
  }
  uint32_t c_base = block_inclusive_scan(c_sum, scratch) - c_sum;
  // bucket starts; the split range ends where the keys drop below kmin
  const uint64_t per_lane = 2u * useful / (lanes ? lanes : 1u);
  uint64_t kmin64 = 4u * avg > kSplitMinKey ? 4u * avg : kSplitMinKey;
  if (per_lane > kmin64) kmin64 = per_lane;
  const uint32_t kmin = kmin64 < kKeyBins - 1u ? static_cast<uint32_t>(kmin64) : kKeyBins - 1u;
  if (t == 0) split_n = static_cast<uint32_t>(n);  // every key at least kmin
#pragma unroll
  for (uint32_t q = 0; q < kRanksPerThread; ++q) {
    const uint32_t key = kKeyBins - 1u - (kRanksPerThread * t + q);
    st[q] = c_base;
    start[key] = c_base;
    c_base += cnt[q];
  }
  __syncthreads();
#pragma unroll
  for (uint32_t q = 0; q < kRanksPerThread; ++q) {
    const uint32_t key = kKeyBins - 1u - (kRanksPerThread * t + q);
    if (key == kmin - 1u) split_n = st[q];  // messages in buckets of key >= kmin
  }
  __syncthreads();
  const uint32_t split = split_n < split_cap ? split_n : split_cap;
  // queue items over the positions past the split range
  uint32_t items[kRanksPerThread], it_sum = 0;
#pragma unroll
  for (uint32_t q = 0; q < kRanksPerThread; ++q) {
    const uint32_t key = kKeyBins - 1u - (kRanksPerThread * t + q);
    const uint32_t b = st[q] > split ? st[q] : split, e = st[q] + cnt[q];
    const uint32_t per = item_msgs(key, steps);
    items[q] = e > b ? (e - b + per - 1u) / per : 0u;
    it_sum += items[q];
  }
  uint32_t it_run = block_inclusive_scan(it_sum, scratch) - it_sum;
#pragma unroll
  for (uint32_t q = 0; q < kRanksPerThread; ++q) {
    it_run += items[q];
    iend[kRanksPerThread * t + q] = it_run;
  }
  if (t == kBlock - 1) {
    ctl[CTL_NITEMS] = it_run;
    ctl[CTL_SPLIT_N] = split;
  }
}

// One workgroup makes the plan once the histogram is complete.  (Folding
// this into the last workgroup of k_count costs more than the launch: every
// workgroup must then fence and wait for its histogram atomics before
// drawing a ticket.)
__global__ __launch_bounds__(kBlock) void k_plan(uint32_t* __restrict__ hist,
                                                 const uint32_t* __restrict__ hist_copies,
                                                 const uint32_t* __restrict__ partials,
                                                 uint32_t* __restrict__ start,
                                                 uint32_t* __restrict__ iend,
                                                 uint32_t* __restrict__ ctl, uint64_t n,
                                                 uint32_t steps, int force_sort,
                                                 uint32_t split_cap, uint64_t lanes) {
  __shared__ uint32_t scratch[kBlock];
  make_plan(hist, hist_copies, partials, start, iend, ctl, n, steps, force_sort, split_cap, lanes,
            scratch);
}

// Two 64-message chunks of arrival order, messages 2 lane and 2 lane + 1 of
// a 128-message pair in each lane (lanes 0-31 hold the first chunk, 32-63
// the second).  Same accounting as count_chunk, with one LDS atomic for the
// pair when all 128 lengths and variants are equal.
template <int V>
__device__ __forceinline__ void count_pair(uint64_t la, uint64_t lb, int va, int vb, uint32_t lane,
                                           uint32_t* lhist, uint64_t& useful, uint64_t& idle,
                                           uint32_t& kmax) {
  const uint32_t lo0 = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(la));
  const uint32_t hi0 = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(la >> 32));
  const uint64_t len0 = (static_cast<uint64_t>(hi0) << 32) | lo0;
  const int var0 = V == kMixed ? __builtin_amdgcn_readfirstlane(va) : V;
  if (__ballot(la != len0 || lb != len0 || va != var0 || vb != var0) == 0) {
    const uint32_t key = key_of(blocks_of<V>(len0, var0));
    if (lane == 0) atomicAdd(&lhist[key], 128u);
    useful += static_cast<uint64_t>(key) * 128u;
    kmax = key > kmax ? key : kmax;
  } else {
    const uint32_t ka = key_of(blocks_of<V>(la, va)), kb = key_of(blocks_of<V>(lb, vb));
    atomicAdd(&lhist[ka], 1u);
    atomicAdd(&lhist[kb], 1u);
    uint32_t sm = ka + kb, mx = ka > kb ? ka : kb;
    kmax = mx > kmax ? mx : kmax;
    for (int d = 16; d >= 1; d >>= 1) {  // within each half of the wave
      sm += __shfl_xor(sm, d);
      const uint32_t o = __shfl_xor(mx, d);
      mx = o > mx ? o : mx;
    }
    const uint32_t s0 = __builtin_amdgcn_readlane(sm, 0), s1 = __builtin_amdgcn_readlane(sm, 32);
    const uint32_t m0 = __builtin_amdgcn_readlane(mx, 0), m1 = __builtin_amdgcn_readlane(mx, 32);
    useful += static_cast<uint64_t>(s0) + s1;
    idle += (64ull * m0 - s0) + (64ull * m1 - s1);
  }
}

// Histogram of block-count keys and the lane slots arrival order would
// idle, into copy blockIdx.x mod kCopies of the histogram and the control
// partials.  A wave takes kCountUnroll whole 128-message pairs per pass, two
// adjacent lengths per lane, and issues all their loads before using any;
// the chunks past the last whole pass (and the ragged last chunk) are taken
// one at a time with bounds checks.
constexpr int kCountUnroll = 8;

template <int V>
__global__ __launch_bounds__(kBlock) void k_count(const uint64_t* __restrict__ lens,
                                                  const uint8_t* __restrict__ vars, uint64_t n,
                                                  uint32_t* __restrict__ hist,
                                                  uint32_t* __restrict__ hist_copies,
                                                  uint32_t* __restrict__ partials) {
  __shared__ uint32_t lhist[kKeyBins];
  __shared__ unsigned long long luseful, lidle;
  __shared__ uint32_t lmax;
  for (uint32_t k = threadIdx.x; k < kKeyBins; k += kBlock) lhist[k] = 0u;
  if (threadIdx.x == 0) {
    luseful = 0ull;
    lidle = 0ull;
    lmax = 0u;
  }
  __syncthreads();
  const uint32_t lane = threadIdx.x & 63u;
  const uint64_t waves = static_cast<uint64_t>(gridDim.x) * (kBlock / 64);
  const uint64_t wave_id = static_cast<uint64_t>(blockIdx.x) * (kBlock / 64) + threadIdx.x / 64;
  uint64_t useful = 0, idle = 0;
  uint32_t kmax = 0;
  const uint64_t passes = (n / 128u) / kCountUnroll;  // passes of whole pairs
  for (uint64_t g = wave_id; g < passes; g += waves) {
    uint64_t la[kCountUnroll], lb[kCountUnroll];
    int va[kCountUnroll], vb[kCountUnroll];
#pragma unroll
    for (int u = 0; u < kCountUnroll; ++u) {
      const uint64_t i = (g * kCountUnroll + u) * 128u + 2u * lane;
      la[u] = lens[i];
      lb[u] = lens[i + 1];
      va[u] = vb[u] = V;
      if constexpr (V == kMixed) {
        va[u] = vars[i];
        vb[u] = vars[i + 1];
      }
    }
#pragma unroll
    for (int u = 0; u < kCountUnroll; ++u)
      count_pair<V>(la[u], lb[u], va[u], vb[u], lane, lhist, useful, idle, kmax);
  }
  for (uint64_t c = passes * kCountUnroll * 2u + wave_id; c * 64u < n; c += waves) {
    const uint64_t i = c * 64u + lane;
    const bool valid = i < n;
    const uint64_t len = valid ? lens[i] : 0u;
    const int var = V == kMixed ? (valid ? vars[i] : 0) : V;
    const uint32_t cnt = n - c * 64u < 64u ? static_cast<uint32_t>(n - c * 64u) : 64u;
    count_chunk<V>(len, var, valid, cnt, lane, lhist, useful, idle, kmax);
  }
  if (lane == 0) {
    atomicAdd(&luseful, static_cast<unsigned long long>(useful));
    atomicAdd(&lidle, static_cast<unsigned long long>(idle));
  }
  atomicMax(&lmax, kmax);
  __syncthreads();
  const uint32_t copy = blockIdx.x % kCopies;
  uint32_t* h = copy ? hist_copies + (copy - 1u) * kKeyBins : hist;
  for (uint32_t k = threadIdx.x; k < kKeyBins; k += kBlock)
    if (lhist[k]) atomicAdd(&h[k], lhist[k]);
  if (threadIdx.x == 0) {
    uint32_t* pc = partials + copy * kPartialWords;
    atomicAdd(reinterpret_cast<unsigned long long*>(pc + P_USEFUL), luseful);
    atomicAdd(reinterpret_cast<unsigned long long*>(pc + P_IDLE), lidle);
    atomicMax(pc + P_MAXKEY, lmax);
  }
}

// Queue item t: its bucket (the smallest rank r with iend[r] > t) and its
// range of positions in the bucketed order.
__device__ __forceinline__ void items_block(uint32_t blk, const uint32_t* __restrict__ hist,
                                            const uint32_t* __restrict__ start,
                                            const uint32_t* __restrict__ iend,
                                            const uint32_t* __restrict__ ctl, uint64_t n,
                                            uint32_t steps, WorkItem* __restrict__ items) {
  const uint32_t t = blk * kBlock + threadIdx.x;
  if (t >= ctl[CTL_NITEMS]) return;
  if (ctl[CTL_IDENTITY]) {
    const uint64_t per = ctl[CTL_ID_PER];
    const uint64_t b = t * per, e = b + per < n ? b + per : n;
    items[t] = WorkItem{static_cast<uint32_t>(b), static_cast<uint32_t>(e), 0u, 0u};
    return;
  }
  uint32_t lo = 0, hi = kKeyBins - 1;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (iend[mid] > t)
      hi = mid;
    else
      lo = mid + 1;
  }
  const uint32_t key = kKeyBins - 1u - lo;
  const uint32_t per = item_msgs(key, steps);
  const uint32_t first_item = lo ? iend[lo - 1] : 0u;
  const uint32_t split = ctl[CTL_SPLIT_N];  // positions before it are split work
  const uint32_t b = (start[key] > split ? start[key] : split) + (t - first_item) * per;
  const uint32_t bucket_end = start[key] + hist[key];
  items[t] = WorkItem{b, b + per < bucket_end ? b + per : bucket_end, key, 0u};
}

// Counting-sort scatter: workgroup w handles messages [w * tile, (w+1) * tile),
// reserves one range per non-empty bucket with a single global atomic, and
// ranks its messages inside each range with LDS atomics.
template <int V>
__device__ __forceinline__ void scatter_block(uint32_t blk, const uint64_t* __restrict__ lens,
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
  const uint64_t first = static_cast<uint64_t>(blk) * kScatterTile;
  const uint64_t last = first + kScatterTile < n ? first + kScatterTile : n;
  uint32_t keys[kScatterTile / kBlock];
#pragma unroll
  for (int q = 0; q < kScatterTile / kBlock; ++q) {
    const uint64_t i = first + static_cast<uint64_t>(q) * kBlock + threadIdx.x;
    keys[q] = i < last ? key_at<V>(lens, vars, i) : 0u;
    if (i < last) atomicAdd(&lcount[keys[q]], 1u);
  }
  __syncthreads();
  for (uint32_t k = threadIdx.x; k < kKeyBins; k += kBlock) {
    const uint32_t c = lcount[k];
    lbase[k] = c ? start[k] + atomicAdd(&cursor[k], c) : 0u;
    lcount[k] = 0u;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kScatterTile / kBlock; ++q) {
    const uint64_t i = first + static_cast<uint64_t>(q) * kBlock + threadIdx.x;
    if (i < last) {
      const uint32_t rank = atomicAdd(&lcount[keys[q]], 1u);
      order[lbase[keys[q]] + rank] = static_cast<uint32_t>(i);
    }
  }
}

// Queue items and the scatter in one launch (both depend only on the plan):
// workgroups [0, iblocks) write queue items, the rest scatter the order.
template <int V>
__global__ __launch_bounds__(kBlock) void k_fill(const uint64_t* __restrict__ lens,
                                                 const uint8_t* __restrict__ vars, uint64_t n,
                                                 const uint32_t* __restrict__ hist,
                                                 const uint32_t* __restrict__ start,
                                                 uint32_t* __restrict__ cursor,
                                                 const uint32_t* __restrict__ iend,
                                                 const uint32_t* __restrict__ ctl, uint32_t steps,
                                                 uint32_t iblocks, WorkItem* __restrict__ items,
                                                 uint32_t* __restrict__ order) {
  if (blockIdx.x < iblocks)
    items_block(blockIdx.x, hist, start, iend, ctl, n, steps, items);
  else
    scatter_block<V>(blockIdx.x - iblocks, lens, vars, n, start, cursor, ctl, order);
}

// Count the dwords where two digest buffers differ (autotuner parity gate).
__global__ __launch_bounds__(kBlock) void k_compare(const uint32_t* __restrict__ a,
                                                    const uint32_t* __restrict__ b, uint64_t words,
                                                    unsigned long long* __restrict__ mismatches) {
  unsigned long long c = 0;
  for (uint64_t k = static_cast<uint64_t>(blockIdx.x) * kBlock + threadIdx.x; k < words;
       k += static_cast<uint64_t>(gridDim.x) * kBlock)
    c += a[k] != b[k];
  if (c) atomicAdd(mismatches, c);
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
  uint32_t* meta = nullptr;  // hist | start | cursor | iend | ctl | sub-queues | simd flags
  uint32_t* order = nullptr;
  uint64_t order_cap = 0;
  WorkItem* items = nullptr;
  uint64_t items_cap = 0;
  uint8_t* tree = nullptr;
  uint64_t tree_cap = 0;
  uint32_t* host_hist = nullptr;  // pinned, for the per-bucket form
};

constexpr uint32_t kMetaWords = kPartialsOff + kCopies * kPartialWords;

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
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
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

// Queue items of a batch of n messages: ceil(n / 64) in arrival order, or at
// most one partial item per bucket more than that when bucketed.
uint64_t max_items(uint64_t n) { return n / 64 + kKeyBins + 1; }

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
    const uint64_t items = max_items(msgs);
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
  int variant;  // 0..3, kMixed, kShake128 or kShake256
  const uint8_t* vars;
  const uint8_t* data;
  const uint64_t* offs;
  const uint64_t* lens;
  uint64_t n;
  uint8_t* out;
  uint64_t stride = 0;  // output bytes per message
};

uint64_t out_stride(int v) {
  return v == kMixed ? 64u : static_cast<uint64_t>(kb::digest_bytes_of(v));
}

template <int V>
int launch_plain(const Batch& b, const uint32_t* order, uint64_t first, uint64_t count,
                 hipStream_t s) {
  if (!count) return KB_OK;
  const uint64_t blocks = (count + kBlock - 1) / kBlock;
  if (blocks > 0x7FFFFFFFull) return fail(KB_EINVAL, "batch too large for one launch");
  {
    TimedLaunch tl(s);
    hipLaunchKernelGGL(k_plain<V>, dim3(static_cast<uint32_t>(blocks)), dim3(kBlock), 0, s,
                       b.data, b.offs, b.lens, b.vars, order, first, count, b.out, b.stride);
  }
  KB_HIP(hipGetLastError());
  return KB_OK;
}

template <int V>
int launch_split(const Batch& b, const uint32_t* order, uint64_t first, uint64_t count,
                 hipStream_t s) {
  if (!count) return KB_OK;
  int dev = 0, cus = 0;
  KB_HIP(hipGetDevice(&dev));
  int rc = cu_count(dev, &cus);
  if (rc) return rc;
  // one group per message up to 16 waves per CU; beyond that groups loop
  uint64_t grid = (count + kSplitGroups - 1) / kSplitGroups;
  if (grid > static_cast<uint64_t>(16 * cus)) grid = 16 * cus;
  {
    TimedLaunch tl(s);
    hipLaunchKernelGGL(k_split<V>, dim3(static_cast<uint32_t>(grid)), dim3(kSplitBlock), 0, s,
                       b.data, b.offs, b.lens, b.vars, order, first, count, b.out, b.stride);
  }
  KB_HIP(hipGetLastError());
  return KB_OK;
}

template <int V>
int run_schedule(const Batch& b, Workspace& w, uint32_t steps, int force_sort, uint64_t lanes,
                 hipStream_t s) {
  uint32_t* hist = w.meta;
  uint32_t* start = w.meta + kKeyBins;
  uint32_t* cursor = w.meta + 2 * kKeyBins;
  uint32_t* iend = w.meta + 3 * kKeyBins;
  uint32_t* ctl = w.meta + 4 * kKeyBins;
  int dev = 0, cus = 0;
  KB_HIP(hipGetDevice(&dev));
  int rc = cu_count(dev, &cus);
  if (rc) return rc;
  hipLaunchKernelGGL(k_reset, dim3(64), dim3(256), 0, s, w.meta, kMetaWords);
  KB_HIP(hipGetLastError());
  // about 2 passes of 4 waves x kCountUnroll 128-message pairs per workgroup,
  // at most 2 workgroups per CU: the workgroups' closing atomics serialise per
  // address, so fewer, longer workgroups finish sooner (on 2^24 lengths the
  // whole schedule costs 48 us at 2 per CU, 54 at 4 and 65 at 8)
  const uint64_t per_wg = 128ull * 4 * kCountUnroll * 2;
  uint64_t cblocks = (b.n + per_wg - 1) / per_wg;
  if (cblocks > static_cast<uint64_t>(2 * cus)) cblocks = 2 * cus;
  hipLaunchKernelGGL(k_count<V>, dim3(static_cast<uint32_t>(cblocks)), dim3(kBlock), 0, s, b.lens,
                     b.vars, b.n, hist, w.meta + kHistCopiesOff, w.meta + kPartialsOff);
  KB_HIP(hipGetLastError());
  // at most eight split messages per SIMD: one 8-group split item for each
  // SIMD's front wave (mixed-variant kernel only; the per-bucket form takes
  // none)
  const uint32_t split_cap = V == kMixed && !force_sort ? 8u * 4u * static_cast<uint32_t>(cus) : 0u;
  hipLaunchKernelGGL(k_plan, dim3(1), dim3(kBlock), 0, s, hist, w.meta + kHistCopiesOff,
                     w.meta + kPartialsOff, start, iend, ctl, b.n, steps, force_sort, split_cap,
                     lanes);
  KB_HIP(hipGetLastError());
  const uint64_t iblocks = (max_items(b.n) + kBlock - 1) / kBlock;
  const uint64_t sblocks = (b.n + kScatterTile - 1) / kScatterTile;
  hipLaunchKernelGGL(k_fill<V>, dim3(static_cast<uint32_t>(iblocks + sblocks)), dim3(kBlock), 0, s,
                     b.lens, b.vars, b.n, hist, start, cursor, iend, ctl, steps,
                     static_cast<uint32_t>(iblocks), w.items, w.order);
  KB_HIP(hipGetLastError());
  return KB_OK;
}

template <int V>
int run_batch(const Batch& b, int mode, const kb_tile* tile, hipStream_t s, Workspace* own) {
  if (mode == KB_MODE_PLAIN) return launch_plain<V>(b, nullptr, 0, b.n, s);
  if (mode == KB_MODE_SPLIT) return launch_split<V>(b, nullptr, 0, b.n, s);
  if (b.n >= 0xFFFFFFFFull) return launch_plain<V>(b, nullptr, 0, b.n, s);  // 32-bit order[]
  Workspace* w = own;
  int rc = own ? KB_OK : get_ws(s, b.n, 0, &w);
  if (rc) return rc;
  uint32_t steps = tile && tile->steps_per_item > 0 ? static_cast<uint32_t>(tile->steps_per_item) : 4u;
  if (mode == KB_MODE_PER_BUCKET) {
    rc = run_schedule<V>(b, *w, steps, 1, 0, s);
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
  rc = run_schedule<V>(b, *w, steps, 0, static_cast<uint64_t>(grid) * kBlock, s);
  if (rc) return rc;
  {
    TimedLaunch tl(s);
    hipLaunchKernelGGL(k_persistent<V>, dim3(grid), dim3(kBlock), 0, s, b.data, b.offs, b.lens,
                       b.vars, w->order, w->items, w->meta + 4 * kKeyBins,
                       reinterpret_cast<unsigned long long*>(w->meta + 4 * kKeyBins + CTL_WORDS),
                       w->meta + 4 * kKeyBins + CTL_WORDS + kQueueAreaDw, b.out,
                       b.stride);
  }
  KB_HIP(hipGetLastError());
  return KB_OK;
}

// `own`: a caller-owned workspace (a captured graph's), else the stream's.
int dispatch(const Batch& b, int mode, const kb_tile* tile, hipStream_t s, Workspace* own = nullptr) {
  switch (b.variant) {
    case 0: return run_batch<0>(b, mode, tile, s, own);
    case 1: return run_batch<1>(b, mode, tile, s, own);
    case 2: return run_batch<2>(b, mode, tile, s, own);
    case 3: return run_batch<3>(b, mode, tile, s, own);
    case kShake128: return run_batch<kShake128>(b, mode, tile, s, own);
    case kShake256: return run_batch<kShake256>(b, mode, tile, s, own);
    default: return run_batch<kMixed>(b, mode, tile, s, own);
  }
}

int check_batch(const Batch& b, int mode) {
  if (b.variant != kMixed && b.variant != kShake128 && b.variant != kShake256 &&
      (b.variant < 0 || b.variant > 3))
    return fail(KB_EINVAL, "variant %d is not a SHA-3 variant (0..3)", b.variant);
  if (mode < KB_MODE_PERSISTENT || mode > KB_MODE_SPLIT)
    return fail(KB_EINVAL, "unknown scheduling mode %d", mode);
  if (b.n == 0) return KB_OK;
  if (!b.data || !b.offs || !b.lens || !b.out || (b.variant == kMixed && !b.vars))
    return fail(KB_EINVAL, "NULL pointer with n > 0");
  if (reinterpret_cast<uintptr_t>(b.offs) % 8 || reinterpret_cast<uintptr_t>(b.lens) % 8)
    return fail(KB_EINVAL, "d_offsets and d_lengths must be 8-byte aligned");
  if (b.variant < kShake128 && reinterpret_cast<uintptr_t>(b.out) % 4)
    return fail(KB_EINVAL, "d_digests must be 4-byte aligned");
  return KB_OK;
}

int batch_entry(int variant, const uint8_t* vars, const uint8_t* data, const uint64_t* offs,
                const uint64_t* lens, uint64_t n, uint8_t* out, int mode, const kb_tile* tile,
                hipStream_t s) {
  g_err.clear();
  if (tile && tile->block_threads != 0 && tile->block_threads != kBlock)
    return fail(KB_EINVAL, "tile.block_threads must be 0 or %d", kBlock);
  Batch b{variant, vars, data, offs, lens, n, out, out_stride(variant)};
  int rc = check_batch(b, mode);
  if (rc || n == 0) return rc;
  return dispatch(b, mode, tile, s);
}

// The levels of a tree over `leaves` leaf digests of D bytes: level l has
// m[l] = ceil(m[l-1] / 2) nodes stored from byte off[l] of the node buffer
// (each level starts 16-byte aligned, so every node pair is 8-byte
// aligned).  Returns L, the number of levels above the leaves.  Level L is
// the root, which goes to the caller's buffer, so the node buffer needs
// off[L] bytes; tree_workspace_bytes() adds one digest of slack.
int tree_levels(uint64_t leaves, uint64_t D, TreeLevels& lv) {
  lv = TreeLevels{};
  lv.m[0] = leaves ? leaves : 1;
  lv.off[0] = 0;
  int L = 0;
  while (lv.m[L] > 1) {
    lv.m[L + 1] = (lv.m[L] + 1) / 2;
    lv.off[L + 1] = (lv.off[L] + lv.m[L] * D + 15u) & ~uint64_t{15};
    ++L;
  }
  return L;
}

// Node-buffer bytes of a tree over `leaves` leaves of D-byte digests; it
// grows with D, so D = 64 sizes a buffer for every variant.
uint64_t tree_workspace_bytes(uint64_t leaves, uint64_t D) {
  TreeLevels lv;
  const int L = tree_levels(leaves, D, lv);
  return lv.off[L] + D;
}

template <int V>
int merkle_impl(const uint8_t* data, uint64_t total, uint64_t leaf, uint8_t* root, hipStream_t s,
                Workspace* own) {
  constexpr uint64_t D = kb::digest_bytes_of(V);
  TreeLevels lv;
  const int L = tree_levels(total ? (total + leaf - 1) / leaf : 1, D, lv);  // levels above the leaves
  // leaves of whole 8-byte words at 8-byte-aligned addresses take the W8 kernel
  const bool w8 = leaf % 8u == 0 && total % 8u == 0 && reinterpret_cast<uintptr_t>(data) % 8u == 0;
  Workspace* w = own;
  int rc = own ? KB_OK : get_ws(s, 0, lv.off[L] + D, &w);
  if (rc) return rc;
  // The leaves and the first level in 256-thread workgroups, then launches of
  // up to 8 levels while over kTreeTop nodes remain, then one workgroup of
  // kTreeTopThreads threads reduces the rest.  The root is written by
  // whichever launch produces level L (the leaf launch itself for one or two
  // leaves).  A leaf workgroup that went on with its narrow levels would hold
  // its CU slot while few lanes work: one level there measured about 1 %
  // faster per root than eight.
  int first = 0;
  do {
    if (first == 0 || lv.m[first] > static_cast<uint64_t>(kTreeTop)) {
      const int cap = first == 0 ? 1 : 8;
      const int levels = L - first < cap ? L - first : cap;
      const uint64_t blocks = (lv.m[first] + kBlock - 1) / kBlock;
      {
        TimedLaunch tl(s);
        if (w8 || first > 0)
          hipLaunchKernelGGL((k_tree<V, kBlock, kb::kPrefetch<V>, true>),
                             dim3(static_cast<uint32_t>(blocks)), dim3(kBlock), 0, s, data, total,
                             leaf, w->tree, root, first, levels, L, lv);
        else
          hipLaunchKernelGGL((k_tree<V, kBlock, kb::kPrefetch<V>, false>),
                             dim3(static_cast<uint32_t>(blocks)), dim3(kBlock), 0, s, data, total,
                             leaf, w->tree, root, first, levels, L, lv);
      }
      KB_HIP(hipGetLastError());
      first += levels;
    } else {
      {
        TimedLaunch tl(s);
        hipLaunchKernelGGL((k_tree<V, kTreeTopThreads, false, true, kTreeTop>), dim3(1),
                           dim3(kTreeTopThreads), 0, s, data, total, leaf, w->tree, root, first,
                           L - first, L, lv);
      }
      KB_HIP(hipGetLastError());
      first = L;
    }
  } while (first < L);
  return KB_OK;
}

// Median of a small vector (modifies it).
double median(std::vector<double>& v) {
  std::sort(v.begin(), v.end());
  return v.empty() ? 0.0 : v[v.size() / 2];
}

struct GraphHolder {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

}  // namespace

struct kb_graph {
  GraphHolder h;
  Workspace ws;  // private: captured kernels point into it
};

namespace {

void free_ws(Workspace& w) {
  if (w.meta) (void)hipFree(w.meta);
  if (w.order) (void)hipFree(w.order);
  if (w.items) (void)hipFree(w.items);
  if (w.tree) (void)hipFree(w.tree);
  if (w.host_hist) (void)hipHostFree(w.host_hist);
  w = Workspace{};
}

// Size a graph's private workspace for `msgs` messages and `tree_bytes`.
int size_ws(Workspace& w, uint64_t msgs, uint64_t tree_bytes, hipStream_t s) {
  uint64_t cap = 0;
  int rc = grow(reinterpret_cast<void**>(&w.meta), &cap, kMetaWords * 4ull, s);
  if (!rc && msgs) rc = grow(reinterpret_cast<void**>(&w.order), &w.order_cap, msgs * 4ull, s);
  if (!rc && msgs)
    rc = grow(reinterpret_cast<void**>(&w.items), &w.items_cap, max_items(msgs) * sizeof(WorkItem), s);
  if (!rc && tree_bytes) rc = grow(reinterpret_cast<void**>(&w.tree), &w.tree_cap, tree_bytes, s);
  return rc;
}

// Capture whatever `enqueue` puts on `stream` into a graph that owns `g`.
template <class F>
int capture(hipStream_t stream, F&& enqueue, kb_graph* g, kb_graph** out) {
  // The null stream cannot be captured; record on a private stream then (a
  // graph remembers its nodes, not the stream it was recorded on).
  hipStream_t own = nullptr;
  if (!stream) {
    const hipError_t ec = hipStreamCreateWithFlags(&own, hipStreamNonBlocking);
    if (ec != hipSuccess) {
      free_ws(g->ws);
      delete g;
      return fail(KB_EHIP, "hipStreamCreateWithFlags: %s", hipGetErrorString(ec));
    }
    stream = own;
  }
  const hipError_t eb = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal);
  if (eb != hipSuccess) {
    if (own) (void)hipStreamDestroy(own);
    free_ws(g->ws);
    delete g;
    return fail(KB_EHIP, "hipStreamBeginCapture: %s", hipGetErrorString(eb));
  }
  int rc = enqueue(stream);
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(stream, &graph);
  if (own) (void)hipStreamDestroy(own);
  hipGraphExec_t exec = nullptr;
  if (rc == KB_OK && e != hipSuccess) rc = fail(KB_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
  if (rc == KB_OK) {
    const hipError_t e2 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e2 != hipSuccess) rc = fail(KB_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e2));
  }
  if (rc != KB_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    free_ws(g->ws);
    delete g;
    return rc;
  }
  g->h.graph = graph;
  g->h.exec = exec;
  *out = g;
  return KB_OK;
}

}  // namespace

namespace kb {
int set_last_error(int code, const char* msg) {
  g_err = msg ? msg : "";
  return code;
}
}  // namespace kb

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

int keccak_batch_xof(int security, const uint8_t* d_data, const uint64_t* d_offsets,
                     const uint64_t* d_lengths, uint64_t n, uint64_t out_len, uint8_t* d_out,
                     hipStream_t stream) {
  g_err.clear();
  if (security != 128 && security != 256)
    return fail(KB_EINVAL, "SHAKE security level must be 128 or 256, not %d", security);
  if (n && out_len == 0) return fail(KB_EINVAL, "out_len must be positive");
  Batch b{security == 128 ? kShake128 : kShake256, nullptr, d_data, d_offsets, d_lengths, n,
          d_out, out_len};
  int rc = check_batch(b, KB_MODE_PERSISTENT);
  if (rc || n == 0) return rc;
  return dispatch(b, KB_MODE_PERSISTENT, nullptr, stream);
}

int keccak_batch_xof_ex(int security, const uint8_t* d_data, const uint64_t* d_offsets,
                        const uint64_t* d_lengths, uint64_t n, uint64_t out_len, uint8_t* d_out,
                        int mode, hipStream_t stream) {
  g_err.clear();
  if (security != 128 && security != 256)
    return fail(KB_EINVAL, "SHAKE security level must be 128 or 256, not %d", security);
  if (n && out_len == 0) return fail(KB_EINVAL, "out_len must be positive");
  Batch b{security == 128 ? kShake128 : kShake256, nullptr, d_data, d_offsets, d_lengths, n,
          d_out, out_len};
  int rc = check_batch(b, mode);
  if (rc || n == 0) return rc;
  return dispatch(b, mode, nullptr, stream);
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
    case 0: return merkle_impl<0>(d_data, total_len, leaf_size, d_root, stream, nullptr);
    case 1: return merkle_impl<1>(d_data, total_len, leaf_size, d_root, stream, nullptr);
    case 2: return merkle_impl<2>(d_data, total_len, leaf_size, d_root, stream, nullptr);
    default: return merkle_impl<3>(d_data, total_len, leaf_size, d_root, stream, nullptr);
  }
}

int keccak_autotune(int variant, const uint8_t* d_variants, const uint8_t* d_data,
                    const uint64_t* d_offsets, const uint64_t* d_lengths, uint64_t n, int reps,
                    kb_tile* best, double* best_ms, int* rejected, hipStream_t stream) {
  g_err.clear();
  if (!best || !best_ms || !rejected) return fail(KB_EINVAL, "NULL output pointer");
  if (variant != -1 && (variant < 0 || variant > 3))
    return fail(KB_EINVAL, "variant %d is neither -1 (mixed) nor a SHA-3 variant", variant);
  const int v = variant == -1 ? kMixed : variant;
  Batch b{v, d_variants, d_data, d_offsets, d_lengths, n, nullptr, out_stride(v)};
  int rc = check_batch(Batch{v, d_variants, d_data, d_offsets, d_lengths, n,
                             reinterpret_cast<uint8_t*>(uintptr_t{256}), 0},
                       KB_MODE_PERSISTENT);
  if (rc) return rc;
  if (n == 0) return fail(KB_EINVAL, "nothing to tune on an empty batch");
  if (reps < 1) reps = 1;
  const uint64_t bytes = n * out_stride(v);
  uint8_t *ref = nullptr, *cand = nullptr;
  unsigned long long* mism = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto cleanup = [&]() {
    if (ref) (void)hipFree(ref);
    if (cand) (void)hipFree(cand);
    if (mism) (void)hipFree(mism);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  if (hipMalloc(&ref, bytes) != hipSuccess || hipMalloc(&cand, bytes) != hipSuccess ||
      hipMalloc(&mism, sizeof(unsigned long long)) != hipSuccess) {
    (void)hipGetLastError();
    cleanup();
    return fail(KB_ENOMEM, "autotune could not allocate %llu bytes", 2ull * bytes);
  }
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    cleanup();
    return fail(KB_EHIP, "hipEventCreate failed");
  }
  b.out = ref;
  rc = dispatch(b, KB_MODE_PLAIN, nullptr, stream);
  if (rc) {
    cleanup();
    return rc;
  }
  const int steps_c[] = {1, 2, 4, 8, 16, 32};
  const int waves_c[] = {1, 2, 0};  // 0 = occupancy maximum
  double best_t = -1.0;
  int nrej = 0;
  for (int sp : steps_c)
    for (int wv : waves_c) {
      kb_tile t{};
      t.steps_per_item = sp;
      t.waves_per_simd = wv;
      b.out = cand;
      // parity gate: the candidate's digests must equal the plain form's
      if (hipMemsetAsync(cand, 0xA5, bytes, stream) != hipSuccess ||
          hipMemsetAsync(mism, 0, sizeof(unsigned long long), stream) != hipSuccess) {
        cleanup();
        return fail(KB_EHIP, "hipMemsetAsync failed");
      }
      rc = dispatch(b, KB_MODE_PERSISTENT, &t, stream);
      if (rc) {
        cleanup();
        return rc;
      }
      hipLaunchKernelGGL(k_compare, dim3(1024), dim3(kBlock), 0, stream,
                         reinterpret_cast<const uint32_t*>(ref), reinterpret_cast<const uint32_t*>(cand),
                         bytes / 4, mism);
      unsigned long long bad = 0;
      if (hipMemcpyAsync(&bad, mism, sizeof bad, hipMemcpyDeviceToHost, stream) != hipSuccess ||
          hipStreamSynchronize(stream) != hipSuccess) {
        cleanup();
        return fail(KB_EHIP, "autotune parity check failed to run");
      }
      if (bad) {
        ++nrej;
        continue;
      }
      std::vector<double> ts;
      for (int r = 0; r < reps; ++r) {
        (void)hipEventRecord(e0, stream);
        rc = dispatch(b, KB_MODE_PERSISTENT, &t, stream);
        (void)hipEventRecord(e1, stream);
        if (rc || hipEventSynchronize(e1) != hipSuccess) {
          cleanup();
          return rc ? rc : fail(KB_EHIP, "autotune timing failed");
        }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        ts.push_back(ms);
      }
      const double tm = median(ts);
      if (best_t < 0.0 || tm < best_t) {
        best_t = tm;
        *best = t;
      }
    }
  cleanup();
  *rejected = nrej;
  if (best_t < 0.0) return fail(KB_EHIP, "every autotune candidate failed its parity check");
  *best_ms = best_t;
  return KB_OK;
}

int keccak_graph_create(int variant, const uint8_t* d_variants, const uint8_t* d_data,
                        const uint64_t* d_offsets, const uint64_t* d_lengths, uint64_t n,
                        uint8_t* d_digests, int mode, const kb_tile* tile, hipStream_t stream,
                        kb_graph** out) {
  g_err.clear();
  if (!out) return fail(KB_EINVAL, "NULL output pointer");
  if (variant != -1 && (variant < 0 || variant > 3))
    return fail(KB_EINVAL, "variant %d is neither -1 (mixed) nor a SHA-3 variant", variant);
  if (mode == KB_MODE_PER_BUCKET)
    return fail(KB_EINVAL, "the per-bucket mode waits on the host and cannot be captured");
  const int v = variant == -1 ? kMixed : variant;
  Batch b{v, d_variants, d_data, d_offsets, d_lengths, n, d_digests, out_stride(v)};
  int rc = check_batch(b, mode);
  if (rc) return rc;
  kb_graph* g = new kb_graph();
  if (n && mode == KB_MODE_PERSISTENT) {
    // everything the capture needs is allocated and looked up first
    int dev = 0, cus = 0;
    rc = hipGetDevice(&dev) == hipSuccess ? cu_count(dev, &cus) : fail(KB_EHIP, "hipGetDevice failed");
    if (!rc) rc = size_ws(g->ws, n, 0, stream);
    if (rc) {
      free_ws(g->ws);
      delete g;
      return rc;
    }
  }
  return capture(stream, [&](hipStream_t cs) { return n ? dispatch(b, mode, tile, cs, &g->ws) : KB_OK; },
                 g, out);
}

int keccak_graph_create_merkle(int variant, const uint8_t* d_data, uint64_t total_len,
                               uint64_t leaf_size, uint8_t* d_root, hipStream_t stream,
                               kb_graph** out) {
  g_err.clear();
  if (!out) return fail(KB_EINVAL, "NULL output pointer");
  if (variant < 0 || variant > 3) return fail(KB_EINVAL, "variant %d is not a SHA-3 variant", variant);
  if (leaf_size == 0) return fail(KB_EINVAL, "leaf_size must be positive");
  if (!d_root || (total_len && !d_data)) return fail(KB_EINVAL, "NULL pointer");
  const uint64_t leaves = total_len ? (total_len + leaf_size - 1) / leaf_size : 1;
  kb_graph* g = new kb_graph();
  const int rc = size_ws(g->ws, 0, tree_workspace_bytes(leaves, kb::digest_bytes_of(variant)), stream);
  if (rc) {
    free_ws(g->ws);
    delete g;
    return rc;
  }
  return capture(stream, [&](hipStream_t cs) {
        switch (variant) {
          case 0: return merkle_impl<0>(d_data, total_len, leaf_size, d_root, cs, &g->ws);
          case 1: return merkle_impl<1>(d_data, total_len, leaf_size, d_root, cs, &g->ws);
          case 2: return merkle_impl<2>(d_data, total_len, leaf_size, d_root, cs, &g->ws);
          default: return merkle_impl<3>(d_data, total_len, leaf_size, d_root, cs, &g->ws);
        }
      }, g, out);
}

int keccak_graph_launch(kb_graph* graph, hipStream_t stream) {
  g_err.clear();
  if (!graph) return fail(KB_EINVAL, "NULL graph");
  KB_HIP(hipGraphLaunch(graph->h.exec, stream));
  return KB_OK;
}

int keccak_graph_destroy(kb_graph* graph) {
  g_err.clear();
  if (!graph) return KB_OK;
  if (graph->h.exec) (void)hipGraphExecDestroy(graph->h.exec);
  if (graph->h.graph) (void)hipGraphDestroy(graph->h.graph);
  free_ws(graph->ws);
  delete graph;
  return KB_OK;
}

uint64_t keccak_tree_workspace_bytes(int variant, uint64_t n_leaves) {
  if (variant < 0 || variant > 3) return 0;
  return tree_workspace_bytes(n_leaves, kb::digest_bytes_of(variant));
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
  const uint64_t tree = max_leaves ? tree_workspace_bytes(max_leaves, 64) : 0ull;
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
