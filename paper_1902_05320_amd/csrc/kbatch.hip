// libkbatch: batch SHA-3 on gfx950 -- kernels, scheduler and the C ABI.
//
// keccak_batch (persistent form) is four launches on the caller's stream,
// with no host synchronisation:
//   k_first   one 64-message chunk of arrival order per wave: a chunk of
//             one-block messages is hashed on the spot; any other chunk is
//             deferred (its block-count keys nb = floor(L/R) + 1 counted,
//             bins 1..4094 exact and 4095 = "4095 or more", its index
//             listed).
//   k_second<.., 0> (plan)  one workgroup: bucket starts in descending nb,
//             longest first; queue items of about `steps_per_item`
//             permutations per lane; the range of the longest messages that
//             the wide split form hashes.
//   k_second<.., 1> (tiles)  the grid fills the queue and scatters the
//             deferred messages into bucketed order.
//   k_second<.., 2> (hashing)  a resident grid: each SIMD's front wave takes
//             the split range and then the longest items at raised
//             priority, the other waves the shortest ones.
// Kernel boundaries order each launch's writes before the next one's reads,
// so no workgroup waits on another or fences.  On a batch with nothing
// deferred the last three find no work and return.
// The plain form is one k_plain launch in arrival order; the per-bucket form
// runs both passes without hashing, reads the bucket sizes back, and
// launches k_plain once per non-empty bucket.
//
// Tree mode: k_tree hashes 256 leaves per workgroup and reduces them one
// level; further k_tree launches reduce 256 nodes per workgroup up to eight
// levels while more than 1024 remain; one 512-thread workgroup reduces the
// rest to the root.  Every level is written to its own region, so no
// workgroup reads a node another one may overwrite.
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

#include "kb_internal.h"
#include "kbatch.h"
#include "sponge_device.h"
#include "split_device.h"
#include "pair_device.h"
#include "wide_device.h"

using kb::kMixed;
using kb::kShake128;
using kb::kShake256;
using kb::Lane;
using kb::SpongeShape;

namespace {

constexpr int kBlock = 256;         // threads per workgroup of the hashing kernels
constexpr int kTreeTop = 1024;      // nodes the workgroup that reduces a tree's last levels takes
constexpr int kTreeTopThreads = 512;  // its threads: two nodes (one pair) each at its first level
constexpr uint32_t kKeyBins = 4096;  // block-count buckets (4095 = "4095 or more")
constexpr uint32_t kScatterChunks = 64;  // deferred 64-message chunks per scatter tile
constexpr uint32_t kLine = 64;       // 32-bit words per 256-byte line

// Control words (uint32 indices into the ctl area), written by the plan.
enum : int {
  CTL_NITEMS = 0,       // queue items of the second pass
  CTL_TILES = 1,        // its tiles: item tiles, then scatter tiles
  CTL_ITEM_TILES = 2,
  CTL_NDEF_CHUNKS = 3,  // chunks the first pass deferred
  CTL_MAXKEY = 4,       // largest block-count key deferred
  CTL_PRIO_KEY = 5,     // front waves raise their priority on items of at least this many blocks
  CTL_SPLIT_N = 6,      // bucketed order positions [0, CTL_SPLIT_N) are hashed in the wide split form
  CTL_USEFUL = 8,       // uint64 (words 8, 9): block counts of the deferred messages
  CTL_DPREFIX = 16,     // words 16..24: exclusive prefix of the deferred sub-list lengths
  CTL_WORDS = 64
};

// Counters of the second pass, one 256-byte line each.
enum : uint32_t {
  SY_CLAIM = 1,       // tiles claimed (line 0 is spare)
  kSyncCounters = 4
};

// One flag per SIMD of the chip, indexed from the wave's hardware id
// (XCC, shader engine, shader array, CU, SIMD); the first wave to claim its
// SIMD's flag takes queue items from the front.
constexpr uint32_t kSimdSlots = 8 * 8 * 2 * 16 * 4;

// The queue is dealt round-robin into kQueues sub-queues (item t goes to
// sub-queue t mod kQueues, so each keeps the longest-first order); a wave
// starts on the sub-queue of its XCD.  Each sub-queue is one uint64 counter
// (items taken from the front | taken from the back << 32) on its own line.
constexpr uint32_t kQueues = 8;
// the sub-queues, then the counter of split items on a line of its own
constexpr uint32_t kQueueAreaDw = (kQueues + 1) * kLine;

// The first pass accumulates into kCopies partial histograms and deferred
// chunk lists, so that the deferring waves' atomics spread over eight
// addresses; the plan folds the histograms and clears the copies it found
// dirty (a non-empty list).  Copy = (workgroup index / kListRun) mod 8: runs
// of consecutive workgroups share a copy, so each list (read end to end by
// the scatter) holds long stretches of neighbouring chunks and a scatter
// tile gathers messages from a few megabytes of the batch, not from all of
// it (measured on the 2^20-message uneven batch: 2.35 against 2.36 ms, and
// the resident workgroups still spread over all eight copies).
constexpr uint32_t kCopies = 8;
constexpr uint32_t kListRun = 64;

// Workspace metadata layout (uint32 words).  Every counter and partial sum
// is zero between calls: the workspace is cleared when it is allocated, and
// each call's plan clears what the call used.
enum : uint32_t {
  M_HIST = 0,                                   // kCopies x kKeyBins partial histograms
  M_FOLD = M_HIST + kCopies * kKeyBins,         // deferred messages per key
  M_START = M_FOLD + kKeyBins,                  // first bucketed position of each key
  M_CURSOR = M_START + kKeyBins,                // scatter cursors
  M_IEND = M_CURSOR + kKeyBins,                 // inclusive prefix of queue items by rank
  M_CTL = M_IEND + kKeyBins,
  M_QUEUES = M_CTL + CTL_WORDS,
  M_SYNC = M_QUEUES + kQueueAreaDw,
  M_DEFCNT = M_SYNC + kSyncCounters * kLine,    // kCopies deferred sub-list lengths, a line each
  M_SIMD = M_DEFCNT + kCopies * kLine,
  kMetaWords = M_SIMD + kSimdSlots
};

struct WorkItem {
  uint32_t begin, end;  // positions in order[]
  uint32_t key;         // block-count bucket of the item
  uint32_t pad;
};

// Arguments of the two passes of the persistent form (by value).
struct PassArgs {
  const uint8_t* data;
  const uint64_t* offs;
  const uint64_t* lens;
  const uint8_t* vars;
  uint64_t n;
  uint8_t* out;
  uint64_t stride;      // output bytes per message
  uint32_t* meta;       // kMetaWords words, layout above
  uint32_t* deferred;   // deferred chunk indices: kCopies sub-lists of defer_seg entries
  uint32_t* order;      // bucketed order of the deferred messages, n entries
  WorkItem* items;      // queue items, max_items(n) entries
  uint32_t steps;       // permutations per lane in one queue item
  uint32_t split_cap;   // most messages the split tail may take (SHA-3 variants)
  // Per block-count class c, packed so that no array is indexed at run time
  // (an indexed member would move the whole argument block to scratch):
  uint64_t class_steps;    // byte c: steps per queue item (0 = `steps`)
  uint32_t class_threads;  // nibble c: 0 = the rule, 1 = one lane, 2 = the wide split tail
  uint64_t lanes;       // resident lanes of the second pass
  uint32_t defer_seg;   // entries of each deferred sub-list (defer_seg_of(n))
  int hash;             // 0: count and scatter only (the per-bucket form)
  const uint32_t* n_dev;  // if set: the message count, read on the device (at most n)
};

// The message count a pass works on: n, or the device word when given.
__device__ __forceinline__ uint64_t pass_count(const PassArgs& a) {
  if (!a.n_dev) return a.n;
  const uint64_t c = *a.n_dev;
  return c < a.n ? c : a.n;
}

template <int V>
__device__ __forceinline__ int rate_of(int var) {
  return V == kMixed ? kb::rate_bytes_rt(var) : SpongeShape<V>::kMaxRate;
}

// Output bytes per message of a SHA-3 form: the digest, or the mixed form's
// 64-byte slot.
template <int V>
__host__ __device__ constexpr uint32_t out_stride_of() {
  static_assert(V <= kMixed, "SHA-3 variants and the mixed form");
  if constexpr (V == kMixed)
    return 64u;
  else
    return static_cast<uint32_t>(kb::digest_bytes_of(V));
}

template <int V>
__device__ __forceinline__ uint64_t blocks_of(uint64_t len, int var) {
  if (V == kMixed && var > 3) return 1;  // no work: the slot is zeroed
  return len / static_cast<uint64_t>(rate_of<V>(var)) + 1u;
}

// Slot of key k in a partial histogram: the 16 keys of a 64-byte group are
// 256 words apart, so the most frequent small keys do not share a line.
__device__ __forceinline__ uint32_t hist_slot(uint32_t k) { return (k & 15u) * (kKeyBins / 16u) + (k >> 4); }

__device__ __forceinline__ uint32_t key_of(uint64_t nb) {
  return nb >= kKeyBins - 1 ? kKeyBins - 1 : static_cast<uint32_t>(nb);
}

// Hash message i (`len` bytes at data + off, variant `var` in the mixed
// form) into its output slot of `stride` bytes (the digest size, 64 in the
// mixed form, the output length for the XOFs).
template <int V, bool PF = kb::kPrefetch<V>>
__device__ __forceinline__ void hash_one(const uint8_t* __restrict__ data, uint64_t off,
                                         uint64_t len, int var, uint64_t i,
                                         uint8_t* __restrict__ out, uint64_t stride, uint32_t* row) {
  uint8_t* o = out + i * stride;
  if constexpr (V >= kShake128) {
    Lane A[25];
    kb::sponge_hash<V, PF>(A, data + off, len, var, row);
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
  kb::sponge_hash<V, PF>(A, data + off, len, var, row);
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

// The wide form (one state word per lane, 32 lanes per state): absorb one
// message into `a` (this lane's word), the next block's word loaded before
// the current block's permutation.
template <int V>
__device__ __forceinline__ void wide_absorb(Lane& a, const uint8_t* msg, uint64_t len, int var,
                                            const kb::wide::WideLane& L) {
  namespace wd = kb::wide;
  using S = SpongeShape<V>;
  a = Lane{0u, 0u};
  const int R = rate_of<V>(var);
  const uint32_t sh = static_cast<uint32_t>(reinterpret_cast<uintptr_t>(msg) & 3u);
  const uint64_t nb = len / static_cast<uint64_t>(R) + 1u;
  wd::WordDw d;
  wd::load_word(d, msg, sh, len, 0, R, L);
  for (uint64_t b = 0; b < nb; ++b) {
    const uint64_t boff = b * static_cast<uint64_t>(R);
    const bool fin = b + 1 == nb;
    wd::absorb_word(a, d, sh, R, fin, fin ? static_cast<uint32_t>(len - boff) : 0u, S::kPadByte, L);
    if (!fin) wd::load_word(d, msg, sh, len, boff + R, R, L);
    wd::wide_permute(a, L);
  }
}

// XOF squeeze in the wide form (Section 3.2): each lane writes its word when
// it lies in the rate, r bits of output per permutation, until out_len bytes
// are out.  Bytes are stored one by one unless out_len is a multiple of 4
// and `out` is 4-byte aligned.
template <int V>
__device__ __forceinline__ void wide_xof(Lane& a, uint8_t* out, uint64_t out_len,
                                         const kb::wide::WideLane& L) {
  constexpr uint32_t R = SpongeShape<V>::kMaxRate;
  const bool words = (out_len & 3u) == 0 && (reinterpret_cast<uintptr_t>(out) & 3u) == 0;
  for (uint64_t done = 0;;) {
    if (8u * L.word < R) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const uint32_t v = h ? a.hi : a.lo;
        const uint64_t at = done + 8u * L.word + 4u * h;
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
    done += R;
    if (done >= out_len) break;
    kb::wide::wide_permute(a, L);
  }
}

// Wide form: each half of a wave hashes one message at a time, message
// order[first + p] (or first + p) for p = state, state + states, ...  One
// wave per workgroup, as in the five-lane form.
constexpr int kWideBlock = 64;
constexpr int kWideStates = kWideBlock / kb::wide::kHalfLanes;

template <int V>
__global__ __launch_bounds__(kWideBlock) void k_wide(const uint8_t* __restrict__ data,
                                                     const uint64_t* __restrict__ offs,
                                                     const uint64_t* __restrict__ lens,
                                                     const uint8_t* __restrict__ vars,
                                                     const uint32_t* __restrict__ order,
                                                     uint64_t first, uint64_t count,
                                                     uint8_t* __restrict__ out, uint64_t stride) {
  namespace wd = kb::wide;
  __shared__ __align__(16) uint64_t lds[kWideStates * wd::kAreaSlots];
  const uint32_t s = threadIdx.x / wd::kHalfLanes, h = threadIdx.x % wd::kHalfLanes;
  wd::WideLane L;
  wd::setup(L, h, lds + s * wd::kAreaSlots);
  const uint64_t states = static_cast<uint64_t>(gridDim.x) * kWideStates;
  const int slot_dw = V == kMixed ? 16 : V >= kShake128 ? 0 : kb::digest_bytes_of(V) / 4;
  for (uint64_t p = static_cast<uint64_t>(blockIdx.x) * kWideStates + s; p < count; p += states) {
    const uint64_t i = order ? order[first + p] : first + p;
    Lane a;
    if constexpr (V >= kShake128) {
      wide_absorb<V>(a, data + offs[i], lens[i], V, L);
      wide_xof<V>(a, out + i * stride, stride, L);
      continue;
    }
    const int var = V == kMixed ? vars[i] : V;
    uint32_t* o = reinterpret_cast<uint32_t*>(out + i * stride);
    if (V == kMixed && var > 3) {  // no such variant: the slot is zeroed
      wd::store_word(o, Lane{0u, 0u}, 0, slot_dw, L);
      continue;
    }
    wide_absorb<V>(a, data + offs[i], lens[i], var, L);
    const int dw = V == kMixed ? kb::digest_bytes_rt(var) / 4 : kb::digest_bytes_of(V) / 4;
    wd::store_word(o, a, dw, slot_dw, L);
  }
}

// The pair form (two lanes per state, each holding one 32-bit half of every
// state word): absorb one message, the next block's halves loaded before the
// current block's permutation.
template <int V>
__device__ __forceinline__ void pair_absorb(uint32_t (&a)[25], const uint8_t* msg, uint64_t len,
                                            int var, uint32_t h, uint32_t hi) {
  namespace pr = kb::pair;
  using S = SpongeShape<V>;
#pragma unroll
  for (int i = 0; i < 25; ++i) a[i] = 0u;
  const int R = rate_of<V>(var);
  const uint32_t sh = static_cast<uint32_t>(reinterpret_cast<uintptr_t>(msg) & 3u);
  const uint64_t nb = len / static_cast<uint64_t>(R) + 1u;
  pr::HalfDw<V> d;
  pr::load_halves<V>(d, msg, sh, len, 0, R, h);
  for (uint64_t b = 0; b < nb; ++b) {
    const uint64_t boff = b * static_cast<uint64_t>(R);
    const bool fin = b + 1 == nb;
    pr::absorb_halves<V>(a, d, sh, R, fin, fin ? static_cast<uint32_t>(len - boff) : 0u, S::kPadByte, h);
    if (!fin) pr::load_halves<V>(d, msg, sh, len, boff + R, R, h);
    pr::pair_permute(a, hi);
  }
}

// XOF squeeze in the pair form: each lane writes its halves of the words in
// the rate, r bits per permutation, until out_len bytes are out.
template <int V>
__device__ __forceinline__ void pair_xof(uint32_t (&a)[25], uint8_t* out, uint64_t out_len,
                                         uint32_t h, uint32_t hi) {
  constexpr uint32_t R = SpongeShape<V>::kMaxRate;
  const bool words = (out_len & 3u) == 0 && (reinterpret_cast<uintptr_t>(out) & 3u) == 0;
  for (uint64_t done = 0;;) {
#pragma unroll
    for (int i = 0; i < static_cast<int>(R / 8); ++i) {
      const uint64_t at = done + 8u * i + 4u * h;
      if (at < out_len) {
        if (words) {
          *reinterpret_cast<uint32_t*>(out + at) = a[i];
        } else {
          for (uint32_t q = 0; q < 4u && at + q < out_len; ++q)
            out[at + q] = static_cast<uint8_t>(a[i] >> (8u * q));
        }
      }
    }
    done += R;
    if (done >= out_len) break;
    kb::pair::pair_permute(a, hi);
  }
}

// Pair form: each pair of lanes hashes one message at a time, message
// order[first + p] (or first + p) for p = state, state + states, ...  One
// wave per workgroup, as in the other lane-split forms.
constexpr int kPairBlock = 64;
constexpr int kPairStates = kPairBlock / kb::pair::kPairLanes;

template <int V>
__global__ __launch_bounds__(kPairBlock) void k_pair(const uint8_t* __restrict__ data,
                                                     const uint64_t* __restrict__ offs,
                                                     const uint64_t* __restrict__ lens,
                                                     const uint8_t* __restrict__ vars,
                                                     const uint32_t* __restrict__ order,
                                                     uint64_t first, uint64_t count,
                                                     uint8_t* __restrict__ out, uint64_t stride) {
  namespace pr = kb::pair;
  const uint32_t st = threadIdx.x / pr::kPairLanes, h = threadIdx.x % pr::kPairLanes;
  const uint32_t hi = h ? ~0u : 0u;
  const uint64_t states = static_cast<uint64_t>(gridDim.x) * kPairStates;
  const int slot_dw = V == kMixed ? 16 : V >= kShake128 ? 0 : kb::digest_bytes_of(V) / 4;
  for (uint64_t p = static_cast<uint64_t>(blockIdx.x) * kPairStates + st; p < count; p += states) {
    const uint64_t i = order ? order[first + p] : first + p;
    uint32_t a[25];
    if constexpr (V >= kShake128) {
      pair_absorb<V>(a, data + offs[i], lens[i], V, h, hi);
      pair_xof<V>(a, out + i * stride, stride, h, hi);
      continue;
    }
    const int var = V == kMixed ? vars[i] : V;
    uint32_t* o = reinterpret_cast<uint32_t*>(out + i * stride);
    if (V == kMixed && var > 3) {  // no such variant: the slot is zeroed
#pragma unroll
      for (int k = 0; k < 25; ++k) a[k] = 0u;
      pr::store_halves(o, a, 0, slot_dw, h);
      continue;
    }
    pair_absorb<V>(a, data + offs[i], lens[i], var, h, hi);
    const int dw = V == kMixed ? kb::digest_bytes_rt(var) / 4 : kb::digest_bytes_of(V) / 4;
    pr::store_halves(o, a, dw, slot_dw, h);
  }
}

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
// permutation), and the levels of at most one pair per half-wave in the wide
// form (one state word per lane, about three times as fast).  The exchange
// areas reuse the staging rows, which no level uses after the first split
// one.
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
template <int V, int T, bool PF, bool W8, int NODES = T, bool WL = false>
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
  constexpr int kWideStatesT = T / kb::wide::kHalfLanes;
  static_assert(2 * kWideStatesT * kb::wide::kAreaSlots <= (kStageDw > kSplitDw ? kStageDw : kSplitDw),
                "the wide exchange areas fit in the kernel's LDS");
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
    if (WL && span <= static_cast<uint64_t>(kWideStatesT)) {
      // one pair per half-wave in the wide form (one state word per lane)
      namespace wd = kb::wide;
      const uint32_t st = threadIdx.x / wd::kHalfLanes, h = threadIdx.x % wd::kHalfLanes;
      const uint64_t j = w * span + st;
      if (st < span && j < lv.m[l + 1]) {
        const uint8_t* src = nodes + lv.off[l] + 2 * j * D;
        uint32_t* d32 = reinterpret_cast<uint32_t*>(dst_of(l + 1, j));
        if (2 * j + 1 < lv.m[l]) {
          wd::WideLane L;
          wd::setup(L, h, reinterpret_cast<uint64_t*>(lds) + st * wd::kAreaSlots);
          Lane a;
          wide_absorb<V>(a, src, 2 * D, V, L);
          wd::store_word(d32, a, static_cast<int>(D / 4), static_cast<int>(D / 4), L);
        } else {
          const uint32_t* s32 = reinterpret_cast<const uint32_t*>(src);
          for (uint32_t q = h; q < D / 4; q += wd::kHalfLanes) d32[q] = s32[q];
        }
      }
    } else if (!kSplitLevels || span > static_cast<uint64_t>(kGroups)) {
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
// Persistent form: two passes
// ---------------------------------------------------------------------------
//
// k_first   one 64-message chunk of arrival order per wave.  A chunk whose
//           messages are all one block long is hashed at once: no lane
//           idles and no ordering could shorten it.  Any other chunk is
//           deferred: its messages' block-count keys are counted and its
//           index is appended to the deferred list.  The launch has no
//           inter-workgroup synchronisation at all (the end of the kernel
//           publishes the counts), so on a batch of one-block messages it
//           costs what the one-thread-per-message launch costs.
// k_second  a resident grid.  The first workgroup to arrive makes the plan
//           for the deferred messages (bucket starts longest first, queue
//           items, the split range) while the others wait for it; then the
//           workgroups take tiles (queue items, and the counting-sort scatter
//           of the deferred messages into bucketed order), wait until every
//           tile is done, and hash: waves pop queue items (longest first)
//           until the queue is drained.
//
// A batch of equal one-block messages is thus hashed in the first launch
// with no sort; the second finds an empty plan and exits.

__device__ __forceinline__ uint32_t load_relaxed(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int V>
__device__ __forceinline__ uint32_t key_at(const uint64_t* __restrict__ lens,
                                           const uint8_t* __restrict__ vars, uint64_t i) {
  return key_of(blocks_of<V>(lens[i], V == kMixed ? vars[i] : V));
}

// One chunk's metadata in a lane, as the first pass needs it: the length
// saturates at 2^32 - 1 (a one-block message is shorter than a rate, and any
// length from 2^32 on has a block count past the last key), and the variant
// is a register only in the mixed form.  Lanes past the batch load message
// 0's (every lane issues the same loads); whether a lane holds a message
// follows from the chunk index.
struct ChunkMeta {
  uint64_t off;
  uint32_t len;
  int var;
};

__device__ __forceinline__ bool lane_valid(const PassArgs& a, uint64_t c, uint32_t lane) {
  return c * 64u + lane < a.n;
}

template <int V>
__device__ __forceinline__ void load_meta(ChunkMeta& m, const PassArgs& a, uint64_t c,
                                          uint32_t lane) {
  const uint64_t i = c * 64u + lane;
  const uint64_t j = i < a.n ? i : 0u;
  m.off = a.offs[j];
  const uint64_t len = a.lens[j];
  m.len = len >> 32 ? 0xFFFFFFFFu : static_cast<uint32_t>(len);
  m.var = V == kMixed ? a.vars[j] : V;
}

// Every valid lane's message is one block long (wave-uniform).
template <int V>
__device__ __forceinline__ bool one_block_chunk(const ChunkMeta& m, bool valid) {
  return __builtin_amdgcn_ballot_w64(valid && m.len >= static_cast<uint32_t>(rate_of<V>(m.var))) == 0;
}

// The first D bytes of the squeezed state, zero past the digest in the
// mixed form's 64-byte slots and all zero for a variant out of range.
template <int V>
__device__ __forceinline__ void take_digest(uint32_t (&dig)[SpongeShape<V>::kMaxDigestDw],
                                            const Lane (&A)[25], int var) {
  using S = SpongeShape<V>;
  const int DW = V == kMixed ? (var > 3 ? 0 : kb::digest_bytes_rt(var) / 4) : S::kMaxDigestDw;
#pragma unroll
  for (int k = 0; k < S::kMaxDigestDw; ++k) {
    const uint32_t v = (k & 1) ? A[k >> 1].hi : A[k >> 1].lo;
    dig[k] = k < DW ? v : 0u;
  }
}

template <int V>
__device__ __forceinline__ void put_digest(uint8_t* out, const uint32_t (&dig)[SpongeShape<V>::kMaxDigestDw]) {
  uint32_t* o = reinterpret_cast<uint32_t*>(out);
#pragma unroll
  for (int k = 0; k < SpongeShape<V>::kMaxDigestDw; ++k) o[k] = dig[k];
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

// Block-count class of a bucket: floor(log2(key)), capped at the last class.
__device__ __forceinline__ uint32_t class_of_key(uint32_t key) {
  const uint32_t c = 31u - __builtin_clz(key ? key : 1u);
  return c < KB_NB_CLASSES - 1u ? c : KB_NB_CLASSES - 1u;
}

// Steps per queue item for a bucket: its class's tuned value, else the default.
__device__ __forceinline__ uint32_t steps_of(const PassArgs& a, uint32_t key) {
  const uint32_t s = static_cast<uint32_t>(a.class_steps >> (8u * class_of_key(key))) & 0xFFu;
  return s ? s : a.steps;
}

// Bucket rank r = kKeyBins - 1 - key orders buckets longest first; in the
// plan, thread t owns ranks 16t .. 16t + 15.
constexpr uint32_t kRanksPerThread = kKeyBins / kBlock;

// The first CTL_SPLIT_N positions of the bucketed order (the longest
// messages) go to the split form: the messages of at least
// max(kSplitMinKey, 2 x the blocks per resident lane) blocks, at most
// `split_cap` of them (twice that when every deferred message qualifies).
// Below the second bound the batch's throughput, not
// its longest chain, sets the time, and a split item (two messages per wave)
// costs throughput.  (An earlier bound of 4 x the mean block count kept a
// batch of a few equal long messages out of the split form: 8 x 64 KiB ran
// at 11.0 us per block of the chain, now 3.8.)
constexpr uint32_t kSplitMinKey = 32;
// Wide split items per SIMD's front wave.  Two measured against one
// (interleaved A/B): serving stream p50 5.23-5.25 against 5.17 ms, p99
// 7.87-7.95 against 7.70-7.78 ms; 4096 x 16 KiB 8.6 against 14.2 us per
// block of the chain; the uneven batch level.  One keeps the serving tail.
constexpr uint32_t kSplitItemsPerSimd = 1;

// The plan, made by one workgroup of the second pass once the first pass
// has finished.  Folds the partial histograms, writes the bucket
// starts (longest first), the split range, the inclusive prefix of queue
// items per rank and the tile counts, and clears every counter and partial
// this call used, so the next call starts from zero.
__device__ void make_plan(const PassArgs& a, uint32_t* scratch) {
  uint32_t* const meta = a.meta;
  uint32_t* const ctl = meta + M_CTL;
  uint32_t* const sync = meta + M_SYNC;
  __shared__ uint32_t s_split, s_ndef, s_maxkey;
  __shared__ unsigned long long s_useful;
  const uint32_t t = threadIdx.x;
  // The deferred sub-lists' lengths (read into a scalar register: the branch
  // on their sum below must be uniform in the compiler's view, since
  // barriers follow it); a copy is dirty if its sub-list is not empty.
  uint32_t ndef_chunks = 0, dirty = 0;
  for (uint32_t x = 0; x < kCopies; ++x) {
    if (t == 0) ctl[CTL_DPREFIX + x] = ndef_chunks;
    const uint32_t nx = load_relaxed(meta + M_DEFCNT + x * kLine);
    dirty |= nx ? 1u << x : 0u;
    ndef_chunks += nx;
  }
  ndef_chunks = __builtin_amdgcn_readfirstlane(ndef_chunks);
  dirty = __builtin_amdgcn_readfirstlane(dirty);
  if (t == 0) {
    s_useful = 0ull;
    s_maxkey = 0u;
  }
  __syncthreads();  // every thread has read the counters
  if (t < kCopies) meta[M_DEFCNT + t * kLine] = 0u;
  if (t == 0) {
    ctl[CTL_DPREFIX + kCopies] = ndef_chunks;
    sync[SY_CLAIM * kLine] = 0u;
    ctl[CTL_NDEF_CHUNKS] = ndef_chunks;
  }
  if (ndef_chunks == 0) {  // every chunk was hashed by the first pass
    if (t == 0) {
      ctl[CTL_NITEMS] = ctl[CTL_TILES] = ctl[CTL_ITEM_TILES] = ctl[CTL_SPLIT_N] = 0u;
      ctl[CTL_PRIO_KEY] = 0xFFFFFFFFu;
      ctl[CTL_MAXKEY] = ctl[CTL_USEFUL] = ctl[CTL_USEFUL + 1] = 0u;
    }
    return;
  }
  // Fold the dirty copies for this thread's 16 consecutive keys lo .. lo + 15
  // (slots g, g + 256, ..., g = lo / 16: for each i the workgroup's loads
  // are contiguous) and clear them.
  static_assert(kRanksPerThread == 16, "a key group of 16 per thread");
  const uint32_t lo = kKeyBins - kRanksPerThread * (t + 1u);
  const uint32_t g = lo >> 4;
  uint32_t byk[kRanksPerThread];  // folded count of key lo + i
#pragma unroll
  for (uint32_t i = 0; i < kRanksPerThread; ++i) byk[i] = 0u;
  for (uint32_t k = 0; k < kCopies; ++k) {
    if (!((dirty >> k) & 1u)) continue;
    uint32_t* h = meta + M_HIST + k * kKeyBins + g;
    uint32_t v[kRanksPerThread];
#pragma unroll
    for (uint32_t i = 0; i < kRanksPerThread; ++i) v[i] = h[i * (kKeyBins / 16u)];
#pragma unroll
    for (uint32_t i = 0; i < kRanksPerThread; ++i) {
      byk[i] += v[i];
      h[i * (kKeyBins / 16u)] = 0u;
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v)
    reinterpret_cast<uint4*>(meta + M_FOLD + lo)[v] =
        make_uint4(byk[4 * v], byk[4 * v + 1], byk[4 * v + 2], byk[4 * v + 3]);
  uint32_t cnt[kRanksPerThread], st[kRanksPerThread], c_sum = 0, kmax = 0;
  uint64_t ublocks = 0;  // blocks of this thread's buckets (a key of 4095 counts 4095)
#pragma unroll
  for (uint32_t q = 0; q < kRanksPerThread; ++q) {
    const uint32_t key = kKeyBins - 1u - (kRanksPerThread * t + q);  // = lo + 15 - q
    cnt[q] = key ? byk[kRanksPerThread - 1u - q] : 0u;
    c_sum += cnt[q];
    ublocks += static_cast<uint64_t>(key) * cnt[q];
    if (cnt[q] && key > kmax) kmax = key;
  }
  if (ublocks) atomicAdd(&s_useful, static_cast<unsigned long long>(ublocks));
  if (kmax) atomicMax(&s_maxkey, kmax);
  const uint32_t c_incl = block_inclusive_scan(c_sum, scratch);  // (its barriers order the above)
  uint32_t c_base = c_incl - c_sum;
  if (t == kBlock - 1) s_ndef = c_incl;
  __syncthreads();
  const uint32_t ndef = __builtin_amdgcn_readfirstlane(s_ndef);  // deferred messages
  const uint64_t useful = s_useful;                              // their blocks
  if (t == 0) {
    ctl[CTL_MAXKEY] = s_maxkey;
    ctl[CTL_USEFUL] = static_cast<uint32_t>(useful);
    ctl[CTL_USEFUL + 1] = static_cast<uint32_t>(useful >> 32);
  }
  const uint64_t avg = useful / (ndef ? ndef : 1u);
  // bucket starts; the split range ends where the keys drop below kmin
  const uint64_t per_lane = 2u * useful / (a.lanes ? a.lanes : 1u);
  uint64_t kmin64 = kSplitMinKey;
  if (per_lane > kmin64) kmin64 = per_lane;
  const uint32_t kmin = kmin64 < kKeyBins - 1u ? static_cast<uint32_t>(kmin64) : kKeyBins - 1u;
  if (t == 0) s_split = ndef;  // until a bucket that stays one lane per message
#pragma unroll
  for (uint32_t q = 0; q < kRanksPerThread; ++q) {
    const uint32_t key = kKeyBins - 1u - (kRanksPerThread * t + q);
    st[q] = c_base;
    meta[M_START + key] = c_base;
    c_base += cnt[q];
  }
  __syncthreads();
  // A bucket goes to the split form if its class's tile says the wide split
  // tail, or (no choice given) by the rule key >= kmin.  The split range
  // is the longest-first prefix of such buckets: it ends at the start of the
  // first non-empty bucket that stays one lane per message.
#pragma unroll
  for (uint32_t q = 0; q < kRanksPerThread; ++q) {
    const uint32_t key = kKeyBins - 1u - (kRanksPerThread * t + q);
    const uint32_t ct = (a.class_threads >> (4u * class_of_key(key))) & 0xFu;
    const bool split_here = ct == 2u || (ct == 0u && key >= kmin);
    if (cnt[q] && !split_here) atomicMin(&s_split, st[q]);
  }
  __syncthreads();
  const uint32_t split_all = __builtin_amdgcn_readfirstlane(s_split);
  // When every deferred message is a split candidate and there are at most
  // twice the cap, the front waves take them all in two rounds: the excess
  // would otherwise run one lane per message, a chain at about a third of
  // the wide form's speed.
  const uint32_t cap =
      split_all == ndef && ndef <= 2u * a.split_cap ? 2u * a.split_cap : a.split_cap;
  const uint32_t split = split_all < cap ? split_all : cap;
  // queue items over the positions past the split range
  uint32_t items[kRanksPerThread], it_sum = 0;
#pragma unroll
  for (uint32_t q = 0; q < kRanksPerThread; ++q) {
    const uint32_t key = kKeyBins - 1u - (kRanksPerThread * t + q);
    const uint32_t b = st[q] > split ? st[q] : split, e = st[q] + cnt[q];
    const uint32_t per = item_msgs(key, steps_of(a, key));
    items[q] = e > b ? (e - b + per - 1u) / per : 0u;
    it_sum += items[q];
  }
  uint32_t it_run = block_inclusive_scan(it_sum, scratch) - it_sum;
#pragma unroll
  for (uint32_t q = 0; q < kRanksPerThread; ++q) {
    it_run += items[q];
    meta[M_IEND + kRanksPerThread * t + q] = it_run;
  }
  // the second pass's scatter cursors, queues and SIMD flags start at zero
  for (uint32_t k = t; k < kKeyBins / 4; k += kBlock)
    reinterpret_cast<uint4*>(meta + M_CURSOR)[k] = make_uint4(0u, 0u, 0u, 0u);
  for (uint32_t k = t; k < kQueueAreaDw / 4; k += kBlock)
    reinterpret_cast<uint4*>(meta + M_QUEUES)[k] = make_uint4(0u, 0u, 0u, 0u);
  for (uint32_t k = t; k < kSimdSlots / 4; k += kBlock)
    reinterpret_cast<uint4*>(meta + M_SIMD)[k] = make_uint4(0u, 0u, 0u, 0u);
  if (t == kBlock - 1) {
    const uint32_t item_tiles = (it_run + kBlock - 1) / kBlock;
    ctl[CTL_NITEMS] = it_run;
    ctl[CTL_SPLIT_N] = split;
    ctl[CTL_PRIO_KEY] = static_cast<uint32_t>(2u * avg + 2u);
    ctl[CTL_ITEM_TILES] = item_tiles;
    ctl[CTL_TILES] = item_tiles + (ndef_chunks + kScatterChunks - 1) / kScatterChunks;
  }
}

// Waves per SIMD the first pass is compiled for: three for the fixed
// variants and the mixed form (the permutation, the staging and a chunk's
// metadata fit in 168 VGPRs); SHAKE128's 168-byte rate needs more LDS, so it
// holds two.
template <int V>
constexpr int kFirstWaves = V == kShake128 ? 2 : 3;

// Deferral bookkeeping, by the deferring wave alone.  With no barrier, a
// launch whose chunks are all hashed runs like the one-thread-per-message
// launch (the two workgroup barriers an LDS histogram needs made the
// uniform batch 23 % slower, measured).  The wave counts its keys into
// the partial histogram of its copy with one atomic per distinct key
// (lanes of equal keys found by ballot) and appends its chunk to its copy's
// deferred sub-list.  The plan derives the block sums from the histogram,
// so no per-wave sums contend for one line.
// Out of line, so that the hashing path stays one straight run of code
// right after the metadata loads: with this code inlined between them the
// uniform batch ran 20 % slower although the permutation's code was byte
// for byte the same (measured twice, with the blocks in either order).
// (Arguments by value: a reference to the argument block would move it to
// scratch.)
constexpr uint32_t kDeferDirectKey = 16;

template <int V>
__device__ __attribute__((noinline)) void defer_chunk(uint32_t* meta, uint32_t* deferred, uint32_t seg,
                                                    uint32_t len, int var, uint64_t c, bool valid,
                                                    uint32_t lane) {
  // the histogram copy and the list copy are the same: the plan folds (and
  // clears) exactly the histogram copies whose lists are not empty
  const uint32_t x = (blockIdx.x / kListRun) % kCopies;
  uint32_t* const hist = meta + M_HIST + x * kKeyBins;
  const uint32_t key = valid ? key_of(blocks_of<V>(len, var)) : 0u;
  // the first valid lane's key is merged across the wave (a chunk of equal
  // lengths takes one atomic: with one atomic per lane, 32768 messages of
  // 4 KiB queued on one histogram slot and the first pass took 188 us);
  // other keys above kDeferDirectKey are rare and mostly distinct within a
  // chunk: one atomic per lane, all issued at once; the frequent small keys
  // are merged across the wave first, one atomic per distinct key
  const uint64_t vm = __builtin_amdgcn_ballot_w64(valid);
  const uint32_t lead = vm ? static_cast<uint32_t>(__builtin_ctzll(vm)) : 0u;
  const uint32_t k0 = __builtin_amdgcn_readlane(key, lead);
  const uint64_t same0 = __builtin_amdgcn_ballot_w64(valid && key == k0);
  if (vm && lane == lead) atomicAdd(&hist[hist_slot(k0)], static_cast<uint32_t>(__builtin_popcountll(same0)));
  const bool rest = valid && key != k0;
  const bool direct = rest && key > kDeferDirectKey;
  if (direct) atomicAdd(&hist[hist_slot(key)], 1u);
  uint64_t todo = __builtin_amdgcn_ballot_w64(rest && !direct);
  while (todo) {  // wave-uniform: one pass per distinct key
    const uint32_t leader = static_cast<uint32_t>(__builtin_ctzll(todo));
    const uint32_t k = __builtin_amdgcn_readlane(key, leader);
    const uint64_t same = __builtin_amdgcn_ballot_w64(rest && !direct && key == k) & todo;
    if (lane == leader) atomicAdd(&hist[hist_slot(k)], static_cast<uint32_t>(__builtin_popcountll(same)));
    todo &= ~same;
  }
  if (lane == 0) {
    const uint32_t slot = atomicAdd(&meta[M_DEFCNT + x * kLine], 1u);
    deferred[static_cast<uint64_t>(x) * seg + slot] = static_cast<uint32_t>(c);
  }
}

// First pass (see above), grid = ceil(n / 256): wave w of workgroup g takes
// chunk 4g + w.  a.hash == 0 defers every chunk (the per-bucket form hashes
// nothing here).
template <int V>
__global__ __launch_bounds__(kBlock, kFirstWaves<V>) void k_first(PassArgs a) {
  using S = SpongeShape<V>;
  a.n = pass_count(a);
  // the staging rows only: 40 KiB for the 136- and 144-byte rates, so four
  // workgroups fit on a CU
  __shared__ __align__(16) uint32_t lds[kBlock * S::kRowDw];
  const uint32_t lane = threadIdx.x & 63u;
  const uint64_t nch = (a.n + 63u) / 64u;
  // (the wave index through readfirstlane: the compiler then sees the chunk
  // and every decision on it as wave-uniform, and branches on scalars)
  const uint64_t c = static_cast<uint64_t>(blockIdx.x) * (kBlock / 64) +
                     __builtin_amdgcn_readfirstlane(threadIdx.x / 64u);
  const bool in = c < nch;
  ChunkMeta m;
  load_meta<V>(m, a, in ? c : 0u, lane);
  const bool valid = in && lane_valid(a, c, lane);
  const bool h = in && a.hash && one_block_chunk<V>(m, valid);  // wave-uniform
  const bool d = in && !h;
  kb::BlockChunks<V> bc;
  if (h) kb::load_block<V>(bc, a.data + m.off, valid ? m.len : 0u);
  if (!h) {
    if (d) defer_chunk<V>(a.meta, a.deferred, a.defer_seg, m.len, m.var, c, valid, lane);
    return;
  }
  // stage the block, absorb it into the zero state, permute, squeeze
  uint32_t* const row = lds + threadIdx.x * S::kRowDw;
  Lane A[25];
  uint32_t w[S::kMaxRateDw];
  kb::stage_block<V>(row, bc, valid ? m.len : 0u, rate_of<V>(m.var), true, w);
  const int RW = rate_of<V>(m.var) / 4;
#pragma unroll
  for (int k = 0; k < 50; ++k) {
    const uint32_t v = (k < S::kMaxRateDw && k < RW) ? w[k < S::kMaxRateDw ? k : 0] : 0u;
    if (k & 1)
      A[k >> 1].hi = v;
    else
      A[k >> 1].lo = v;
  }
  kb::keccak_rounds_0_22(A);
  kb::keccak_round(A, 23);
  if constexpr (V >= kShake128) {
    if (valid) kb::squeeze_xof<V>(A, a.out + (c * 64u + lane) * a.stride, a.stride);
  } else {
    uint32_t dig[S::kMaxDigestDw];
    take_digest<V>(dig, A, m.var);
    if (valid) put_digest<V>(a.out + (c * 64u + lane) * a.stride, dig);
  }
}

// Queue item q of the second pass: its bucket (the smallest rank r with
// iend[r] > q) and its range of positions in the bucketed order.
__device__ __forceinline__ void items_tile(const PassArgs& a, uint32_t tile) {
  const uint32_t* meta = a.meta;
  const uint32_t* ctl = meta + M_CTL;
  const uint32_t q = tile * kBlock + threadIdx.x;
  if (q >= ctl[CTL_NITEMS]) return;
  const uint32_t* iend = meta + M_IEND;
  uint32_t lo = 0, hi = kKeyBins - 1;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (iend[mid] > q)
      hi = mid;
    else
      lo = mid + 1;
  }
  const uint32_t key = kKeyBins - 1u - lo;
  const uint32_t per = item_msgs(key, steps_of(a, key));
  const uint32_t first_item = lo ? iend[lo - 1] : 0u;
  const uint32_t split = ctl[CTL_SPLIT_N];  // positions before it are split work
  const uint32_t start = meta[M_START + key];
  const uint32_t b = (start > split ? start : split) + (q - first_item) * per;
  const uint32_t bucket_end = start + meta[M_FOLD + key];
  a.items[q] = WorkItem{b, b + per < bucket_end ? b + per : bucket_end, key, 0u};
}

// Counting-sort scatter of kScatterChunks deferred chunks: one global
// atomic per non-empty bucket reserves the tile's range, LDS atomics rank
// the messages inside it.
template <int V>
__device__ __forceinline__ void scatter_tile(const PassArgs& a, uint32_t tile, uint32_t* lcount,
                                             uint32_t* lbase) {
  constexpr uint32_t kPer = kScatterChunks * 64u / kBlock;  // messages per thread
  const uint32_t nchunks = a.meta[M_CTL + CTL_NDEF_CHUNKS];
  for (uint32_t k = threadIdx.x; k < kKeyBins; k += kBlock) lcount[k] = 0u;
  __syncthreads();
  const uint32_t first = tile * kScatterChunks;
  uint32_t keys[kPer];
  uint64_t msg[kPer];
#pragma unroll
  for (uint32_t q = 0; q < kPer; ++q) {
    const uint32_t slot = (q * kBlock + threadIdx.x) / 64u, lane = threadIdx.x & 63u;
    msg[q] = ~0ull;
    keys[q] = 0u;
    if (first + slot < nchunks) {
      const uint32_t j = first + slot;  // in the sub-lists end to end
      uint32_t x = 0;
#pragma unroll
      for (uint32_t y = 1; y < kCopies; ++y) x = j >= a.meta[M_CTL + CTL_DPREFIX + y] ? y : x;
      const uint32_t e = j - a.meta[M_CTL + CTL_DPREFIX + x];
      const uint64_t i = static_cast<uint64_t>(a.deferred[static_cast<uint64_t>(x) * a.defer_seg + e]) * 64u + lane;
      if (i < a.n) {
        msg[q] = i;
        keys[q] = key_at<V>(a.lens, a.vars, i);
        atomicAdd(&lcount[keys[q]], 1u);
      }
    }
  }
  __syncthreads();
  for (uint32_t k = threadIdx.x; k < kKeyBins; k += kBlock) {
    const uint32_t c = lcount[k];
    lbase[k] = c ? a.meta[M_START + k] + atomicAdd(&a.meta[M_CURSOR + k], c) : 0u;
    lcount[k] = 0u;
  }
  __syncthreads();
#pragma unroll
  for (uint32_t q = 0; q < kPer; ++q)
    if (msg[q] != ~0ull) {
      const uint32_t rank = atomicAdd(&lcount[keys[q]], 1u);
      a.order[lbase[keys[q]] + rank] = static_cast<uint32_t>(msg[q]);
    }
  __syncthreads();  // the LDS arrays are reused by the next tile
}

// Second pass (see above), as three launches of one template: PH = 0 makes
// the plan, PH = 1 fills the queue and the bucketed order, PH = 2 hashes.
// Kernel boundaries order the plan before the tiles and the tiles before
// the hashing.  (Earlier forms did the plan and the tiles in the hashing
// launch's workgroups, the others spinning on a published word and then
// fencing: on the uneven 2^20 batch the plan and tiles took 84 us of it,
// the acquire fences of hundreds of workgroups each invalidating an L2.)
// On each SIMD one wave (the first to claim the SIMD's flag) takes items
// from the front at raised issue priority while they are long, so the long
// absorb chains that bound the makespan run back to back at full rate; the
// other resident waves take the shortest items from the back and fill the
// issue slots the front wave leaves idle.  Both
// ends of a sub-queue advance one packed 64-bit counter, so no item is taken
// twice.  A wave drains the sub-queue of its own XCD first and then the
// others in turn, so every item is taken whatever the mapping of waves to
// XCDs, and every wave leaves once all sub-queues are empty.
template <int V, bool PF, int PH>
__global__ __launch_bounds__(kBlock) void k_second(PassArgs a) {
  using S = SpongeShape<V>;
  a.n = pass_count(a);
  constexpr uint32_t kStageDw = kBlock * S::kRowDw;
  constexpr uint32_t kLdsDw = kStageDw > 2 * kKeyBins ? kStageDw : 2 * kKeyBins;
  __shared__ __align__(16) uint32_t lds[kLdsDw];
  __shared__ uint32_t s_tile;
  static_assert(2 * kWideStates * kb::wide::kAreaSlots <= 64 * S::kRowDw,
                "a wave's staging rows hold its wide exchange areas");
  const uint32_t* ctl = a.meta + M_CTL;
  uint32_t* const sync = a.meta + M_SYNC;
  if constexpr (PH == 0) {
    make_plan(a, lds);  // one workgroup
    return;
  } else if constexpr (PH == 1) {
    // Tiles are claimed one at a time from a counter.  One thread claims;
    // the loop condition is a scalar read after a barrier, so the loop (with
    // the barriers in it) is uniform as the compiler sees it.
    const uint32_t tiles = __builtin_amdgcn_readfirstlane(ctl[CTL_TILES]);
    if (!tiles) return;  // the first pass hashed everything
    const uint32_t item_tiles = ctl[CTL_ITEM_TILES];
    if (threadIdx.x == 0) s_tile = atomicAdd(&sync[SY_CLAIM * kLine], 1u);
    __syncthreads();
    uint32_t tile = __builtin_amdgcn_readfirstlane(s_tile);
    while (tile < tiles) {
      __syncthreads();  // every thread has read s_tile
      if (tile < item_tiles)
        items_tile(a, tile);
      else
        scatter_tile<V>(a, tile - item_tiles, lds, lds + kKeyBins);
      __syncthreads();
      if (threadIdx.x == 0) s_tile = atomicAdd(&sync[SY_CLAIM * kLine], 1u);
      __syncthreads();
      tile = __builtin_amdgcn_readfirstlane(s_tile);
    }
    return;
  } else {
    if (!__builtin_amdgcn_readfirstlane(ctl[CTL_TILES])) return;  // the first pass hashed everything
    uint32_t* row = lds + threadIdx.x * S::kRowDw;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t n_items = ctl[CTL_NITEMS];
    const uint32_t prio_key = ctl[CTL_PRIO_KEY];
    unsigned long long* const queues = reinterpret_cast<unsigned long long*>(a.meta + M_QUEUES);
    uint32_t claim = 0;
    if (lane == 0) claim = atomicCAS(&a.meta[M_SIMD + simd_slot()], 0u, 1u) == 0u ? 1u : 0u;
    const bool front = __builtin_amdgcn_readfirstlane(__shfl(claim, 0)) != 0u;
    const unsigned long long step = 1ull << (front ? 0 : 32);
    const uint32_t home = __builtin_amdgcn_s_getreg((3 << 11) | 20) & (kQueues - 1u);
    // Split items first: the front waves hash the longest messages (bucketed
    // positions [0, split_n)) two at a time, one per half-wave, in the wide
    // lane-split form (one state word per lane), whose chain of permutations
    // runs about three times as fast as one thread's.  The exchange areas are
    // this wave's own staging rows.  The XOFs squeeze in the same form.
    const uint32_t split_n = ctl[CTL_SPLIT_N];
    // With no split tail and no more queue items than SIMDs, the front waves
    // (one per SIMD) take every item: a second wave on a SIMD would share its
    // issue slots and stretch both items' chains while other SIMDs idle.  The
    // mixed-variant kernel keeps every wave claiming: in it this test alone
    // moved the hashing code and cost the uneven batch a tenth.
    if constexpr (V != kMixed)
      if (!front && split_n == 0u && n_items <= a.split_cap / (kSplitItemsPerSimd * kWideStates)) return;
    {
      if (front && split_n) {
        namespace wd = kb::wide;
        uint64_t* area = reinterpret_cast<uint64_t*>(lds + (threadIdx.x & ~63u) * S::kRowDw);
        const uint32_t half = lane / wd::kHalfLanes;
        wd::WideLane L;
        wd::setup(L, lane % wd::kHalfLanes, area + half * wd::kAreaSlots);
        const int slot_dw = V >= kShake128 ? 0 : static_cast<int>(out_stride_of<V <= kMixed ? V : 1>() / 4u);
        uint32_t* split_ctr = reinterpret_cast<uint32_t*>(queues + kQueues * (kLine / 2));
        __builtin_amdgcn_s_setprio(3);
        for (;;) {
          uint32_t d = 0;
          if (lane == 0)
            d = __hip_atomic_fetch_add(split_ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          d = __builtin_amdgcn_readfirstlane(__shfl(d, 0));
          if (d >= (split_n + kWideStates - 1u) / kWideStates) break;
          const uint32_t pos = d * kWideStates + half;
          if (pos < split_n) {
            const uint32_t i = a.order[pos];
            const int var = V == kMixed ? a.vars[i] : V;
            uint32_t* o = reinterpret_cast<uint32_t*>(a.out + static_cast<uint64_t>(i) * a.stride);
            if constexpr (V >= kShake128) {
              Lane w;
              wide_absorb<V>(w, a.data + a.offs[i], a.lens[i], V, L);
              wide_xof<V>(w, a.out + static_cast<uint64_t>(i) * a.stride, a.stride, L);
            } else if (V == kMixed && var > 3) {
              wd::store_word(o, Lane{0u, 0u}, 0, slot_dw, L);
            } else {
              Lane w;
              wide_absorb<V>(w, a.data + a.offs[i], a.lens[i], var, L);
              const int dw = V == kMixed ? kb::digest_bytes_rt(var) / 4 : kb::digest_bytes_of(V) / 4;
              wd::store_word(o, w, dw, slot_dw, L);
            }
          }
        }
        __builtin_amdgcn_s_setprio(0);
      }
    }
    uint32_t qi = 0;  // sub-queues tried so far
    for (;;) {
      // choose the next item; the hashing below appears once in the kernel
      uint32_t t = 0xFFFFFFFFu;
      while (qi < kQueues) {
        const uint32_t x = (home + qi) & (kQueues - 1u);
        const uint32_t m = n_items > x ? (n_items - x + kQueues - 1u) / kQueues : 0u;
        unsigned long long old = 0;
        if (lane == 0)
          old = __hip_atomic_fetch_add(queues + x * (kLine / 2), step, __ATOMIC_RELAXED,
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
      if (t == 0xFFFFFFFFu) break;
      const WorkItem it = a.items[t];
      if (front && it.key >= prio_key)
        __builtin_amdgcn_s_setprio(3);
      else
        __builtin_amdgcn_s_setprio(0);
      // the next message's index and metadata are loaded while this one hashes
      uint32_t pos = it.begin + lane;
      uint64_t i = 0, off = 0, len = 0;
      int var = V;
      if (pos < it.end) {
        i = a.order[pos];
        off = a.offs[i];
        len = a.lens[i];
        if constexpr (V == kMixed) var = a.vars[i];
      }
      while (pos < it.end) {
        const uint32_t pn = pos + 64u;
        uint64_t in = 0, offn = 0, lenn = 0;
        int varn = V;
        if (pn < it.end) {
          in = a.order[pn];
          offn = a.offs[in];
          lenn = a.lens[in];
          if constexpr (V == kMixed) varn = a.vars[in];
        }
        hash_one<V, PF>(a.data, off, len, var, i, a.out, a.stride, row);
        pos = pn;
        i = in;
        off = offn;
        len = lenn;
        var = varn;
      }
    }
    __builtin_amdgcn_s_setprio(0);
  }
}

__global__ void k_reset(uint32_t* __restrict__ meta, uint32_t words) {
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < words; k += gridDim.x * blockDim.x)
    meta[k] = 0u;
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
  uint32_t* meta = nullptr;      // kMetaWords words (layout above), cleared at allocation
  uint32_t* order = nullptr;     // bucketed order
  uint64_t order_cap = 0;
  WorkItem* items = nullptr;     // queue items
  uint64_t items_cap = 0;
  uint32_t* deferred = nullptr;  // deferred chunk list
  uint64_t deferred_cap = 0;
  uint8_t* tree = nullptr;       // tree node buffer
  uint64_t tree_cap = 0;
  uint32_t* host_fold = nullptr;  // pinned: bucket sizes and starts, for the per-bucket form
};

// Measurement hook state (keccak_timing_*): event pairs around kernel
// launches, each tagged with the kind of kernel it brackets.
struct Timing {
  uint32_t kinds = 0;  // bit k set: launches of kernel kind k are bracketed
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
  std::vector<int> kind;
  size_t used = 0;
};
std::mutex g_tmu;
Timing g_timing;

// Brackets one kernel launch with events when timing is enabled.
struct TimedLaunch {
  hipEvent_t stop = nullptr;
  hipStream_t s;
  TimedLaunch(hipStream_t st, int kind) : s(st) {
    std::lock_guard<std::mutex> lk(g_tmu);
    if (kind < 0 || kind > 31 || !((g_timing.kinds >> kind) & 1u)) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
    if (g_timing.used == g_timing.pool.size()) {
      std::pair<hipEvent_t, hipEvent_t> e{nullptr, nullptr};
      if (hipEventCreate(&e.first) != hipSuccess || hipEventCreate(&e.second) != hipSuccess) {
        (void)hipGetLastError();
        return;
      }
      g_timing.pool.push_back(e);
      g_timing.kind.push_back(kind);
    }
    g_timing.kind[g_timing.used] = kind;
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

// Deferred chunks are listed per partial copy (copy = (first-pass workgroup
// index / kListRun) mod kCopies): of the ceil(ceil(n / 256) / kListRun) runs
// of workgroups, copy x takes at most ceil(runs / 8), each of at most
// kListRun workgroups of 4 chunks, which bounds the length of each sub-list.
constexpr uint64_t defer_seg_of(uint64_t n) {
  const uint64_t runs = ((n + kBlock - 1) / kBlock + kListRun - 1) / kListRun;
  return 4u * kListRun * ((runs + kCopies - 1) / kCopies);
}

// Queue items of a batch of n messages: at most ceil(n / 64) whole ones and
// one partial item per bucket.
uint64_t max_items(uint64_t n) { return n / 64 + kKeyBins + 1; }

// Clear a freshly allocated metadata area with a kernel on the stream (not
// a memset: the call may be recorded into a graph).
int clear_meta(uint32_t* meta, hipStream_t s) {
  hipLaunchKernelGGL(k_reset, dim3(64), dim3(256), 0, s, meta, static_cast<uint32_t>(kMetaWords));
  KB_HIP(hipGetLastError());
  return KB_OK;
}

// Size the batch part of a workspace for `msgs` messages.
int grow_batch(Workspace& w, uint64_t msgs, hipStream_t stream) {
  int rc = grow(reinterpret_cast<void**>(&w.order), &w.order_cap, msgs * 4ull, stream);
  if (!rc)
    rc = grow(reinterpret_cast<void**>(&w.items), &w.items_cap, max_items(msgs) * sizeof(WorkItem),
              stream);
  if (!rc) rc = grow(reinterpret_cast<void**>(&w.deferred), &w.deferred_cap, kCopies * defer_seg_of(msgs) * 4ull, stream);
  return rc;
}

int get_ws(hipStream_t stream, uint64_t msgs, uint64_t tree_bytes, Workspace** out) {
  int dev = 0;
  KB_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_mu);
  Workspace& w = g_ws[std::make_pair(dev, stream)];
  if (!w.meta) {
    uint64_t cap = 0;
    int rc = grow(reinterpret_cast<void**>(&w.meta), &cap, kMetaWords * 4ull, stream);
    if (!rc) rc = clear_meta(w.meta, stream);
    if (rc) return rc;
  }
  if (msgs) {
    int rc = grow_batch(w, msgs, stream);
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
    TimedLaunch tl(s, KB_KERNEL_PLAIN);
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
    TimedLaunch tl(s, KB_KERNEL_SPLIT);
    hipLaunchKernelGGL(k_split<V>, dim3(static_cast<uint32_t>(grid)), dim3(kSplitBlock), 0, s,
                       b.data, b.offs, b.lens, b.vars, order, first, count, b.out, b.stride);
  }
  KB_HIP(hipGetLastError());
  return KB_OK;
}

template <int V>
int launch_wide(const Batch& b, const uint32_t* order, uint64_t first, uint64_t count,
                hipStream_t s) {
  if (!count) return KB_OK;
  int dev = 0, cus = 0;
  KB_HIP(hipGetDevice(&dev));
  int rc = cu_count(dev, &cus);
  if (rc) return rc;
  // one state per message up to 16 waves per CU; beyond that states loop
  uint64_t grid = (count + kWideStates - 1) / kWideStates;
  if (grid > static_cast<uint64_t>(16 * cus)) grid = 16 * cus;
  {
    TimedLaunch tl(s, KB_KERNEL_WIDE);
    hipLaunchKernelGGL(k_wide<V>, dim3(static_cast<uint32_t>(grid)), dim3(kWideBlock), 0, s,
                       b.data, b.offs, b.lens, b.vars, order, first, count, b.out, b.stride);
  }
  KB_HIP(hipGetLastError());
  return KB_OK;
}

template <int V>
int launch_pair(const Batch& b, const uint32_t* order, uint64_t first, uint64_t count,
                hipStream_t s) {
  if (!count) return KB_OK;
  int dev = 0, cus = 0;
  KB_HIP(hipGetDevice(&dev));
  int rc = cu_count(dev, &cus);
  if (rc) return rc;
  // one state per message up to 16 waves per CU; beyond that states loop
  uint64_t grid = (count + kPairStates - 1) / kPairStates;
  if (grid > static_cast<uint64_t>(16 * cus)) grid = 16 * cus;
  {
    TimedLaunch tl(s, KB_KERNEL_PAIR);
    hipLaunchKernelGGL(k_pair<V>, dim3(static_cast<uint32_t>(grid)), dim3(kPairBlock), 0, s,
                       b.data, b.offs, b.lens, b.vars, order, first, count, b.out, b.stride);
  }
  KB_HIP(hipGetLastError());
  return KB_OK;
}

// Workgroups of `kernel` that fit on the chip at once, capped by the tile's
// waves per SIMD (a 256-thread workgroup is one wave on each of a CU's four
// SIMDs).
// The occupancy query is cached per (device, kernel): it does not change,
// and asked on every call it was a large part of a small batch's host time.
std::map<std::pair<int, const void*>, int> g_occupancy;

int resident_grid(const void* kernel, const kb_tile* tile, int cus, uint32_t* grid) {
  int dev = 0, per_cu = 0;
  KB_HIP(hipGetDevice(&dev));
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_occupancy.find({dev, kernel});
    if (it != g_occupancy.end()) per_cu = it->second;
  }
  if (per_cu == 0) {
    KB_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, 0));
    if (per_cu < 1) per_cu = 1;
    std::lock_guard<std::mutex> lk(g_mu);
    g_occupancy[{dev, kernel}] = per_cu;
  }
  if (tile && tile->waves_per_simd > 0 && tile->waves_per_simd < per_cu) per_cu = tile->waves_per_simd;
  *grid = static_cast<uint32_t>(per_cu * cus);
  return KB_OK;
}

// The second pass for a tile's staging form: blocks loaded when absorbed
// (KB_STAGING_DIRECT, SHA-3 variants) or the next block prefetched into
// registers while the current one is permuted.
template <int V>
const void* second_pass_kernel(const kb_tile* tile) {
  if constexpr (V <= kMixed) {
    if (tile && tile->staging == KB_STAGING_DIRECT) return reinterpret_cast<const void*>(&k_second<V, false, 2>);
  }
  return reinterpret_cast<const void*>(&k_second<V, true, 2>);
}

// The persistent form (two passes) or, with mode KB_MODE_PER_BUCKET, the
// same passes without hashing followed by one plain launch per bucket, the
// bucket sizes read back on the host.
template <int V>
int run_two_pass(const Batch& b, Workspace& w, int mode, const kb_tile* tile, hipStream_t s,
                 const uint32_t* n_dev) {
  const bool per_bucket = mode == KB_MODE_PER_BUCKET;
  int dev = 0, cus = 0;
  KB_HIP(hipGetDevice(&dev));
  int rc = cu_count(dev, &cus);
  if (rc) return rc;
  uint32_t grid1 = 0, grid2 = 0;
  // first pass: one 64-message chunk per wave
  const uint64_t g1 = (b.n + kBlock - 1) / kBlock;
  if (g1 > 0x7FFFFFFFull) return fail(KB_EINVAL, "batch too large for one launch");
  grid1 = static_cast<uint32_t>(g1 ? g1 : 1);
  const void* second = second_pass_kernel<V>(tile);
  if (!rc) rc = resident_grid(second, tile, cus, &grid2);
  if (rc) return rc;
  PassArgs a{};
  a.data = b.data;
  a.offs = b.offs;
  a.lens = b.lens;
  a.vars = b.vars;
  a.n = b.n;
  a.out = b.out;
  a.stride = b.stride;
  a.meta = w.meta;
  a.deferred = w.deferred;
  a.defer_seg = static_cast<uint32_t>(defer_seg_of(b.n));
  a.order = w.order;
  a.items = w.items;
  a.steps = tile && tile->steps_per_item > 0 ? static_cast<uint32_t>(tile->steps_per_item) : 4u;
  // at most kSplitItemsPerSimd wide split items (a state per half-wave) for
  // each SIMD's front wave (the per-bucket form takes none)
  a.split_cap = !per_bucket ? kSplitItemsPerSimd * kWideStates * 4u * static_cast<uint32_t>(cus) : 0u;
  a.class_steps = 0;
  a.class_threads = 0;
  for (int c = 0; tile && c < KB_NB_CLASSES; ++c) {  // ranges checked by check_tile
    a.class_steps |= static_cast<uint64_t>(tile->class_steps[c] & 0xFF) << (8 * c);
    const int32_t tc = tile->class_threads[c];
    const uint32_t ct = tc == KB_THREADS_WIDE ? 2u : static_cast<uint32_t>(tc);
    a.class_threads |= ct << (4 * c);
  }
  a.lanes = static_cast<uint64_t>(grid2) * kBlock;
  a.hash = per_bucket ? 0 : 1;
  a.n_dev = n_dev;
  {
    TimedLaunch tl(s, KB_KERNEL_FIRST_PASS);
    hipLaunchKernelGGL(k_first<V>, dim3(grid1), dim3(kBlock), 0, s, a);
  }
  KB_HIP(hipGetLastError());
  {
    TimedLaunch tl(s, KB_KERNEL_SCHEDULE);
    hipLaunchKernelGGL((k_second<V, kb::kPrefetch<V>, 0>), dim3(1), dim3(kBlock), 0, s, a);
  }
  KB_HIP(hipGetLastError());
  {
    TimedLaunch tl(s, KB_KERNEL_SCHEDULE);
    hipLaunchKernelGGL((k_second<V, kb::kPrefetch<V>, 1>), dim3(grid2), dim3(kBlock), 0, s, a);
  }
  KB_HIP(hipGetLastError());
  if (!per_bucket) {
    TimedLaunch tl(s, KB_KERNEL_SECOND_PASS);
    void* args[] = {&a};
    KB_HIP(hipLaunchKernel(second, dim3(grid2), dim3(kBlock), args, 0, s));
  }
  KB_HIP(hipGetLastError());
  if (!per_bucket) return KB_OK;
  if (!w.host_fold)
    KB_HIP(hipHostMalloc(reinterpret_cast<void**>(&w.host_fold), 2 * kKeyBins * 4, 0));
  static_assert(M_START == M_FOLD + kKeyBins, "bucket sizes and starts are adjacent");
  KB_HIP(hipMemcpyAsync(w.host_fold, w.meta + M_FOLD, 2 * kKeyBins * 4, hipMemcpyDeviceToHost, s));
  KB_HIP(hipStreamSynchronize(s));
  for (int key = static_cast<int>(kKeyBins) - 1; key >= 1; --key) {
    const uint32_t c = w.host_fold[key];
    if (!c) continue;
    rc = launch_plain<V>(b, w.order, w.host_fold[kKeyBins + key], c, s);
    if (rc) return rc;
  }
  return KB_OK;
}

// n_dev (persistent form only): the message count is read from that device
// word when the kernels run, b.n being its upper bound.
template <int V>
int run_batch(const Batch& b, int mode, const kb_tile* tile, hipStream_t s, Workspace* own,
              const uint32_t* n_dev) {
  if (mode == KB_MODE_PLAIN) return launch_plain<V>(b, nullptr, 0, b.n, s);
  if (mode == KB_MODE_SPLIT) return launch_split<V>(b, nullptr, 0, b.n, s);
  if (mode == KB_MODE_WIDE) return launch_wide<V>(b, nullptr, 0, b.n, s);
  if (mode == KB_MODE_PAIR) return launch_pair<V>(b, nullptr, 0, b.n, s);
  if (b.n >= 0xFFFFFFFFull) return launch_plain<V>(b, nullptr, 0, b.n, s);  // 32-bit order[]
  Workspace* w = own;
  int rc = own ? KB_OK : get_ws(s, b.n, 0, &w);
  if (rc) return rc;
  return run_two_pass<V>(b, *w, mode, tile, s, n_dev);
}

// `own`: a caller-owned workspace (a captured graph's), else the stream's.
int dispatch(const Batch& b, int mode, const kb_tile* tile, hipStream_t s, Workspace* own = nullptr,
             const uint32_t* n_dev = nullptr) {
  switch (b.variant) {
    case 0: return run_batch<0>(b, mode, tile, s, own, n_dev);
    case 1: return run_batch<1>(b, mode, tile, s, own, n_dev);
    case 2: return run_batch<2>(b, mode, tile, s, own, n_dev);
    case 3: return run_batch<3>(b, mode, tile, s, own, n_dev);
    case kShake128: return run_batch<kShake128>(b, mode, tile, s, own, n_dev);
    case kShake256: return run_batch<kShake256>(b, mode, tile, s, own, n_dev);
    default: return run_batch<kMixed>(b, mode, tile, s, own, n_dev);
  }
}

int check_batch(const Batch& b, int mode) {
  if (b.variant != kMixed && b.variant != kShake128 && b.variant != kShake256 &&
      (b.variant < 0 || b.variant > 3))
    return fail(KB_EINVAL, "variant %d is not a SHA-3 variant (0..3)", b.variant);
  if (mode < KB_MODE_PERSISTENT || mode > KB_MODE_PAIR)
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

// A tile's fields must lie in their documented ranges.
int check_tile(const kb_tile* t) {
  if (!t) return KB_OK;
  if (t->block_threads != 0 && t->block_threads != kBlock)
    return fail(KB_EINVAL, "tile.block_threads must be 0 or %d", kBlock);
  if (t->waves_per_simd < 0 || t->waves_per_simd > 8)
    return fail(KB_EINVAL, "tile.waves_per_simd must be in 0..8");
  if (t->steps_per_item < 0 || t->steps_per_item > 255)
    return fail(KB_EINVAL, "tile.steps_per_item must be in 0..255");
  if (t->staging < KB_STAGING_DEFAULT || t->staging > KB_STAGING_PREFETCH)
    return fail(KB_EINVAL, "tile.staging must be a kb_staging value");
  for (int c = 0; c < KB_NB_CLASSES; ++c) {
    if (t->class_steps[c] < 0 || t->class_steps[c] > 255)
      return fail(KB_EINVAL, "tile.class_steps[%d] must be in 0..255", c);
    if (t->class_threads[c] != 0 && t->class_threads[c] != 1 && t->class_threads[c] != KB_THREADS_WIDE)
      return fail(KB_EINVAL, "tile.class_threads[%d] must be 0, 1 or %d", c, KB_THREADS_WIDE);
  }
  return KB_OK;
}

int batch_entry(int variant, const uint8_t* vars, const uint8_t* data, const uint64_t* offs,
                const uint64_t* lens, uint64_t n, uint8_t* out, int mode, const kb_tile* tile,
                hipStream_t s) {
  g_err.clear();
  if (int rc = check_tile(tile)) return rc;
  Batch b{variant, vars, data, offs, lens, n, out, out_stride(variant)};
  int rc = check_batch(b, mode);
  if (rc || n == 0) return rc;
  // With no tile given, the autotuner's cache (KBATCH_TUNE) may hold one for
  // this batch; a malformed cache file is an error, not a silent default.
  kb_tile cached;
  int from_cache = 0;
  if (!tile && mode == KB_MODE_PERSISTENT && variant <= kMixed) {
    from_cache = kb::tune_lookup(nullptr, variant == kMixed ? -1 : variant, n, &cached);
    if (from_cache < 0) return from_cache;
    if (from_cache) {
      if ((rc = check_tile(&cached))) return rc;
      tile = &cached;
    }
  }
  kb::note_tile(tile, from_cache);
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
        TimedLaunch tl(s, KB_KERNEL_TREE);
        if (first > 0)
          hipLaunchKernelGGL((k_tree<V, kBlock, kb::kPrefetch<V>, true, kBlock, true>),
                             dim3(static_cast<uint32_t>(blocks)), dim3(kBlock), 0, s, data, total,
                             leaf, w->tree, root, first, levels, L, lv);
        else if (w8)
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
        TimedLaunch tl(s, KB_KERNEL_TREE);
        hipLaunchKernelGGL((k_tree<V, kTreeTopThreads, false, true, kTreeTop, true>), dim3(1),
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
  if (w.deferred) (void)hipFree(w.deferred);
  if (w.tree) (void)hipFree(w.tree);
  if (w.host_fold) (void)hipHostFree(w.host_fold);
  w = Workspace{};
}

// Size a graph's private workspace for `msgs` messages and `tree_bytes`
// (cleared on the stream before the capture starts).
int size_ws(Workspace& w, uint64_t msgs, uint64_t tree_bytes, hipStream_t s) {
  uint64_t cap = 0;
  int rc = grow(reinterpret_cast<void**>(&w.meta), &cap, kMetaWords * 4ull, s);
  if (!rc) rc = clear_meta(w.meta, s);
  if (!rc && msgs) rc = grow_batch(w, msgs, s);
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

// The allocation-free entry point's workspace: one static array per device,
// laid out as a Workspace for at most KB_NOALLOC_MAX_MSGS messages.
namespace {
constexpr uint64_t align256(uint64_t x) { return (x + 255u) & ~uint64_t{255}; }
constexpr uint64_t kNoAllocMax = KB_NOALLOC_MAX_MSGS;
constexpr uint64_t kScratchOrderOff = align256(uint64_t{kMetaWords} * 4u);
constexpr uint64_t kScratchItemsOff = kScratchOrderOff + align256(kNoAllocMax * 4u);
constexpr uint64_t kScratchDeferredOff =
    kScratchItemsOff + align256((kNoAllocMax / 64 + kKeyBins + 1) * sizeof(WorkItem));
constexpr uint64_t kScratchBytes = kScratchDeferredOff + align256(kCopies * defer_seg_of(kNoAllocMax) * 4u);
}  // namespace

static __device__ __align__(256) uint8_t scratch[kScratchBytes];

namespace {
std::mutex g_scratch_mu;
std::map<int, uint8_t*> g_scratch;  // device -> the array's address on that device

// The static workspace of the current device.  On the first call on a
// device its address is looked up (host code must not use the array's name:
// that is a host-side stand-in) and its metadata cleared on `stream`.
int scratch_ws(hipStream_t stream, Workspace* w) {
  int dev = 0;
  KB_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch.find(dev);
  if (it == g_scratch.end()) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(KB_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    const int rc = clear_meta(static_cast<uint32_t*>(p), stream);
    if (rc) return rc;
    it = g_scratch.emplace(dev, static_cast<uint8_t*>(p)).first;
  }
  uint8_t* base = it->second;
  *w = Workspace{};
  w->meta = reinterpret_cast<uint32_t*>(base);
  w->order = reinterpret_cast<uint32_t*>(base + kScratchOrderOff);
  w->order_cap = kNoAllocMax * 4u;
  w->items = reinterpret_cast<WorkItem*>(base + kScratchItemsOff);
  w->items_cap = (kNoAllocMax / 64 + kKeyBins + 1) * sizeof(WorkItem);
  w->deferred = reinterpret_cast<uint32_t*>(base + kScratchDeferredOff);
  w->deferred_cap = kCopies * defer_seg_of(kNoAllocMax) * 4u;
  return KB_OK;
}
}  // namespace

namespace kb {
int set_last_error(int code, const char* msg) {
  g_err = msg ? msg : "";
  return code;
}
hipGraph_t native_graph(kb_graph* g) { return g ? g->h.graph : nullptr; }
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

int keccak_batch_noalloc(int variant, const uint8_t* d_data, const uint64_t* d_offsets,
                         const uint64_t* d_lengths, uint64_t n, uint8_t* d_digests,
                         hipStream_t stream) {
  g_err.clear();
  if (variant < 0 || variant > 3)
    return fail(KB_EINVAL, "variant %d is not a SHA-3 variant (0..3)", variant);
  Batch b{variant, nullptr, d_data, d_offsets, d_lengths, n, d_digests, out_stride(variant)};
  int rc = check_batch(b, KB_MODE_PERSISTENT);
  if (rc || n == 0) return rc;
  if (n > kNoAllocMax)
    return fail(KB_EINVAL, "n = %llu is more than the %llu messages the static workspace holds",
                static_cast<unsigned long long>(n), static_cast<unsigned long long>(kNoAllocMax));
  Workspace w;
  rc = scratch_ws(stream, &w);
  if (rc) return rc;
  return dispatch(b, KB_MODE_PERSISTENT, nullptr, stream, &w);
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
  if (n >= 0xFFFFFFFFull) return fail(KB_EINVAL, "the persistent form takes fewer than 2^32 messages");
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
  int nrej = 0;
  // Run one candidate: its digests must equal the plain form's bit for bit
  // (else it is rejected, < 0), then the median of `reps` timed runs.
  auto trial = [&](const kb_tile& t, double* ms) -> int {
    *ms = -1.0;
    b.out = cand;
    if (hipMemsetAsync(cand, 0xA5, bytes, stream) != hipSuccess ||
        hipMemsetAsync(mism, 0, sizeof(unsigned long long), stream) != hipSuccess)
      return fail(KB_EHIP, "hipMemsetAsync failed");
    int r = dispatch(b, KB_MODE_PERSISTENT, &t, stream);
    if (r) return r;
    hipLaunchKernelGGL(k_compare, dim3(1024), dim3(kBlock), 0, stream,
                       reinterpret_cast<const uint32_t*>(ref), reinterpret_cast<const uint32_t*>(cand),
                       bytes / 4, mism);
    unsigned long long bad = 0;
    if (hipMemcpyAsync(&bad, mism, sizeof bad, hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess)
      return fail(KB_EHIP, "autotune parity check failed to run");
    if (bad) {
      ++nrej;
      return KB_OK;
    }
    std::vector<double> ts;
    for (int k = 0; k < reps; ++k) {
      (void)hipEventRecord(e0, stream);
      r = dispatch(b, KB_MODE_PERSISTENT, &t, stream);
      (void)hipEventRecord(e1, stream);
      if (r) return r;
      if (hipEventSynchronize(e1) != hipSuccess) return fail(KB_EHIP, "autotune timing failed");
      float m = 0.f;
      (void)hipEventElapsedTime(&m, e0, e1);
      ts.push_back(m);
    }
    *ms = median(ts);
    return KB_OK;
  };
  kb_tile cur{};
  double cur_ms = -1.0;
  auto consider = [&](const kb_tile& t) -> int {
    double ms = -1.0;
    const int r = trial(t, &ms);
    if (r) return r;
    if (ms >= 0.0 && (cur_ms < 0.0 || ms < cur_ms)) {
      cur = t;
      cur_ms = ms;
    }
    return KB_OK;
  };
  // 1. launch-wide: resident waves per SIMD x staging form
  for (int wv : {0, 1, 2, 3})
    for (int st : {KB_STAGING_PREFETCH, KB_STAGING_DIRECT}) {
      kb_tile t{};
      t.waves_per_simd = wv;
      t.staging = st;
      if ((rc = consider(t))) break;
    }
  // 2. the default steps per queue item
  for (int sp : {1, 2, 8, 16, 32}) {
    if (rc) break;
    kb_tile t = cur;
    t.steps_per_item = sp;
    rc = consider(t);
  }
  if (!rc && cur_ms < 0.0) rc = fail(KB_EHIP, "every autotune candidate failed its parity check");
  // The block-count classes present among the messages the second pass
  // hashes (its bucket sizes, read back from the last run's plan).
  uint32_t present = 0;
  if (!rc) {
    Workspace* w = nullptr;
    rc = get_ws(stream, n, 0, &w);
    std::vector<uint32_t> fold(kKeyBins);
    uint32_t ndef_chunks = 0;  // the plan writes the bucket sizes only when some chunk was deferred
    if (!rc && (hipMemcpyAsync(fold.data(), w->meta + M_FOLD, kKeyBins * 4, hipMemcpyDeviceToHost,
                               stream) != hipSuccess ||
                hipMemcpyAsync(&ndef_chunks, w->meta + M_CTL + CTL_NDEF_CHUNKS, 4,
                               hipMemcpyDeviceToHost, stream) != hipSuccess ||
                hipStreamSynchronize(stream) != hipSuccess))
      rc = fail(KB_EHIP, "autotune could not read the bucket sizes");
    for (uint32_t key = 1; !rc && ndef_chunks && key < kKeyBins; ++key)
      if (fold[key]) present |= 1u << kb::nb_class_of(key);
  }
  // 3. threads per state by class: the wide split tail for the longest
  // classes (from class c up) and one lane per message below, for each c
  // present, and one lane everywhere
  if (!rc && present) {
    const kb_tile base = cur;
    for (int c = KB_NB_CLASSES; c >= 1 && !rc; --c) {  // c = KB_NB_CLASSES: no split class
      if (c < KB_NB_CLASSES && !((present >> c) & 1u)) continue;
      kb_tile t = base;
      for (int k = 0; k < KB_NB_CLASSES; ++k)
        if ((present >> k) & 1u) t.class_threads[k] = k >= c ? KB_THREADS_WIDE : 1;
      rc = consider(t);
    }
  }
  // 4. steps per queue item by class, one class at a time
  for (int c = 0; c < KB_NB_CLASSES && !rc; ++c) {
    if (!((present >> c) & 1u)) continue;
    const kb_tile base = cur;
    for (int sp : {1, 4, 16}) {
      kb_tile t = base;
      t.class_steps[c] = sp;
      if ((rc = consider(t))) break;
    }
  }
  cleanup();
  if (rc) return rc;
  *best = cur;
  *best_ms = cur_ms;
  *rejected = nrej;
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

int keccak_graph_create_counted(int variant, const uint8_t* d_variants, const uint8_t* d_data,
                                const uint64_t* d_offsets, const uint64_t* d_lengths,
                                const uint32_t* d_count, uint64_t max_n, uint8_t* d_digests,
                                hipStream_t stream, kb_graph** out) {
  g_err.clear();
  if (!out) return fail(KB_EINVAL, "NULL output pointer");
  if (variant != -1 && (variant < 0 || variant > 3))
    return fail(KB_EINVAL, "variant %d is neither -1 (mixed) nor a SHA-3 variant", variant);
  if (!d_count) return fail(KB_EINVAL, "NULL count pointer");
  if (max_n == 0 || max_n >= 0xFFFFFFFFull) return fail(KB_EINVAL, "max_n must be in [1, 2^32 - 1)");
  const int v = variant == -1 ? kMixed : variant;
  Batch b{v, d_variants, d_data, d_offsets, d_lengths, max_n, d_digests, out_stride(v)};
  int rc = check_batch(b, KB_MODE_PERSISTENT);
  if (rc) return rc;
  kb_graph* g = new kb_graph();
  int dev = 0, cus = 0;
  rc = hipGetDevice(&dev) == hipSuccess ? cu_count(dev, &cus) : fail(KB_EHIP, "hipGetDevice failed");
  if (!rc) rc = size_ws(g->ws, max_n, 0, stream);
  if (rc) {
    free_ws(g->ws);
    delete g;
    return rc;
  }
  return capture(stream,
                 [&](hipStream_t cs) { return dispatch(b, KB_MODE_PERSISTENT, nullptr, cs, &g->ws, d_count); },
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
      free_ws(w);
      (void)hipSetDevice(prev);
    } else {
      rc = KB_EHIP;
    }
  }
  g_ws.clear();
  if (rc) fail(rc, "keccak_release: a device could not be synchronised");
  return rc;
}

int keccak_timing_enable_kinds(uint32_t kinds) {
  g_err.clear();
  if (kinds >> (KB_KERNEL_PAIR + 1)) return fail(KB_EINVAL, "unknown kernel kind in mask 0x%x", kinds);
  std::lock_guard<std::mutex> lk(g_tmu);
  g_timing.kinds = kinds;
  g_timing.used = 0;
  return KB_OK;
}

int keccak_timing_enable(int on) {
  return keccak_timing_enable_kinds(on ? (2u << KB_KERNEL_PAIR) - 1u : 0u);
}

// Sum of the bracketed durations of kernels of kind `kind` (-1: every kind).
int timing_sum(int kind, double* total_ms, uint64_t* launches) {
  g_err.clear();
  if (!total_ms || !launches) return fail(KB_EINVAL, "NULL output pointer");
  std::lock_guard<std::mutex> lk(g_tmu);
  double sum = 0.0;
  uint64_t cnt = 0;
  for (size_t k = 0; k < g_timing.used; ++k) {
    if (kind >= 0 && g_timing.kind[k] != kind) continue;
    auto& e = g_timing.pool[k];
    KB_HIP(hipEventSynchronize(e.second));
    float ms = 0.f;
    KB_HIP(hipEventElapsedTime(&ms, e.first, e.second));
    sum += ms;
    ++cnt;
  }
  *total_ms = sum;
  *launches = cnt;
  return KB_OK;
}

int keccak_timing_read(double* total_ms, uint64_t* launches) {
  return timing_sum(-1, total_ms, launches);
}

int keccak_timing_read_kernel(int kind, double* total_ms, uint64_t* launches) {
  if (kind < KB_KERNEL_FIRST_PASS || kind > KB_KERNEL_PAIR) {
    g_err.clear();
    return fail(KB_EINVAL, "unknown kernel kind %d", kind);
  }
  return timing_sum(kind, total_ms, launches);
}

const char* keccak_last_error(void) { return g_err.c_str(); }

// KB_SOURCE_HASH: the build's hash of the kernel sources (first 16 hex
// digits of the SHA-256 over this directory's files, as the build computes it)
#ifndef KB_SOURCE_HASH
#define KB_SOURCE_HASH "unknown"
#endif
const char* keccak_version(void) { return "kbatch 0.1 (gfx950) src " KB_SOURCE_HASH; }

}  // extern "C"
