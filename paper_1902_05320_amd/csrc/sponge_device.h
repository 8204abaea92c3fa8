// The SHA-3 sponge (Section 3.2, eqs. 11-16) for one message per thread.
//
// Each block of the padded message P = M || 01 || pad10*1 reaches the state
// through LDS:
//   1. the 16-byte-aligned chunks that hold the block's bytes are copied from
//      HBM straight into LDS with global_load_lds_dwordx4 (no VGPRs), chunk j
//      of lane L at wave_lds[256 j + 4 L] -- the instruction's fixed layout;
//      chunk slots past the message end are zeroed with LDS stores.  A block
//      at any byte offset needs at most ceil((R + 15) / 16) chunks;
//   2. on the final block the chunk holding the message end is read back,
//      bytes past the end cleared and the suffix/pad byte 0x06 merged (bits
//      0,1 of the suffix "01", then the first pad bit), and 0x80 (the last pad
//      bit) is stored on byte R-1, or 0x86 when both fall on byte R-1 -- the
//      byte form of N || pad10*1 with j = (-m-2) mod r;
//   3. the block is read back as dwords and realigned with v_alignbyte.
// The copy for block b+1 is issued before the permutation of block b and
// completes under it, so a long message's chain of permutations does not
// wait on HBM latency between blocks.
//
// Variant `V` is 0..3 (SHA3-224/256/384/512, rate fixed at compile time) or
// kMixed (rate chosen per thread at run time).
#pragma once

#include "keccak_device.h"

namespace kb {

constexpr int kMixed = 4;

template <int V>
struct SpongeShape {
  static constexpr int kMaxRate = V == kMixed ? 144 : rate_bytes_of(V);
  static constexpr int kMaxRateDw = kMaxRate / 4;
  // 16-byte chunks that can hold R bytes starting at any offset mod 16
  static constexpr int kChunks = (kMaxRate + 15 + 15) / 16;
  // LDS dwords per wave: kChunks chunks of 64 lanes x 16 bytes
  static constexpr int kWaveDw = kChunks * 256;
  static constexpr int kMaxDigestDw = V == kMixed ? 16 : digest_bytes_of(V) / 4;
};

__device__ __forceinline__ int rate_bytes_rt(int v) { return 200 - 2 * (v == 0 ? 28 : v == 1 ? 32 : v == 2 ? 48 : 64); }
__device__ __forceinline__ int digest_bytes_rt(int v) { return v == 0 ? 28 : v == 1 ? 32 : v == 2 ? 48 : 64; }

typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) void global_void_t;

// Wait until this wave's outstanding global loads, including the copies into
// LDS, have landed.  Inline asm with a memory clobber, so that no LDS access
// is moved above it.
__device__ __forceinline__ void wait_vmem() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Wait until this wave's LDS reads have returned their data, so that a copy
// into the same LDS slots issued next cannot overtake them.
__device__ __forceinline__ void wait_lds() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

// Start the copy of one block: `p` is the block's first message byte and
// `rem` = min(bytes left, R).  Only chunks holding at least one message byte
// are read; the others are zeroed.  `wave_lds` is the wave's (uniform) LDS
// area.
template <int V>
__device__ __forceinline__ void issue_block(uint32_t* wave_lds, uint32_t lane, const uint8_t* p,
                                            uint32_t rem) {
  using S = SpongeShape<V>;
  const uint32_t s16 = static_cast<uint32_t>(reinterpret_cast<uintptr_t>(p) & 15u);
  // the aligned base comes from pointer arithmetic, so it stays a global pointer
  const uint4* base = reinterpret_cast<const uint4*>(p - s16);
  const uint32_t nv = s16 + rem;
  wait_lds();
#pragma unroll
  for (int j = 0; j < S::kChunks; ++j) {
    if (rem != 0u && 16u * j < nv)
      __builtin_amdgcn_global_load_lds((global_void_t*)(base + j),
                                       (lds_void_t*)(wave_lds + 256 * j), 16, 0, 0);
    else
      *reinterpret_cast<uint4*>(wave_lds + 256 * j + 4 * lane) = make_uint4(0u, 0u, 0u, 0u);
  }
}

// Finish a block whose copy was issued: wait for it, apply the padding on the
// final block, and return the block as little-endian dwords w[0..kMaxRateDw).
template <int V>
__device__ __forceinline__ void finish_block(uint32_t* wave_lds, uint32_t lane, uint32_t s16,
                                             uint32_t rem, int R, bool fin,
                                             uint32_t (&w)[SpongeShape<V>::kMaxRateDw]) {
  using S = SpongeShape<V>;
  wait_vmem();
  uint32_t* mine = wave_lds + 4 * lane;
  if (fin) {
    // the chunk holding byte nv (the first byte past the message)
    const uint32_t nv = s16 + rem;
    const uint32_t cut = nv & 15u;
    uint4* cp = reinterpret_cast<uint4*>(mine + 256 * (nv >> 4));
    uint4 c = *cp;
    uint32_t d[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int keep = static_cast<int>(cut) - 4 * q;  // bytes of dword q before the end
      uint32_t m = keep >= 4 ? 0xFFFFFFFFu : keep <= 0 ? 0u : (1u << (8 * keep)) - 1u;
      d[q] &= m;
      if (static_cast<uint32_t>(q) == (cut >> 2)) d[q] |= 0x06u << (8u * (cut & 3u));
    }
    *cp = make_uint4(d[0], d[1], d[2], d[3]);
    const uint32_t last = s16 + static_cast<uint32_t>(R) - 1u;
    reinterpret_cast<uint8_t*>(mine + 256 * (last >> 4))[last & 15u] =
        rem + 1u == static_cast<uint32_t>(R) ? 0x86u : 0x80u;
  }
  // dword q of the row is chunk q/4, dword q%4; message dword k is row dword
  // q0 + k with q0 = s16/4, so the reads for k = 4m + r come from four bases
  const uint32_t q0 = s16 >> 2;
  const uint32_t* a[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const uint32_t q = q0 + r;
    a[r] = mine + 256 * (q >> 2) + (q & 3u);
  }
  uint32_t u[S::kMaxRateDw + 1];
#pragma unroll
  for (int k = 0; k <= S::kMaxRateDw; ++k) u[k] = a[k & 3][256 * (k >> 2)];
  const uint32_t sh = s16 & 3u;
#pragma unroll
  for (int k = 0; k < S::kMaxRateDw; ++k) w[k] = __builtin_amdgcn_alignbyte(u[k + 1], u[k], sh);
}

// Absorb the whole message and run the permutation on every block; on return
// A holds Keccak-f[1600] of the last absorbed state, i.e. the squeezed output
// lanes (d <= r for every SHA-3 variant, so one squeeze suffices).
template <int V>
__device__ __forceinline__ void sponge_hash(Lane (&A)[25], const uint8_t* msg, uint64_t len,
                                            int var, uint32_t* wave_lds, uint32_t lane) {
  using S = SpongeShape<V>;
  const int R = V == kMixed ? rate_bytes_rt(var) : rate_bytes_of(V);
  const int RW = R / 4;
  // blocks of the padded message: the 2 suffix bits and the pad fit after
  // any byte-aligned message, so nb = floor(L / R) + 1
  const uint64_t nb = len / static_cast<uint64_t>(R) + 1u;
  const uint32_t s16 = static_cast<uint32_t>(reinterpret_cast<uintptr_t>(msg) & 15u);
  issue_block<V>(wave_lds, lane, msg, nb == 1 ? static_cast<uint32_t>(len) : static_cast<uint32_t>(R));
  for (uint64_t b = 0; b < nb; ++b) {
    const bool fin = b + 1u == nb;
    const uint64_t off = b * static_cast<uint64_t>(R);
    const uint32_t rem = fin ? static_cast<uint32_t>(len - off) : static_cast<uint32_t>(R);
    uint32_t w[S::kMaxRateDw];
    finish_block<V>(wave_lds, lane, (s16 + static_cast<uint32_t>(off)) & 15u, rem, R, fin, w);
    if (!fin) {
      // prefetch block b+1 into LDS while this block is permuted
      const uint64_t off1 = off + static_cast<uint64_t>(R);
      const uint32_t rem1 = b + 2u == nb ? static_cast<uint32_t>(len - off1) : static_cast<uint32_t>(R);
      issue_block<V>(wave_lds, lane, msg + off1, rem1);
    }
    if (b == 0) {
#pragma unroll
      for (int k = 0; k < 50; ++k) {
        const uint32_t v = (k < S::kMaxRateDw && k < RW) ? w[k < S::kMaxRateDw ? k : 0] : 0u;
        if (k & 1)
          A[k >> 1].hi = v;
        else
          A[k >> 1].lo = v;
      }
    } else {
#pragma unroll
      for (int k = 0; k < S::kMaxRateDw; ++k) {
        const uint32_t v = k < RW ? w[k] : 0u;
        if (k & 1)
          A[k >> 1].hi ^= v;
        else
          A[k >> 1].lo ^= v;
      }
    }
    keccak_rounds_0_22(A);
    if (!fin) keccak_round(A, 23);
  }
  keccak_round(A, 23);
}

// Trunc_d of the squeezed state: the first D bytes are dwords 0..D/4-1 in
// lane order (lo, hi).  `out` must be 4-byte aligned.  In the mixed form every
// slot is 64 bytes, zero past the digest.
template <int V>
__device__ __forceinline__ void store_digest(uint8_t* out, const Lane (&A)[25], int var) {
  using S = SpongeShape<V>;
  uint32_t* o = reinterpret_cast<uint32_t*>(out);
  const int DW = V == kMixed ? digest_bytes_rt(var) / 4 : digest_bytes_of(V) / 4;
#pragma unroll
  for (int k = 0; k < S::kMaxDigestDw; ++k) {
    const uint32_t v = (k & 1) ? A[k >> 1].hi : A[k >> 1].lo;
    o[k] = k < DW ? v : 0u;
  }
}

}  // namespace kb
