// The SHA-3 sponge (Section 3.2, eqs. 11-16) for one message per thread.
//
// Each block of the padded message P = M || 01 || pad10*1 is staged through a
// per-thread row of LDS before it is xored into the state:
//   1. the 16-byte-aligned chunks that hold the block's bytes are read with
//      global_load_dwordx4 (for the next block while the current one is
//      permuted) and stored to the row unchanged, so a block at any byte
//      offset costs at most ceil((R + 15) / 16) vector loads;
//   2. on the final block the bytes past the message end are cleared and the
//      suffix/padding bytes are written with byte-granular LDS stores: 0x06
//      (bits 0,1 of the suffix "01" then the first pad bit; 0x1F for the
//      SHAKE suffix "1111") at the message end, 0x80 (the last pad bit) on
//      byte R-1, or the two OR-ed when both fall on byte R-1 -- the byte form
//      of N || pad10*1 with j = (-m-2) mod r;
//   3. the row is read back as dwords and realigned with v_alignbyte.
// The data-dependent byte positions thus cost LDS address arithmetic, not
// per-dword VALU masking.
//
// Variant `V` is 0..3 (SHA3-224/256/384/512, rate fixed at compile time),
// kMixed (one of those four chosen per thread at run time), or kShake128 /
// kShake256 (the XOFs of eqs. 17-18: suffix 1111, so the byte after the
// message is 0x1F, and any output length).
#pragma once

#include "keccak_device.h"

namespace kb {

constexpr int kMixed = 4;
constexpr int kShake128 = 5;  // Keccak[256]: rate 168 bytes
constexpr int kShake256 = 6;  // Keccak[512]: rate 136 bytes

template <int V>
struct SpongeShape {
  static constexpr int kMaxRate =
      V == kMixed ? 144 : V == kShake128 ? 168 : V == kShake256 ? 136 : rate_bytes_of(V);
  static constexpr int kMaxRateDw = kMaxRate / 4;
  // 16-byte chunks that can hold R bytes starting at any offset mod 16
  static constexpr int kChunks = (kMaxRate + 15 + 15) / 16;
  // the LDS row is the chunk area; the read-back (dwords s16/4 .. s16/4 + R/4,
  // s16 < 16) stays inside it, and clearing stores past it are dropped
  static constexpr int kRowDw = kChunks * 4;
  static_assert(3 + kMaxRate / 4 < kRowDw, "read-back must stay inside the row");
  static constexpr int kMaxDigestDw = V == kMixed ? 16 : V >= kShake128 ? 0 : digest_bytes_of(V) / 4;
  // the suffix bits and the first pad bit, as the byte after the message:
  // SHA-3 "01" then 1 -> 0x06; SHAKE "1111" then 1 -> 0x1F
  static constexpr uint32_t kPadByte = V >= kShake128 ? 0x1Fu : 0x06u;
};

__device__ __forceinline__ int rate_bytes_rt(int v) { return 200 - 2 * (v == 0 ? 28 : v == 1 ? 32 : v == 2 ? 48 : 64); }
__device__ __forceinline__ int digest_bytes_rt(int v) { return v == 0 ? 28 : v == 1 ? 32 : v == 2 ? 48 : 64; }

// The 16-byte-aligned chunks holding one block's bytes: `p` points at the
// block's first message byte, `rem` = min(bytes left, R).  Only chunks
// holding at least one message byte are read; the rest are zero.
template <int V>
struct BlockChunks {
  uint4 c[SpongeShape<V>::kChunks];
  uint32_t s16;  // p mod 16
};

template <int V>
__device__ __forceinline__ void load_block(BlockChunks<V>& bc, const uint8_t* p, uint32_t rem) {
  using S = SpongeShape<V>;
  bc.s16 = static_cast<uint32_t>(reinterpret_cast<uintptr_t>(p) & 15u);
  // derive the aligned base by pointer arithmetic (not from an integer) so
  // the loads stay in the global address space
  const uint4* base = reinterpret_cast<const uint4*>(p - bc.s16);
  const uint32_t nv = bc.s16 + rem;
#pragma unroll
  for (int j = 0; j < S::kChunks; ++j) {
    bc.c[j] = make_uint4(0u, 0u, 0u, 0u);
    if (rem != 0u && 16u * j < nv) bc.c[j] = base[j];
  }
}

// Stage loaded chunks through `row`, apply the padding on the final block
// (`fin`, rem < R then) and return the block as little-endian dwords
// w[0 .. kMaxRateDw).
template <int V>
__device__ __forceinline__ void stage_block(uint32_t* __restrict__ row, const BlockChunks<V>& bc,
                                            uint32_t rem, int R, bool fin,
                                            uint32_t (&w)[SpongeShape<V>::kMaxRateDw]) {
  using S = SpongeShape<V>;
  const uint32_t s16 = bc.s16;
  const uint32_t nv = s16 + rem;  // row bytes [s16, nv) hold message bytes
  uint4* row4 = reinterpret_cast<uint4*>(row);
#pragma unroll
  for (int j = 0; j < S::kChunks; ++j) row4[j] = bc.c[j];
  if (fin) {
    // clear the tail of the last chunk: up to three whole dwords past the
    // dword holding byte nv, then bytes nv..nv+2 (suffix byte first)
    // (nv < s16 + R <= 4 kRowDw, so the suffix byte is always inside the row)
    const uint32_t d0 = (nv + 3u) >> 2;
#pragma unroll
    for (uint32_t k = 0; k < 3; ++k)
      if (d0 + k < static_cast<uint32_t>(S::kRowDw)) row[d0 + k] = 0u;
    uint8_t* rb = reinterpret_cast<uint8_t*>(row);
    rb[nv] = S::kPadByte;
    if (nv + 1u < 4u * S::kRowDw) rb[nv + 1] = 0u;
    if (nv + 2u < 4u * S::kRowDw) rb[nv + 2] = 0u;
    rb[s16 + R - 1] = rem + 1u == static_cast<uint32_t>(R) ? (S::kPadByte | 0x80u) : 0x80u;
  }
  const uint32_t* src = row + (s16 >> 2);
  const uint32_t sh = s16 & 3u;
#pragma unroll
  for (int k = 0; k < S::kMaxRateDw; ++k) w[k] = __builtin_amdgcn_alignbyte(src[k + 1], src[k], sh);
}

// Absorb the whole message and run the permutation on every block; on return
// A holds Keccak-f[1600] of the last absorbed state, i.e. the squeezed output
// lanes (d <= r for every SHA-3 variant, so one squeeze suffices).
// With prefetch on, the chunks of block b+1 are loaded into registers before
// the permutation of block b and land while it runs, so a multi-block
// message's chain of permutations does not wait for HBM between blocks.  It
// costs the registers of one block of chunks (about 40 VGPRs).  Measured by
// interleaved A/B on one box: 4 KiB Merkle leaves 1.14 ms per 1 GiB root
// with it against 1.23 without (three waves per SIMD against four); the
// mixed-variant batch of lengths up to 16 KiB 2.40 ms against 2.52, although
// the mixed kernel then holds two waves per SIMD instead of three (206 VGPRs;
// capping it at three spills); one-block messages are level either way.
// The chain of the longest message bounds a batch of uneven lengths, so the
// latency of each block matters more than the occupancy.
template <int V>
constexpr bool kPrefetch = true;

template <int V, bool PF = kPrefetch<V>>
__device__ __forceinline__ void sponge_hash(Lane (&A)[25], const uint8_t* msg, uint64_t len,
                                            int var, uint32_t* __restrict__ row) {
  using S = SpongeShape<V>;
  const int R = V == kMixed ? rate_bytes_rt(var) : S::kMaxRate;
  const int RW = R / 4;
  // blocks of the padded message: the 2 suffix bits and the pad fit after
  // any byte-aligned message, so nb = floor(L / R) + 1
  const uint64_t nb = len / static_cast<uint64_t>(R) + 1u;
  BlockChunks<V> bc;
  if (PF) load_block<V>(bc, msg, nb == 1 ? static_cast<uint32_t>(len) : static_cast<uint32_t>(R));
  for (uint64_t b = 0; b < nb; ++b) {
    const bool fin = b + 1u == nb;
    const uint64_t off = b * static_cast<uint64_t>(R);
    const uint32_t rem = fin ? static_cast<uint32_t>(len - off) : static_cast<uint32_t>(R);
    if (!PF) load_block<V>(bc, msg + off, rem);
    uint32_t w[S::kMaxRateDw];
    stage_block<V>(row, bc, rem, R, fin, w);
    if (PF && !fin) {
      const uint64_t off1 = off + static_cast<uint64_t>(R);
      load_block<V>(bc, msg + off1,
                    b + 2u == nb ? static_cast<uint32_t>(len - off1) : static_cast<uint32_t>(R));
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
    if (!fin || V >= kShake128) keccak_round(A, 23);
  }
  if (V < kShake128) keccak_round(A, 23);
}

// The sponge for a message of whole 8-byte words at an 8-byte-aligned
// address (len % 8 == 0, fixed variant).  Every block then starts 8-byte
// aligned (R is a multiple of 8), so its bytes can go from HBM straight into
// LDS with the loads that write LDS directly (no VGPRs hold them in flight)
// and come back as whole 64-bit words, with no byte realignment.
//
// A wave's area (WordArea<V>::kDw dwords, wave-uniform address) holds one
// block for its 64 lanes, chunk-major: slot c (c < R/16) is 64 lanes x 16
// bytes, lane l's bytes 16c..16c+15 of its block at byte 16l of the slot;
// then two slots of 64 lanes x 4 bytes hold an 8-byte half chunk.  A half
// chunk is the block's last 8 bytes when R % 16 == 8 (SHA3-256/384/512), or
// the end of a final block that stops 8 bytes into a chunk; a block has at
// most one (rem % 16 == 8), and nothing is read past the message end.
template <int V>
struct WordArea {
  static constexpr int R = rate_bytes_of(V);
  static constexpr int kChunks16 = R / 16;
  static constexpr int kHalfDw = kChunks16 * 256;  // dword offset of the half-chunk slots
  static constexpr int kDw = kHalfDw + 2 * 64;
  static_assert(R % 8 == 0, "blocks of whole words");
};

// Start the loads of `rem` bytes (rem % 8 == 0, rem <= R) at `g` into `area`
// (wave-uniform).  When every active lane loads a whole block the pattern is
// fixed and issued without per-chunk lane masks.
template <int V>
__device__ __forceinline__ void words_to_lds(const uint8_t* g, uint32_t rem,
                                             __attribute__((address_space(3))) uint32_t* area) {
  using W = WordArea<V>;
  if (__builtin_amdgcn_ballot_w64(rem != static_cast<uint32_t>(W::R)) == 0) {
#pragma unroll
    for (int c = 0; c < W::kChunks16; ++c)
      __builtin_amdgcn_global_load_lds(g + 16 * c, area + 256 * c, 16, 0, 0);
    if constexpr (W::R % 16 != 0) {
      __builtin_amdgcn_global_load_lds(g + 16 * W::kChunks16, area + W::kHalfDw, 4, 0, 0);
      __builtin_amdgcn_global_load_lds(g + 16 * W::kChunks16 + 4, area + W::kHalfDw + 64, 4, 0, 0);
    }
    return;
  }
#pragma unroll
  for (int c = 0; c < W::kChunks16; ++c)
    if (16u * c + 16u <= rem) __builtin_amdgcn_global_load_lds(g + 16 * c, area + 256 * c, 16, 0, 0);
  if (rem & 8u) {
    const uint32_t h = rem & ~15u;
    __builtin_amdgcn_global_load_lds(g + h, area + W::kHalfDw, 4, 0, 0);
    __builtin_amdgcn_global_load_lds(g + h + 4, area + W::kHalfDw + 64, 4, 0, 0);
  }
}

template <int V, bool PF>
__device__ __forceinline__ void sponge_hash_words(Lane (&A)[25], const uint8_t* msg, uint64_t len,
                                                  __attribute__((address_space(3))) uint32_t* area,
                                                  uint32_t lane) {
  static_assert(V >= 0 && V <= 3, "SHA3-224/256/384/512 only");
  using W = WordArea<V>;
  constexpr int R = W::R;
  constexpr int RQ = R / 8;  // 64-bit words per block = lanes absorbed
  const uint64_t nb = len / R + 1u;
  auto rem_of = [&](uint64_t b) -> uint32_t {
    return b + 1u == nb ? static_cast<uint32_t>(len - b * static_cast<uint64_t>(R))
                        : static_cast<uint32_t>(R);
  };
  // s_waitcnt fields (gfx9): vmcnt in [3:0] and [15:14], expcnt [6:4], lgkmcnt [11:8]
  constexpr int kWaitVm0 = 0x0F70;   // vector memory (these loads included) drained
  constexpr int kWaitLgkm0 = 0xC07F;  // LDS reads drained
  if (PF) words_to_lds<V>(msg, rem_of(0), area);
  // this lane's 16 bytes in chunk slot 0 (dwords; adjacent pairs read as one 64-bit load)
  const __attribute__((address_space(3))) uint32_t* mine = area + 4u * lane;
  for (uint64_t b = 0; b < nb; ++b) {
    const bool fin = b + 1u == nb;
    const uint32_t rem = rem_of(b);
    if (!PF) words_to_lds<V>(msg + b * static_cast<uint64_t>(R), rem, area);
    __builtin_amdgcn_s_waitcnt(kWaitVm0);
    uint2 q[RQ];
    const uint2 half = make_uint2(area[W::kHalfDw + lane], area[W::kHalfDw + 64 + lane]);
#pragma unroll
    for (int j = 0; j < RQ; ++j) {
      if (j < 2 * W::kChunks16) {
        const int d = 256 * (j / 2) + 2 * (j % 2);
        q[j] = make_uint2(mine[d], mine[d + 1]);
      } else {
        q[j] = half;
      }
    }
    // (a wave-uniform test first: the selects below would otherwise run on
    // every block, not only where some lane is at its final one)
    if (__builtin_amdgcn_ballot_w64(fin) != 0 && fin) {
      // past the message: zero; the half chunk of a block ending mid-chunk
#pragma unroll
      for (int j = 0; j < RQ; ++j) {
        if (8u * j >= rem) q[j] = make_uint2(0u, 0u);
        else if ((rem & 8u) && 8u * j + 8u == rem) q[j] = half;
      }
      const uint32_t pw = rem / 8u;
#pragma unroll
      for (int j = 0; j < RQ; ++j) q[j].x |= static_cast<uint32_t>(j) == pw ? 0x06u : 0u;
      q[RQ - 1].y |= 0x80000000u;
    }
    if (b == 0) {
#pragma unroll
      for (int k = 0; k < 25; ++k)
        A[k] = k < RQ ? Lane{q[k < RQ ? k : 0].x, q[k < RQ ? k : 0].y} : Lane{0u, 0u};
    } else {
#pragma unroll
      for (int k = 0; k < RQ; ++k) {
        A[k].lo ^= q[k].x;
        A[k].hi ^= q[k].y;
      }
    }
    if (PF && !fin) {
      __builtin_amdgcn_s_waitcnt(kWaitLgkm0);  // this block's reads done before the area is reused
      words_to_lds<V>(msg + (b + 1u) * static_cast<uint64_t>(R), rem_of(b + 1u), area);
    }
    keccak_rounds_0_22(A);
    if (!fin) keccak_round(A, 23);
  }
  keccak_round(A, 23);
}

// XOF squeeze (Section 3.2: the output is read r bits at a time, applying
// the permutation between reads, until out_len bytes are produced).  A holds
// the state after the last absorbed block's permutation.  Bytes are stored
// one by one unless out_len is a multiple of 4 and `out` is 4-byte aligned.
template <int V>
__device__ __forceinline__ void squeeze_xof(Lane (&A)[25], uint8_t* out, uint64_t out_len) {
  constexpr int R = SpongeShape<V>::kMaxRate;
  const bool words = (out_len & 3u) == 0 && (reinterpret_cast<uintptr_t>(out) & 3u) == 0;
  for (uint64_t done = 0;;) {
#pragma unroll
    for (int k = 0; k < R / 4; ++k) {
      const uint32_t v = (k & 1) ? A[k >> 1].hi : A[k >> 1].lo;
      const uint64_t at = done + 4u * k;
      if (at >= out_len) break;
      if (words) {
        *reinterpret_cast<uint32_t*>(out + at) = v;
      } else {
        for (int q = 0; q < 4 && at + q < out_len; ++q) out[at + q] = static_cast<uint8_t>(v >> (8 * q));
      }
    }
    done += R;
    if (done >= out_len) break;
    keccak_f1600(A);
  }
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
