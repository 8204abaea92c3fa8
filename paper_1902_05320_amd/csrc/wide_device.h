// Wide lane-split sponge: one Keccak-f[1600] state per 32 lanes of a wave,
// one 64-bit state word per lane (lanes 25..31 of each half idle), two
// messages per wave.  The serial absorb chain of one message (Section 3.2)
// then costs each lane about twenty VALU instructions per round instead of
// the ~180 of one thread per message or the ~86 of the five-lane form; the
// price is two exchanges through LDS per round.
//
// Lane i of a half holds word i = x + 5y (Section 3.1, eq. 1).  Each half
// owns an LDS area of kAreaSlots 64-bit slots:
//   theta area  slots 6x + y: column x, padded to six slots (48 bytes) so
//               that a column is read with two 16-byte and one 8-byte load
//   chi area    slots 30 + 10y + x and 30 + 10y + x + 5: row y written twice,
//               so that words x, x+1, x+2 (mod 5) of a row lie at three
//               consecutive slots
//   spare       slot 80, written by the idle lanes
// Per round (eq. 10):
//   theta  every lane writes its word to the theta area and reads columns
//          x - 1 and x + 1, so it forms C[x-1] and C[x+1] itself and applies
//          D[x] = C[x-1] ^ rot(C[x+1], 1) to its word (eqs. 2-4);
//   rho    rotates by the lane's own amount (eq. 5);
//   pi     is where the word is written in the chi area: word (x, y) goes to
//          (y, 2x + 3y) (eq. 6);
//   chi    reads its row neighbours x + 1 and x + 2 (eq. 7);
//   iota   lane 0 only (eqs. 8-9).
// The exchanges rely on a wave's LDS operations executing in issue order:
// every lane's write precedes the reads of the same round, and a slot is
// written again only after the reads of the previous round have returned
// (the new value depends on them).
#pragma once

#include "sponge_device.h"

namespace kb {
namespace wide {

constexpr int kHalfLanes = 32;   // lanes per state
constexpr int kThetaSlots = 30;
constexpr int kChiBase = 30;
constexpr int kSpare = 80;
constexpr int kAreaSlots = 82;   // 656 bytes, a multiple of 16

// Per-lane constants of the wide form.
struct WideLane {
  uint32_t word;       // state word of this lane (25 and up: idle)
  uint32_t sh;         // rho: v_alignbit amount
  bool swap;           // rho: swap the halves first
  uint32_t iota;       // all ones on word 0
  uint64_t* tw;        // theta write slot
  const uint64_t* cm;  // column x - 1
  const uint64_t* cp;  // column x + 1
  uint64_t* pw0;       // pi destination, both copies of its row
  uint64_t* pw1;
  const uint64_t* cr;  // row neighbours x, x + 1, x + 2 of this lane's word after pi
};

// `h` is the lane's index in its half, `area` the half's kAreaSlots slots
// (16-byte aligned).
__device__ __forceinline__ void setup(WideLane& L, uint32_t h, uint64_t* area) {
  const bool on = h < 25u;
  const uint32_t i = on ? h : 0u;
  const uint32_t x = i % 5u, y = i / 5u;
  int n = 0;
#pragma unroll
  for (int k = 0; k < 25; ++k)
    if (static_cast<int>(i) == k) n = kMaps.rot[k];
  // rotl(v, n) as in the five-lane form: for 0 < n < 32 alignbit by 32 - n;
  // n = 32 is alignbit by 0 (a swap); n > 32 and n = 0 swap first
  L.swap = n == 0 || n > 32;
  L.sh = static_cast<uint32_t>((32 - (n & 31)) & 31);
  L.word = h;
  L.iota = h == 0u ? ~0u : 0u;
  L.tw = on ? area + 6u * x + y : area + kSpare;
  L.cm = area + 6u * ((x + 4u) % 5u);
  L.cp = area + 6u * ((x + 1u) % 5u);
  // pi: word (x, y) becomes word (y, 2x + 3y)
  const uint32_t px = y, py = (2u * x + 3u * y) % 5u;
  L.pw0 = on ? area + kChiBase + 10u * py + px : area + kSpare;
  L.pw1 = on ? area + kChiBase + 10u * py + px + 5u : area + kSpare;
  L.cr = area + kChiBase + 10u * y + x;
}

__device__ __forceinline__ uint64_t pack(Lane v) {
  return static_cast<uint64_t>(v.lo) | (static_cast<uint64_t>(v.hi) << 32);
}
__device__ __forceinline__ Lane unpack(uint64_t v) {
  return Lane{static_cast<uint32_t>(v), static_cast<uint32_t>(v >> 32)};
}

// Column parity of the five words at `col` (two 16-byte and one 8-byte LDS load).
__device__ __forceinline__ Lane column_parity(const uint64_t* col) {
  const uint4 w01 = reinterpret_cast<const uint4*>(col)[0];
  const uint4 w23 = reinterpret_cast<const uint4*>(col)[1];
  const uint2 w4 = reinterpret_cast<const uint2*>(col)[4];
  return Lane{xor3(xor3(w01.x, w01.z, w23.x), w23.z, w4.x), xor3(xor3(w01.y, w01.w, w23.y), w23.w, w4.y)};
}

// One round (eq. 10) on the half's state, one word per lane.
__device__ __forceinline__ void wide_round(Lane& a, const WideLane& L, int r) {
  // theta (eqs. 2-4)
  *L.tw = pack(a);
  __asm__ volatile("" ::: "memory");
  const Lane cm = column_parity(L.cm);
  const Lane cp = column_parity(L.cp);
  __asm__ volatile("" ::: "memory");
  const Lane d = rotl(cp, 1);
  a.lo = xor3(a.lo, cm.lo, d.lo);
  a.hi = xor3(a.hi, cm.hi, d.hi);
  // rho (eq. 5) by the lane's amount
  {
    const uint32_t lo = L.swap ? a.hi : a.lo, hi = L.swap ? a.lo : a.hi;
    a = Lane{__builtin_amdgcn_alignbit(lo, hi, L.sh), __builtin_amdgcn_alignbit(hi, lo, L.sh)};
  }
  // pi (eq. 6) as the write position, chi (eq. 7) along the row
  const uint64_t v = pack(a);
  *L.pw0 = v;
  *L.pw1 = v;
  __asm__ volatile("" ::: "memory");
  const Lane b0 = unpack(L.cr[0]), b1 = unpack(L.cr[1]), b2 = unpack(L.cr[2]);
  __asm__ volatile("" ::: "memory");
  a.lo = b0.lo ^ (~b1.lo & b2.lo);
  a.hi = b0.hi ^ (~b1.hi & b2.hi);
  // iota (eqs. 8-9) on word 0 (the mask passes through an empty asm so the
  // masked constants are formed round by round, not hoisted into registers)
  uint32_t m = L.iota;
  __asm__ volatile("" : "+v"(m));
  if (kRC.lo[r]) a.lo ^= m & kRC.lo[r];
  if (kRC.hi[r]) a.hi ^= m & kRC.hi[r];
}

__device__ __forceinline__ void wide_permute(Lane& a, const WideLane& L) {
#pragma unroll
  for (int r = 0; r < 24; ++r) wide_round(a, L, r);
}

// The dwords holding the bytes of this lane's word of the block at message
// byte `boff` (message bytes [boff + 8 word, boff + 8 word + 8) that exist),
// read from aligned dwords (`sh` = message address mod 4).
struct WordDw {
  uint32_t w[3];
};

__device__ __forceinline__ void load_word(WordDw& d, const uint8_t* msg, uint32_t sh, uint64_t len,
                                          uint64_t boff, int R, const WideLane& L) {
  d.w[0] = d.w[1] = d.w[2] = 0u;
  const uint64_t o = boff + 8u * L.word;
  if (8u * L.word < static_cast<uint32_t>(R) && o < len) {
    const uint64_t left = len - o;
    const uint32_t nv = sh + (left < 8u ? static_cast<uint32_t>(left) : 8u);
    const uint32_t* base = reinterpret_cast<const uint32_t*>(msg + o - sh);
#pragma unroll
    for (int k = 0; k < 3; ++k)
      if (4u * k < nv) d.w[k] = base[k];
  }
}

// Xor this lane's word of one block into the state (eq. 12's P_i); on the
// final block (`rem` message bytes left, rem < R) only message bytes are
// kept and the suffix/pad10*1 bytes are added: `pad` at byte rem, 0x80 on
// byte R - 1.
__device__ __forceinline__ void absorb_word(Lane& a, const WordDw& d, uint32_t sh, int R, bool fin,
                                            uint32_t rem, uint32_t pad, const WideLane& L) {
  uint32_t lo = __builtin_amdgcn_alignbyte(d.w[1], d.w[0], sh);
  uint32_t hi = __builtin_amdgcn_alignbyte(d.w[2], d.w[1], sh);
  if (fin) {
    const int v = static_cast<int>(rem) - 8 * static_cast<int>(L.word);  // message bytes in this word
    if (v < 4) lo = v <= 0 ? 0u : lo & ((1u << (8 * v)) - 1u);
    if (v < 8) hi = v <= 4 ? 0u : hi & ((1u << (8 * (v - 4))) - 1u);
    if (v >= 0 && v < 4) lo ^= pad << (8 * v);
    if (v >= 4 && v < 8) hi ^= pad << (8 * (v - 4));
    if (8 * static_cast<int>(L.word) == R - 8) hi ^= 0x80000000u;
  }
  if (8u * L.word < static_cast<uint32_t>(R)) {
    a.lo ^= lo;
    a.hi ^= hi;
  }
}

// The digest (Section 3.2, eq. 15): words 0 .. D/8 of the final state, each
// written by the lane that holds it; with `slot_dw` = 16 (mixed form) the
// slot is filled with zeros past the digest.
__device__ __forceinline__ void store_word(uint32_t* o, Lane a, int dw, int slot_dw, const WideLane& L) {
  const int k = 2 * static_cast<int>(L.word);
  if (L.word < 25u) {
    if (k < slot_dw) o[k] = k < dw ? a.lo : 0u;
    if (k + 1 < slot_dw) o[k + 1] = k + 1 < dw ? a.hi : 0u;
  }
}

}  // namespace wide
}  // namespace kb
