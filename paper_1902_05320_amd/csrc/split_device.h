// Lane-split sponge: one Keccak-f[1600] state shared by five lanes of a
// wave, for the latency of few long messages.  One message's absorb is a
// serial chain of permutations (Section 3.2, eq. 13), so one thread per
// message leaves a lone long message at the issue rate of a single wave;
// splitting the state cuts the instructions each lane issues per round from
// about 180 to about 90.
//
// A group is eight consecutive lanes of the wave (one 8-lane DPP half-row).
// Lanes t = 0..4 each hold five 64-bit words of the state in registers
// j = 0..4; lanes 5..7 hold zeros so the theta column sums can run as full
// half-row DPP xors.  Word (x, y) is state word x + 5y (Section 3.1, eq. 1).
// Two layouts alternate:
//   diagonal  register j of lane t holds word (j, (j + 2t) mod 5)
//   row       register j of lane t holds word ((j + 2t) mod 5, t)
// A round starts in the diagonal layout, where every lane holds exactly one
// word of each column, so theta's column parity of column j is the xor of
// register j over the group (three DPP xors).  rho rotates each word by its
// own amount, which here depends on the lane.  pi sends (x, y) to
// (y, 2x + 3y) (eq. 6); applied to (j, j + 2t) that is (j + 2t, t), so pi
// turns the diagonal layout into the row layout without moving any data.
// chi combines words along a row, and since register j + k of lane t holds
// the word k columns further along the row, it reads registers j + 1 and
// j + 2 in every lane alike.  iota touches word (0, 0): register 0 of lane 0.
// One exchange through LDS then restores the diagonal layout: word (c, r)
// sits in register (c - 2r) mod 5 of lane r in the row layout.
//
// The exchange relies on a wave's LDS operations executing in issue order:
// every lane's row is written before any lane of the wave reads it back,
// and a row is overwritten only after the reads of the previous round
// returned (the new values depend on them).
#pragma once

#include "sponge_device.h"

namespace kb {
namespace split {

constexpr int kGroupLanes = 8;            // lanes per state
constexpr int kGroupSlots = 8 * 5;        // LDS words per group: one 5-word row per lane
constexpr int kAbsent = 25;               // "no state word" for the zero lanes

// Xor of v over the eight lanes of the group (quad_perm [1,0,3,2], then
// quad_perm [2,3,0,1], then row_half_mirror).
__device__ __forceinline__ uint32_t group_xor(uint32_t v) {
  v ^= static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0xB1, 0xF, 0xF, false));
  v ^= static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x4E, 0xF, 0xF, false));
  v ^= static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0x141, 0xF, 0xF, false));
  return v;
}

// Per-lane constants of the split form.
struct SplitLane {
  uint32_t sh[5];    // v_alignbit amount of register j's rho rotation
  bool swap[5];      // rho first swaps the halves of register j
  uint32_t li[5];    // state word of register j in the diagonal layout (kAbsent on zero lanes)
  uint32_t iota;     // all ones on lane 0, which holds word (0, 0) after chi
  uint64_t* row;     // LDS row this lane writes in the exchange
  const uint64_t* src[5];  // LDS word register j is read back from
};

// `t` is the lane's index in its group, `grp` the group's kGroupSlots words
// of LDS, `zero` one LDS word that holds 0.
__device__ __forceinline__ void setup(SplitLane& L, uint32_t t, uint64_t* grp, const uint64_t* zero) {
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    int n = 0, li = kAbsent, rr = 0;
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      const int y = (j + 2 * q) % 5;
      if (t == static_cast<uint32_t>(q)) {
        n = kMaps.rot[j + 5 * y];
        li = j + 5 * y;
        rr = 5 * y + (q - j + 5) % 5;  // row y, register (q - j) mod 5 = (j - 2y) mod 5
      }
    }
    // rotl(v, n): for 0 < n < 32 alignbit by 32 - n; n = 32 is alignbit by 0
    // (a swap); n > 32 and n = 0 swap first and then rotate by n - 32 resp. 32
    L.swap[j] = n == 0 || n > 32;
    L.sh[j] = static_cast<uint32_t>((32 - (n & 31)) & 31);
    L.li[j] = static_cast<uint32_t>(li);
    L.src[j] = t < 5 ? grp + rr : zero;
  }
  L.iota = t == 0 ? ~0u : 0u;
  L.row = grp + 5 * t;
}

__device__ __forceinline__ Lane rotl_lane(Lane v, uint32_t sh, bool sw) {
  const uint32_t lo = sw ? v.hi : v.lo, hi = sw ? v.lo : v.hi;
  return Lane{__builtin_amdgcn_alignbit(lo, hi, sh), __builtin_amdgcn_alignbit(hi, lo, sh)};
}

// One round (eq. 10) on the group's state, diagonal layout in and out.
__device__ __forceinline__ void split_round(Lane (&a)[5], const SplitLane& L, int r) {
  // theta (eqs. 2-4): column parities over the group
  Lane C[5];
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    C[j].lo = group_xor(a[j].lo);
    C[j].hi = group_xor(a[j].hi);
  }
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    const Lane d = rotl(C[(j + 1) % 5], 1);
    a[j].lo = xor3(a[j].lo, C[(j + 4) % 5].lo, d.lo);
    a[j].hi = xor3(a[j].hi, C[(j + 4) % 5].hi, d.hi);
  }
  // rho (eq. 5) with per-lane amounts; pi (eq. 6) is the change of layout
#pragma unroll
  for (int j = 0; j < 5; ++j) a[j] = rotl_lane(a[j], L.sh[j], L.swap[j]);
  // chi (eq. 7) along the row
  Lane b[5];
#pragma unroll
  for (int j = 0; j < 5; ++j) b[j] = a[j];
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    a[j].lo = b[j].lo ^ (~b[(j + 1) % 5].lo & b[(j + 2) % 5].lo);
    a[j].hi = b[j].hi ^ (~b[(j + 1) % 5].hi & b[(j + 2) % 5].hi);
  }
  // iota (eqs. 8-9).  The lane mask passes through an empty asm so that the
  // 37 masked round constants are formed round by round instead of being
  // hoisted out of the block loop into as many registers.
  uint32_t m = L.iota;
  __asm__ volatile("" : "+v"(m));
  if (kRC.lo[r]) a[0].lo ^= m & kRC.lo[r];
  if (kRC.hi[r]) a[0].hi ^= m & kRC.hi[r];
  // back to the diagonal layout through LDS
#pragma unroll
  for (int j = 0; j < 5; ++j)
    L.row[j] = static_cast<uint64_t>(a[j].lo) | (static_cast<uint64_t>(a[j].hi) << 32);
  __asm__ volatile("" ::: "memory");
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    const uint64_t v = *L.src[j];
    a[j].lo = static_cast<uint32_t>(v);
    a[j].hi = static_cast<uint32_t>(v >> 32);
  }
  __asm__ volatile("" ::: "memory");
}

__device__ __forceinline__ void split_permute(Lane (&a)[5], const SplitLane& L) {
#pragma unroll
  for (int r = 0; r < 24; ++r) split_round(a, L, r);
}

// The dwords holding the bytes of register j's word in one block, read
// ahead of the permutation that precedes their absorption.
struct BlockWords {
  uint32_t w[5][3];
};

// Load register j's word of the block starting at message byte `boff`:
// message bytes [boff + 8 li, boff + 8 li + 8), from the aligned dwords that
// hold at least one message byte (`sh` = message address mod 4).
__device__ __forceinline__ void load_words(BlockWords& bw, const uint8_t* msg, uint32_t sh,
                                           uint64_t len, uint64_t boff, int R, const SplitLane& L) {
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    bw.w[j][0] = bw.w[j][1] = bw.w[j][2] = 0u;
    const uint64_t o = boff + 8u * L.li[j];
    if (8u * L.li[j] < static_cast<uint32_t>(R) && o < len) {
      const uint64_t left = len - o;
      const uint32_t nv = sh + (left < 8u ? static_cast<uint32_t>(left) : 8u);
      const uint32_t* base = reinterpret_cast<const uint32_t*>(msg + o - sh);
#pragma unroll
      for (int k = 0; k < 3; ++k)
        if (4u * k < nv) bw.w[j][k] = base[k];
    }
  }
}

// Xor one block into the state (eq. 12's P_i); on the final block (`rem`
// message bytes left, rem < R) keep only message bytes and add the suffix
// and pad10*1 bytes: `pad` at byte rem, 0x80 on byte R - 1.
__device__ __forceinline__ void absorb_words(Lane (&a)[5], const BlockWords& bw, uint32_t sh,
                                             int R, bool fin, uint32_t rem, uint32_t pad,
                                             const SplitLane& L) {
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    const uint32_t li = L.li[j];
    uint32_t lo = __builtin_amdgcn_alignbyte(bw.w[j][1], bw.w[j][0], sh);
    uint32_t hi = __builtin_amdgcn_alignbyte(bw.w[j][2], bw.w[j][1], sh);
    if (fin) {
      const int v = static_cast<int>(rem) - 8 * static_cast<int>(li);  // message bytes in this word
      if (v < 4) lo = v <= 0 ? 0u : lo & ((1u << (8 * v)) - 1u);
      if (v < 8) hi = v <= 4 ? 0u : hi & ((1u << (8 * (v - 4))) - 1u);
      if (v >= 0 && v < 4) lo ^= pad << (8 * v);
      if (v >= 4 && v < 8) hi ^= pad << (8 * (v - 4));
      if (8 * static_cast<int>(li) == R - 8) hi ^= 0x80000000u;
    }
    if (8u * li < static_cast<uint32_t>(R)) {
      a[j].lo ^= lo;
      a[j].hi ^= hi;
    }
  }
}

// The digest: words 0 .. D/8 of the final state (Section 3.2, eq. 15),
// written by the lanes that hold them; in the mixed form (`slot_dw` = 16)
// the slot is filled with zeros past the digest.
__device__ __forceinline__ void store_words(uint32_t* o, const Lane (&a)[5], int dw, int slot_dw,
                                            const SplitLane& L) {
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    const int k = 2 * static_cast<int>(L.li[j]);
    if (k < slot_dw) o[k] = k < dw ? a[j].lo : 0u;
    if (k + 1 < slot_dw) o[k + 1] = k + 1 < dw ? a[j].hi : 0u;
  }
}

}  // namespace split
}  // namespace kb
