// Pair lane-split sponge: one Keccak-f[1600] state per two adjacent lanes of
// a wave, 32 messages per wave.  Lane h = 0 of a pair holds the low 32-bit
// halves of the 25 state words, lane h = 1 the high halves (Section 3.1's
// lanes as 32-bit pairs, split across the two lanes).  Every step of a round
// is then half as many instructions per lane as one thread per message, and
// a 64-bit rotation takes the partner lane's half through one DPP move
// (quad_perm [1, 0, 3, 2]): for 0 < n < 32 both lanes compute
// alignbit(own, partner, 32 - n), for n > 32 alignbit(partner, own, 64 - n),
// and n = 32 is the partner's half itself.  About 120 VALU instructions per
// lane and round (30 of them DPP moves), against about 180 for one thread
// per message, and no exchange through memory: a message's chain of
// permutations runs about 1.5 times as fast at a third more issue slots per
// permutation, which suits the longest messages of a large uneven batch.
#pragma once

#include "sponge_device.h"

namespace kb {
namespace pair {

constexpr int kPairLanes = 2;

// The partner lane's value (lanes 2k and 2k + 1 swap).
__device__ __forceinline__ uint32_t partner(uint32_t v) {
  return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(v), 0xB1, 0xF, 0xF, false));
}

// Rotation of the 64-bit word whose half this lane holds, by a compile-time n.
__device__ __forceinline__ uint32_t rotl_half(uint32_t v, int n) {
  if (n == 0) return v;
  const uint32_t p = partner(v);
  if (n == 32) return p;
  if (n < 32) return __builtin_amdgcn_alignbit(v, p, 32 - n);
  return __builtin_amdgcn_alignbit(p, v, 64 - n);
}

// One round (eq. 10) on this lane's halves; `hi` is all ones on the lane
// holding the high halves.
__device__ __forceinline__ void pair_round(uint32_t (&a)[25], uint32_t hi, int r) {
  // theta (eqs. 2-4)
  uint32_t C[5], R[5];
#pragma unroll
  for (int x = 0; x < 5; ++x) C[x] = xor3(xor3(a[x], a[x + 5], a[x + 10]), a[x + 15], a[x + 20]);
#pragma unroll
  for (int x = 0; x < 5; ++x) R[x] = rotl_half(C[x], 1);
#pragma unroll
  for (int y = 0; y < 5; ++y)
#pragma unroll
    for (int x = 0; x < 5; ++x) a[x + 5 * y] = xor3(a[x + 5 * y], C[(x + 4) % 5], R[(x + 1) % 5]);
  // rho and pi (eqs. 5-6)
  uint32_t B[25];
#pragma unroll
  for (int i = 0; i < 25; ++i) B[kMaps.dst[i]] = rotl_half(a[i], kMaps.rot[i]);
  // chi (eq. 7)
#pragma unroll
  for (int y = 0; y < 5; ++y)
#pragma unroll
    for (int x = 0; x < 5; ++x)
      a[x + 5 * y] = B[x + 5 * y] ^ (~B[(x + 1) % 5 + 5 * y] & B[(x + 2) % 5 + 5 * y]);
  // iota (eqs. 8-9): the low or high half of the round constant (the mask
  // passes through an empty asm so the selected constants are formed round
  // by round instead of being hoisted into registers)
  uint32_t m = hi;
  __asm__ volatile("" : "+v"(m));
  if (kRC.lo[r] | kRC.hi[r]) a[0] ^= (m & kRC.hi[r]) | (~m & kRC.lo[r]);
}

__device__ __forceinline__ void pair_permute(uint32_t (&a)[25], uint32_t hi) {
#pragma unroll
  for (int r = 0; r < 24; ++r) pair_round(a, hi, r);
}

// The two aligned dwords holding this lane's half of each word of one block
// (message bytes [boff + 8 i + 4 h, +4) that exist), `sh` = address mod 4.
template <int V>
struct HalfDw {
  uint32_t w[SpongeShape<V>::kMaxRate / 8][2];
};

template <int V>
__device__ __forceinline__ void load_halves(HalfDw<V>& d, const uint8_t* msg, uint32_t sh,
                                            uint64_t len, uint64_t boff, int R, uint32_t h) {
  constexpr int kWords = SpongeShape<V>::kMaxRate / 8;
#pragma unroll
  for (int i = 0; i < kWords; ++i) {
    d.w[i][0] = d.w[i][1] = 0u;
    const uint64_t o = boff + 8u * i + 4u * h;
    if (8 * i < R && o < len) {
      const uint64_t left = len - o;
      const uint32_t nv = sh + (left < 4u ? static_cast<uint32_t>(left) : 4u);
      const uint32_t* base = reinterpret_cast<const uint32_t*>(msg + o - sh);
      d.w[i][0] = base[0];
      if (nv > 4u) d.w[i][1] = base[1];
    }
  }
}

// Xor this lane's halves of one block into the state; on the final block
// (`rem` message bytes left, rem < R) keep only message bytes and add the
// suffix/pad10*1 bytes: `pad` at byte rem, 0x80 on byte R - 1.
template <int V>
__device__ __forceinline__ void absorb_halves(uint32_t (&a)[25], const HalfDw<V>& d, uint32_t sh,
                                              int R, bool fin, uint32_t rem, uint32_t pad,
                                              uint32_t h) {
  constexpr int kWords = SpongeShape<V>::kMaxRate / 8;
#pragma unroll
  for (int i = 0; i < kWords; ++i) {
    uint32_t v = __builtin_amdgcn_alignbyte(d.w[i][1], d.w[i][0], sh);
    if (fin) {
      const int k = static_cast<int>(rem) - (8 * i + 4 * static_cast<int>(h));  // message bytes here
      if (k < 4) v = k <= 0 ? 0u : v & ((1u << (8 * k)) - 1u);
      if (k >= 0 && k < 4) v ^= pad << (8 * k);
      if (8 * i == R - 8 && h) v ^= 0x80000000u;
    }
    if (8 * i < R) a[i] ^= v;
  }
}

// The digest's dwords 2 i + h (Section 3.2, eq. 15) from this lane, zero past
// the digest up to `slot_dw`.
__device__ __forceinline__ void store_halves(uint32_t* o, const uint32_t (&a)[25], int dw, int slot_dw,
                                             uint32_t h) {
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int k = 2 * i + static_cast<int>(h);
    if (k < slot_dw) o[k] = k < dw ? a[i] : 0u;
  }
}

}  // namespace pair
}  // namespace kb
