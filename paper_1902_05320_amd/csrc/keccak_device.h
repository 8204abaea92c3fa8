// Keccak-f[1600] and the SHA-3 sponge as gfx950 device code.
//
// Layout: one 1600-bit state per thread, 25 lanes of 64 bits held as 50
// 32-bit VGPRs (lo/hi halves).  Lane (x, y) is index x + 5y (Section 3.1,
// eq. 1) and holds the little-endian 64-bit word at byte 8(x + 5y) of the
// state, so message bytes absorb with plain little-endian dword loads.
//
// All 24 rounds are fully unrolled: pi (eq. 6) is pure register renaming,
// the rho (eq. 5) rotation amounts and the iota round constants (eqs. 8-9)
// are instruction immediates, and no memory is touched by the permutation.
// Per round the VALU work is
//   theta column parities   20 v_bitop3 (3-input xor)
//   theta rot-by-1 of C     10 v_alignbit
//   theta apply             50 v_bitop3 (A ^ C[x-1] ^ rot(C[x+1]))
//   rho                     48 v_alignbit (no offset is 0 or 32 mod 64)
//   chi                     50 v_bitop3 (a ^ (~b & c))
//   iota                    1-2 v_xor with a literal
// about 180 instructions, 4.3K per permutation.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kb {

// ---------------------------------------------------------------------------
// Compile-time constants, generated from their definitions.
// ---------------------------------------------------------------------------

struct RoundConstants {
  uint32_t lo[24];
  uint32_t hi[24];
};

// iota (Definition 5): RC bit 2^j - 1 of round i_r is rc(j + 7 i_r), j = 0..6.
// rc is the output bit of the degree-8 LFSR x^8 + x^6 + x^5 + x^4 + 1; here it
// runs in Galois form on a byte (bit i = register cell i): emit bit 0, shift
// up, and fold a carried-out bit 7 back into cells 0, 4, 5, 6 (mask 0x71).
constexpr RoundConstants make_round_constants() {
  RoundConstants t{};
  unsigned reg = 1u;
  for (int r = 0; r < 24; ++r) {
    unsigned long long c = 0;
    for (int j = 0; j < 7; ++j) {
      if (reg & 1u) c |= 1ull << ((1u << j) - 1u);
      reg = (reg & 0x80u) ? (((reg << 1) ^ 0x71u) & 0xFFu) : ((reg << 1) & 0xFFu);
    }
    t.lo[r] = static_cast<uint32_t>(c);
    t.hi[r] = static_cast<uint32_t>(c >> 32);
  }
  return t;
}

struct LaneMaps {
  int rot[25];  // rho: left-rotation amount of lane i
  int dst[25];  // pi: where lane i goes
};

// rho (Definition 2): walking (x, y) from (1, 0) with (x, y) <- (y, 2x + 3y),
// step t rotates its lane by (t+1)(t+2)/2 mod 64.  pi (Definition 3) sends
// lane (X, Y) to (Y, 2X + 3Y mod 5), the inverse reading of A'[x, y] =
// A[x + 3y, x].
constexpr LaneMaps make_lane_maps() {
  LaneMaps m{};
  for (int i = 0; i < 25; ++i) m.rot[i] = 0;
  int x = 1, y = 0;
  for (int t = 0; t < 24; ++t) {
    m.rot[x + 5 * y] = ((t + 1) * (t + 2) / 2) % 64;
    const int nx = y, ny = (2 * x + 3 * y) % 5;
    x = nx;
    y = ny;
  }
  for (int X = 0; X < 5; ++X)
    for (int Y = 0; Y < 5; ++Y) m.dst[X + 5 * Y] = Y + 5 * ((2 * X + 3 * Y) % 5);
  return m;
}

constexpr RoundConstants kRC = make_round_constants();
constexpr LaneMaps kMaps = make_lane_maps();

// ---------------------------------------------------------------------------
// 64-bit lanes as 32-bit pairs.
// ---------------------------------------------------------------------------

struct Lane {
  uint32_t lo, hi;
};

__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);  // truth table of a^b^c
}

// Left rotation by a compile-time amount (after unrolling) with v_alignbit:
// alignbit(a, b, s) = low 32 bits of ({a, b} >> s).
__device__ __forceinline__ Lane rotl(Lane v, int n) {
  if (n == 0) return v;
  if (n == 32) return Lane{v.hi, v.lo};
  if (n < 32)
    return Lane{__builtin_amdgcn_alignbit(v.lo, v.hi, 32 - n),
                __builtin_amdgcn_alignbit(v.hi, v.lo, 32 - n)};
  return Lane{__builtin_amdgcn_alignbit(v.hi, v.lo, 64 - n),
              __builtin_amdgcn_alignbit(v.lo, v.hi, 64 - n)};
}

// One round Rnd(A, i_r) = iota(chi(pi(rho(theta(A))))) (eq. 10), in place.
// `r` must fold to a constant after unrolling.
__device__ __forceinline__ void keccak_round(Lane (&A)[25], int r) {
  // theta (eqs. 2-4)
  Lane C[5];
#pragma unroll
  for (int x = 0; x < 5; ++x) {
    C[x].lo = xor3(xor3(A[x].lo, A[x + 5].lo, A[x + 10].lo), A[x + 15].lo, A[x + 20].lo);
    C[x].hi = xor3(xor3(A[x].hi, A[x + 5].hi, A[x + 10].hi), A[x + 15].hi, A[x + 20].hi);
  }
  Lane R1[5];
#pragma unroll
  for (int x = 0; x < 5; ++x) R1[x] = rotl(C[x], 1);
#pragma unroll
  for (int y = 0; y < 5; ++y)
#pragma unroll
    for (int x = 0; x < 5; ++x) {
      Lane& a = A[x + 5 * y];
      a.lo = xor3(a.lo, C[(x + 4) % 5].lo, R1[(x + 1) % 5].lo);
      a.hi = xor3(a.hi, C[(x + 4) % 5].hi, R1[(x + 1) % 5].hi);
    }
  // rho and pi
  Lane B[25];
#pragma unroll
  for (int i = 0; i < 25; ++i) B[kMaps.dst[i]] = rotl(A[i], kMaps.rot[i]);
  // chi (eq. 7)
#pragma unroll
  for (int y = 0; y < 5; ++y)
#pragma unroll
    for (int x = 0; x < 5; ++x) {
      const Lane a = B[x + 5 * y], b = B[(x + 1) % 5 + 5 * y], c = B[(x + 2) % 5 + 5 * y];
      A[x + 5 * y].lo = a.lo ^ (~b.lo & c.lo);
      A[x + 5 * y].hi = a.hi ^ (~b.hi & c.hi);
    }
  // iota (eqs. 8-9)
  if (kRC.lo[r]) A[0].lo ^= kRC.lo[r];
  if (kRC.hi[r]) A[0].hi ^= kRC.hi[r];
}

// Rounds 0..22 of Keccak-f[1600]; the last round is issued by the caller so
// that the final block can let dead-code elimination drop the lanes it does
// not output.
__device__ __forceinline__ void keccak_rounds_0_22(Lane (&A)[25]) {
#pragma unroll
  for (int r = 0; r < 23; ++r) keccak_round(A, r);
}

__device__ __forceinline__ void keccak_f1600(Lane (&A)[25]) {
  keccak_rounds_0_22(A);
  keccak_round(A, 23);
}

// ---------------------------------------------------------------------------
// SHA-3 parameters (Section 3.3): c = 2d, r = 1600 - c.
// ---------------------------------------------------------------------------

// Variants 0..3 are SHA3-224/256/384/512: digest D = d/8 bytes, capacity
// c = 2d bits, rate R = 200 - 2D bytes.
__host__ __device__ constexpr int digest_bytes_of(int v) {
  return v == 0 ? 28 : v == 1 ? 32 : v == 2 ? 48 : 64;
}
__host__ __device__ constexpr int rate_bytes_of(int v) { return 200 - 2 * digest_bytes_of(v); }

static_assert(rate_bytes_of(0) == 144 && rate_bytes_of(1) == 136 && rate_bytes_of(2) == 104 &&
                  rate_bytes_of(3) == 72,
              "SHA-3 rates");

}  // namespace kb
