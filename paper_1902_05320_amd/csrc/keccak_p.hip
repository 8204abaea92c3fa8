// Keccak-p[b, n_r] for every width of Table 1 (Section 3.1): b = 25w with
// w = 2^l, l = 0..6, and any number of rounds n_r.  Round i_r runs from
// 12 + 2l - n_r to 12 + 2l - 1 (FIPS 202's indexing; the paper leaves it
// unstated), so Keccak-p[1600, 24] is Keccak-f[1600].
//
// One thread per state.  A lane of w <= 32 bits lives in one 32-bit
// register (masked to w bits, rotations modulo w); a 64-bit lane in a lo/hi
// pair as in the SHA-3 path.  The rho amounts are the same walk taken
// modulo w, and round constant i_r keeps the bits 2^j - 1 < w of the 64-bit
// one (eq. 8: j = 0..l), looked up by i_r mod 255 since rc has period 255.
//
// States are packed b-bit strings: state s occupies ceil(b/8) bytes from
// byte s * ceil(b/8), and string bit k is bit k mod 8 of byte k / 8 (eq. 1
// with that bit order), so for w >= 8 each lane is w/8 little-endian bytes.
// For b = 25, 50 and 100 the unused high bits of the last byte are cleared.
#include <hip/hip_runtime.h>

#include "kb_internal.h"
#include "kbatch.h"
#include "keccak_device.h"

namespace {

struct RoundConstantsAll {
  uint32_t lo[255];
  uint32_t hi[255];
};

// The 64-bit round constants for i_r = 0..254, from the same LFSR as the
// SHA-3 path (rc is periodic with period 255, so these cover every i_r).
constexpr RoundConstantsAll make_rc_all() {
  RoundConstantsAll t{};
  unsigned reg = 1u;
  for (int r = 0; r < 255; ++r) {
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

__constant__ RoundConstantsAll kRCAll = make_rc_all();

constexpr int log2_of(int w) { return w <= 1 ? 0 : 1 + log2_of(w / 2); }

template <int W>
__device__ __forceinline__ uint32_t rotw(uint32_t v, int n) {
  constexpr uint32_t M = W >= 32 ? 0xFFFFFFFFu : (1u << W) - 1u;
  n %= W;
  if (n == 0) return v;
  return ((v << n) | (v >> (W - n))) & M;
}

__device__ __forceinline__ int rc_index(int ir) { return ((ir % 255) + 255) % 255; }

// n_r rounds from i_r = ir0 on lanes of W <= 32 bits.
template <int W>
__device__ void rounds_narrow(uint32_t (&A)[25], int ir0, int nr) {
  constexpr uint32_t M = W >= 32 ? 0xFFFFFFFFu : (1u << W) - 1u;
  for (int k = 0; k < nr; ++k) {
    uint32_t C[5], B[25];
#pragma unroll
    for (int x = 0; x < 5; ++x) C[x] = A[x] ^ A[x + 5] ^ A[x + 10] ^ A[x + 15] ^ A[x + 20];
#pragma unroll
    for (int x = 0; x < 5; ++x) {
      const uint32_t D = C[(x + 4) % 5] ^ rotw<W>(C[(x + 1) % 5], 1);
#pragma unroll
      for (int y = 0; y < 5; ++y) A[x + 5 * y] ^= D;
    }
#pragma unroll
    for (int i = 0; i < 25; ++i) B[kb::kMaps.dst[i]] = rotw<W>(A[i], kb::kMaps.rot[i]);
#pragma unroll
    for (int y = 0; y < 5; ++y)
#pragma unroll
      for (int x = 0; x < 5; ++x)
        A[x + 5 * y] = B[x + 5 * y] ^ (~B[(x + 1) % 5 + 5 * y] & B[(x + 2) % 5 + 5 * y] & M);
    A[0] ^= kRCAll.lo[rc_index(ir0 + k)] & M;
  }
}

// n_r rounds from i_r = ir0 on 64-bit lanes.
__device__ void rounds_wide(kb::Lane (&A)[25], int ir0, int nr) {
  for (int k = 0; k < nr; ++k) {
    kb::Lane C[5], B[25];
#pragma unroll
    for (int x = 0; x < 5; ++x) {
      C[x].lo = kb::xor3(kb::xor3(A[x].lo, A[x + 5].lo, A[x + 10].lo), A[x + 15].lo, A[x + 20].lo);
      C[x].hi = kb::xor3(kb::xor3(A[x].hi, A[x + 5].hi, A[x + 10].hi), A[x + 15].hi, A[x + 20].hi);
    }
#pragma unroll
    for (int x = 0; x < 5; ++x) {
      const kb::Lane r = kb::rotl(C[(x + 1) % 5], 1);
#pragma unroll
      for (int y = 0; y < 5; ++y) {
        A[x + 5 * y].lo = kb::xor3(A[x + 5 * y].lo, C[(x + 4) % 5].lo, r.lo);
        A[x + 5 * y].hi = kb::xor3(A[x + 5 * y].hi, C[(x + 4) % 5].hi, r.hi);
      }
    }
#pragma unroll
    for (int i = 0; i < 25; ++i) B[kb::kMaps.dst[i]] = kb::rotl(A[i], kb::kMaps.rot[i]);
#pragma unroll
    for (int y = 0; y < 5; ++y)
#pragma unroll
      for (int x = 0; x < 5; ++x) {
        const kb::Lane a = B[x + 5 * y], b = B[(x + 1) % 5 + 5 * y], c = B[(x + 2) % 5 + 5 * y];
        A[x + 5 * y].lo = a.lo ^ (~b.lo & c.lo);
        A[x + 5 * y].hi = a.hi ^ (~b.hi & c.hi);
      }
    const int i = rc_index(ir0 + k);
    A[0].lo ^= kRCAll.lo[i];
    A[0].hi ^= kRCAll.hi[i];
  }
}

constexpr int kThreads = 256;

template <int W>
__global__ __launch_bounds__(kThreads) void k_keccak_p(uint8_t* __restrict__ states, uint64_t n,
                                                       int ir0, int nr) {
  constexpr int kBits = 25 * W;
  constexpr int kBytes = (kBits + 7) / 8;
  const uint64_t s = static_cast<uint64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (s >= n) return;
  uint8_t* p = states + s * kBytes;
  if constexpr (W == 64) {
    kb::Lane A[25];
#pragma unroll
    for (int j = 0; j < 25; ++j) {
      uint32_t lo = 0, hi = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        lo |= static_cast<uint32_t>(p[8 * j + q]) << (8 * q);
        hi |= static_cast<uint32_t>(p[8 * j + 4 + q]) << (8 * q);
      }
      A[j] = kb::Lane{lo, hi};
    }
    rounds_wide(A, ir0, nr);
#pragma unroll
    for (int j = 0; j < 25; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        p[8 * j + q] = static_cast<uint8_t>(A[j].lo >> (8 * q));
        p[8 * j + 4 + q] = static_cast<uint8_t>(A[j].hi >> (8 * q));
      }
  } else {
    // the state as 32-bit words of the bit string; a lane (W divides 32)
    // never straddles two words
    constexpr int kWords = (kBits + 31) / 32;
    constexpr uint32_t M = W >= 32 ? 0xFFFFFFFFu : (1u << W) - 1u;
    uint32_t wd[kWords];
#pragma unroll
    for (int k = 0; k < kWords; ++k) wd[k] = 0u;
#pragma unroll
    for (int k = 0; k < kBytes; ++k) wd[k / 4] |= static_cast<uint32_t>(p[k]) << (8 * (k % 4));
    uint32_t A[25];
#pragma unroll
    for (int j = 0; j < 25; ++j) A[j] = (wd[(W * j) / 32] >> ((W * j) % 32)) & M;
    rounds_narrow<W>(A, ir0, nr);
#pragma unroll
    for (int k = 0; k < kWords; ++k) wd[k] = 0u;
#pragma unroll
    for (int j = 0; j < 25; ++j) wd[(W * j) / 32] |= A[j] << ((W * j) % 32);
#pragma unroll
    for (int k = 0; k < kBytes; ++k) p[k] = static_cast<uint8_t>(wd[k / 4] >> (8 * (k % 4)));
  }
}

template <int W>
int launch(uint8_t* d_states, uint64_t n, int nr, hipStream_t stream) {
  const int ir0 = 12 + 2 * log2_of(W) - nr;
  const uint64_t blocks = (n + kThreads - 1) / kThreads;
  if (blocks > 0x7FFFFFFFull) return kb::set_last_error(KB_EINVAL, "too many states for one launch");
  hipLaunchKernelGGL(k_keccak_p<W>, dim3(static_cast<uint32_t>(blocks)), dim3(kThreads), 0, stream,
                     d_states, n, ir0, nr);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return kb::set_last_error(KB_EHIP, hipGetErrorString(e));
  return KB_OK;
}

}  // namespace

extern "C" int keccak_p_batch(int b, int n_rounds, uint8_t* d_states, uint64_t n,
                              hipStream_t stream) {
  kb::set_last_error(KB_OK, "");
  if (n_rounds < 1 || n_rounds > 4096)
    return kb::set_last_error(KB_EINVAL, "n_rounds must be in [1, 4096]");
  if (n && !d_states) return kb::set_last_error(KB_EINVAL, "NULL d_states with n > 0");
  if (n == 0) {
    switch (b) {
      case 25: case 50: case 100: case 200: case 400: case 800: case 1600: return KB_OK;
      default: return kb::set_last_error(KB_EINVAL, "b must be 25, 50, 100, 200, 400, 800 or 1600");
    }
  }
  switch (b) {
    case 25: return launch<1>(d_states, n, n_rounds, stream);
    case 50: return launch<2>(d_states, n, n_rounds, stream);
    case 100: return launch<4>(d_states, n, n_rounds, stream);
    case 200: return launch<8>(d_states, n, n_rounds, stream);
    case 400: return launch<16>(d_states, n, n_rounds, stream);
    case 800: return launch<32>(d_states, n, n_rounds, stream);
    case 1600: return launch<64>(d_states, n, n_rounds, stream);
    default: return kb::set_last_error(KB_EINVAL, "b must be 25, 50, 100, 200, 400, 800 or 1600");
  }
}
