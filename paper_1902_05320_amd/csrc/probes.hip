// Measurement probes: the chip's sustained 32-bit VALU issue rate and shader
// clock, the throughput of the library's own Keccak-f[1600] on register-held
// states (no memory traffic), and a device-to-device copy of known size (for
// scaling memory counters).  They back the roofline figures reported for the
// hashing kernels; nothing on the hashing path calls them.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kbatch.h"
#include "keccak_device.h"

namespace {

constexpr int kProbeBlock = 256;
constexpr int kChains = 16;  // independent dependency chains per thread

// Each iteration issues kChains independent v_bitop3 (each chain depends
// only on itself), so with enough resident waves the SIMDs issue at their
// logic-op rate; no memory is touched inside the loop.
__global__ __launch_bounds__(kProbeBlock) void k_valu_probe(uint32_t iters, uint32_t seed,
                                                            uint32_t* __restrict__ sink,
                                                            uint64_t* __restrict__ clocks) {
  uint32_t a[kChains], k1[kChains], k2[kChains];
#pragma unroll
  for (int j = 0; j < kChains; ++j) {
    a[j] = seed + threadIdx.x * 7u + j;
    k1[j] = threadIdx.x * 5u + j;
    k2[j] = threadIdx.x ^ (11u * j);
  }
  const bool timer = blockIdx.x == 0 && threadIdx.x == 0;
  uint64_t c0 = 0, w0 = 0;
  if (timer) {
    c0 = clock64();
    w0 = wall_clock64();
  }
  for (uint32_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int j = 0; j < kChains; ++j) a[j] = __builtin_amdgcn_bitop3_b32(a[j], k1[j], k2[j], 0xd2);
  }
  uint32_t r = 0;
#pragma unroll
  for (int j = 0; j < kChains; ++j) r ^= a[j];
  if (timer) {
    clocks[0] = clock64() - c0;
    clocks[1] = wall_clock64() - w0;
  }
  if (r == 0x9E3779B9u) sink[0] = r;  // keeps the chains live
}

// Each thread applies the permutation `iters` times to one state held in
// registers: the hashing kernels' arithmetic with nothing else around it, so
// its rate is what the permutation's instruction stream itself sustains.
__global__ __launch_bounds__(kProbeBlock) void k_perm_probe(uint32_t iters,
                                                            uint32_t* __restrict__ sink) {
  kb::Lane A[25];
#pragma unroll
  for (int k = 0; k < 25; ++k)
    A[k] = kb::Lane{threadIdx.x * 7u + static_cast<uint32_t>(k), blockIdx.x + 3u * k};
  for (uint32_t it = 0; it < iters; ++it) kb::keccak_f1600(A);
  uint32_t r = 0;
#pragma unroll
  for (int k = 0; k < 25; ++k) r ^= A[k].lo ^ A[k].hi;
  if (r == 0x9E3779B9u) sink[0] = r;  // keeps the states live
}

__global__ __launch_bounds__(kProbeBlock) void k_copy_probe(const uint4* __restrict__ src,
                                                           uint4* __restrict__ dst, uint64_t n16) {
  for (uint64_t k = static_cast<uint64_t>(blockIdx.x) * kProbeBlock + threadIdx.x; k < n16;
       k += static_cast<uint64_t>(gridDim.x) * kProbeBlock)
    dst[k] = src[k];
}

}  // namespace

extern "C" {

int keccak_probe_valu(uint32_t iters, double* tops, double* sclk_mhz, hipStream_t stream) {
  if (!tops || !sclk_mhz || iters == 0) return KB_EINVAL;
  int dev = 0, cus = 0, wall_khz = 0;
  if (hipGetDevice(&dev) != hipSuccess) return KB_EHIP;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return KB_EHIP;
  if (hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess)
    return KB_EHIP;
  uint32_t* sink = nullptr;
  uint64_t* clocks = nullptr;
  if (hipMalloc(&sink, 4) != hipSuccess) return KB_ENOMEM;
  if (hipMalloc(&clocks, 16) != hipSuccess) {
    (void)hipFree(sink);
    return KB_ENOMEM;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = KB_OK;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = KB_EHIP;
  const uint32_t grid = static_cast<uint32_t>(cus) * 8u;  // 8 waves per SIMD
  if (rc == KB_OK) {
    hipLaunchKernelGGL(k_valu_probe, dim3(grid), dim3(kProbeBlock), 0, stream, iters / 8 + 1, 1u,
                       sink, clocks);  // warm the clocks up
    (void)hipEventRecord(e0, stream);
    hipLaunchKernelGGL(k_valu_probe, dim3(grid), dim3(kProbeBlock), 0, stream, iters, 1u, sink,
                       clocks);
    (void)hipEventRecord(e1, stream);
    if (hipGetLastError() != hipSuccess || hipEventSynchronize(e1) != hipSuccess) rc = KB_EHIP;
  }
  if (rc == KB_OK) {
    float ms = 0.f;
    uint64_t c[2] = {0, 0};
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess ||
        hipMemcpy(c, clocks, 16, hipMemcpyDeviceToHost) != hipSuccess) {
      rc = KB_EHIP;
    } else {
      const double ops = static_cast<double>(grid) * kProbeBlock * iters * kChains;
      *tops = ops / (ms * 1e-3) / 1e12;
      const double wall_s = static_cast<double>(c[1]) / (wall_khz * 1e3);
      *sclk_mhz = wall_s > 0 ? static_cast<double>(c[0]) / wall_s / 1e6 : 0.0;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(sink);
  (void)hipFree(clocks);
  return rc;
}

int keccak_probe_perm(uint32_t iters, int waves_per_simd, double* gperm_s, int* waves_used,
                      hipStream_t stream) {
  if (!gperm_s || !waves_used || iters == 0 || waves_per_simd < 0) return KB_EINVAL;
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return KB_EHIP;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return KB_EHIP;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_perm_probe, kProbeBlock, 0) !=
          hipSuccess ||
      per_cu < 1)
    return KB_EHIP;
  // a 256-thread workgroup puts one wave on each SIMD of its CU
  const int waves = waves_per_simd == 0 || waves_per_simd > per_cu ? per_cu : waves_per_simd;
  uint32_t* sink = nullptr;
  if (hipMalloc(&sink, 4) != hipSuccess) return KB_ENOMEM;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = KB_OK;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = KB_EHIP;
  const uint32_t grid = static_cast<uint32_t>(cus) * static_cast<uint32_t>(waves);
  if (rc == KB_OK) {
    hipLaunchKernelGGL(k_perm_probe, dim3(grid), dim3(kProbeBlock), 0, stream, iters / 4 + 1,
                       sink);  // warm the clocks up
    (void)hipEventRecord(e0, stream);
    hipLaunchKernelGGL(k_perm_probe, dim3(grid), dim3(kProbeBlock), 0, stream, iters, sink);
    (void)hipEventRecord(e1, stream);
    if (hipGetLastError() != hipSuccess || hipEventSynchronize(e1) != hipSuccess) rc = KB_EHIP;
  }
  if (rc == KB_OK) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess || ms <= 0.f) {
      rc = KB_EHIP;
    } else {
      *gperm_s = static_cast<double>(grid) * kProbeBlock * iters / (ms * 1e-3) / 1e9;
      *waves_used = waves;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(sink);
  return rc;
}

int keccak_probe_copy(const uint8_t* d_src, uint8_t* d_dst, uint64_t bytes, double* gbps,
                      hipStream_t stream) {
  if (!d_src || !d_dst || !gbps || bytes % 16 || !bytes) return KB_EINVAL;
  if (reinterpret_cast<uintptr_t>(d_src) % 16 || reinterpret_cast<uintptr_t>(d_dst) % 16)
    return KB_EINVAL;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return KB_EHIP;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return KB_EHIP;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return KB_EHIP;
  }
  const uint32_t grid = static_cast<uint32_t>(cus) * 16u;
  const uint64_t n16 = bytes / 16;
  int rc = KB_OK;
  (void)hipEventRecord(e0, stream);
  hipLaunchKernelGGL(k_copy_probe, dim3(grid), dim3(kProbeBlock), 0, stream,
                     reinterpret_cast<const uint4*>(d_src), reinterpret_cast<uint4*>(d_dst), n16);
  (void)hipEventRecord(e1, stream);
  float ms = 0.f;
  if (hipGetLastError() != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
      hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
    rc = KB_EHIP;
  else
    *gbps = 2.0 * static_cast<double>(bytes) / (ms * 1e-3) / 1e9;  // read + write
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

}  // extern "C"
