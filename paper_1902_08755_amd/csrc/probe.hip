// Bandwidth probes: the reference points for the measured fraction of HBM
// bandwidth. mode 0 reads `bytes` with 16-byte loads (several in flight per
// lane) and folds them into one word per workgroup; mode 1 copies `bytes`
// from src to dst with 16-byte loads and stores. All accesses are marked
// non-temporal (streaming), which reads and copies faster than the default
// policy on a buffer far larger than the caches. Grid-stride over 32
// workgroups per compute unit.
#include "cmp_internal.hpp"

namespace cmp {

constexpr int kProbeUnroll = 8;

__global__ __launch_bounds__(kThreads) void probe_read_kernel(const u32x4* __restrict__ src,
                                                              int64_t n16, uint32_t* sink) {
  uint32_t acc = 0;
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n16;
       i += stride * kProbeUnroll) {
    // unconditional loads (an index past the end reads the last unit and is
    // discarded): a branch between loads would issue them one at a time
    u32x4 v[kProbeUnroll];
#pragma unroll
    for (int k = 0; k < kProbeUnroll; ++k) {
      const int64_t j = i + k * stride;
      v[k] = __builtin_nontemporal_load(&src[j < n16 ? j : n16 - 1]);
    }
#pragma unroll
    for (int k = 0; k < kProbeUnroll; ++k)
      if (i + k * stride < n16) acc ^= v[k].x ^ v[k].y ^ v[k].z ^ v[k].w;
  }
  if (acc == 0x9E3779B9u) sink[0] = acc;   // (practically) never taken; keeps the loads
}

__global__ __launch_bounds__(kThreads) void probe_copy_kernel(const u32x4* __restrict__ src,
                                                              u32x4* __restrict__ dst, int64_t n16) {
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n16;
       i += stride * kProbeUnroll) {
    u32x4 v[kProbeUnroll];
#pragma unroll
    for (int k = 0; k < kProbeUnroll; ++k) {
      const int64_t j = i + k * stride;
      v[k] = __builtin_nontemporal_load(&src[j < n16 ? j : n16 - 1]);
    }
#pragma unroll
    for (int k = 0; k < kProbeUnroll; ++k)
      if (i + k * stride < n16) __builtin_nontemporal_store(v[k], &dst[i + k * stride]);
  }
}

}  // namespace cmp

using namespace cmp;

extern "C" cmp_status cmp_bandwidth_probe(int32_t mode, const void* src, void* dst, size_t bytes,
                                          void* stream) {
  CMP_RANGE("cmp_bandwidth_probe");
  CMP_REQUIRE(mode == 0 || mode == 1, "mode %d: 0 read, 1 copy", mode);
  CMP_REQUIRE(src && dst && ((uintptr_t)src & 15) == 0 && ((uintptr_t)dst & 15) == 0,
              "src and dst must be 16-byte aligned device pointers");
  CMP_REQUIRE(bytes % 16 == 0, "bytes must be a multiple of 16");
  int dev = 0, cus = 0;
  CMP_CHECK_HIP(hipGetDevice(&dev));
  CMP_CHECK_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int64_t n16 = (int64_t)(bytes / 16);
  int64_t grid = (int64_t)cus * 32;
  const int64_t need = (n16 + kThreads * kProbeUnroll - 1) / (kThreads * kProbeUnroll);
  if (need < grid) grid = need > 0 ? need : 1;
  hipStream_t s = (hipStream_t)stream;
  if (mode == 0)
    hipLaunchKernelGGL(probe_read_kernel, dim3((unsigned)grid), dim3(kThreads), 0, s,
                       (const u32x4*)src, n16, (uint32_t*)dst);
  else
    hipLaunchKernelGGL(probe_copy_kernel, dim3((unsigned)grid), dim3(kThreads), 0, s,
                       (const u32x4*)src, (u32x4*)dst, n16);
  CMP_CHECK_HIP(hipGetLastError());
  return CMP_OK;
}
