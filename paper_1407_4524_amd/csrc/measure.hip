// Measurement kernels: a plain device copy, hand-written, whose achieved
// bandwidth is the copy ceiling the stream-collide kernel is set against, and
// whose bytes (known exactly) calibrate the HBM traffic counters.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "domain.hpp"
#include "lbm.h"

namespace lbm {

// U 16-byte vectors per thread, each load/store instruction of a wavefront
// covering 1 KiB of consecutive bytes; all U loads issued before any store.
template <int U, bool NT>
__global__ __launch_bounds__(256) void k_copy(const float4* __restrict__ src, float4* __restrict__ dst, int64_t n) {
  const int64_t base = (int64_t)blockIdx.x * (256 * U) + threadIdx.x;
  float4 v[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t k = base + (int64_t)u * 256;
    const int64_t kk = k < n ? k : 0;
    if constexpr (NT) {
      v[u].x = __builtin_nontemporal_load(&src[kk].x);
      v[u].y = __builtin_nontemporal_load(&src[kk].y);
      v[u].z = __builtin_nontemporal_load(&src[kk].z);
      v[u].w = __builtin_nontemporal_load(&src[kk].w);
    } else {
      v[u] = src[kk];
    }
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t k = base + (int64_t)u * 256;
    if (k >= n) break;
    if constexpr (NT) {
      __builtin_nontemporal_store(v[u].x, &dst[k].x);
      __builtin_nontemporal_store(v[u].y, &dst[k].y);
      __builtin_nontemporal_store(v[u].z, &dst[k].z);
      __builtin_nontemporal_store(v[u].w, &dst[k].w);
    } else {
      dst[k] = v[u];
    }
  }
}

// the same with a fixed grid of `blocks` workgroups striding over the array
template <int U>
__global__ __launch_bounds__(256) void k_copy_stride(const float4* __restrict__ src, float4* __restrict__ dst,
                                                     int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * (256 * U);
  for (int64_t base = (int64_t)blockIdx.x * (256 * U) + threadIdx.x; base < n; base += stride) {
    float4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t k = base + (int64_t)u * 256;
      v[u] = src[k < n ? k : 0];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t k = base + (int64_t)u * 256;
      if (k < n) dst[k] = v[u];
    }
  }
}

}  // namespace lbm

extern "C" lbm_status lbm_copy(const void* src, void* dst, size_t bytes, int32_t variant, void* stream) {
  using namespace lbm;
  if (!src || !dst) return host::fail(LBM_E_INVAL, "null buffer");
  if (bytes == 0) return LBM_OK;
  if (bytes % 16 != 0 || ((uintptr_t)src | (uintptr_t)dst) % 16 != 0)
    return host::fail(LBM_E_INVAL, "copy size and addresses must be multiples of 16 bytes");
  const int64_t n = (int64_t)(bytes / 16);
  hipStream_t s = (hipStream_t)stream;
  auto grid = [&](int u) { return dim3((unsigned)((n + 256 * u - 1) / (256 * u))); };
  switch (variant) {
    case 0: hipLaunchKernelGGL((k_copy<1, false>), grid(1), dim3(256), 0, s, (const float4*)src, (float4*)dst, n); break;
    case 1: hipLaunchKernelGGL((k_copy<2, false>), grid(2), dim3(256), 0, s, (const float4*)src, (float4*)dst, n); break;
    case 2: hipLaunchKernelGGL((k_copy<4, false>), grid(4), dim3(256), 0, s, (const float4*)src, (float4*)dst, n); break;
    case 3: hipLaunchKernelGGL((k_copy<4, true>), grid(4), dim3(256), 0, s, (const float4*)src, (float4*)dst, n); break;
    case 4: hipLaunchKernelGGL((k_copy_stride<4>), dim3(2048), dim3(256), 0, s, (const float4*)src, (float4*)dst, n); break;
    case 5: hipLaunchKernelGGL((k_copy_stride<2>), dim3(4096), dim3(256), 0, s, (const float4*)src, (float4*)dst, n); break;
    default: return host::fail(LBM_E_INVAL, "unknown copy variant");
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return host::fail(LBM_E_HIP, std::string("copy launch: ") + hipGetErrorString(e));
  return LBM_OK;
}
