// Plain streaming copy: the bandwidth reference the decode kernel's HBM
// traffic and throughput are compared against.
#include "mjd_internal.h"

namespace mjd {

__global__ __launch_bounds__(256) void copy16(v4i* __restrict__ dst, const v4i* __restrict__ src, size_t n) {
  const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
  for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
    __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t stream) {
  const size_t n = bytes / 16;
  size_t blocks = (n + 255) / 256;
  if (blocks > 256 * 64) blocks = 256 * 64;  // grid-stride beyond 64 workgroups per CU
  hipLaunchKernelGGL(copy16, dim3(static_cast<uint32_t>(blocks)), dim3(256), 0, stream,
                     static_cast<v4i*>(dst), static_cast<const v4i*>(src), n);
  return hipGetLastError();
}

}  // namespace mjd
