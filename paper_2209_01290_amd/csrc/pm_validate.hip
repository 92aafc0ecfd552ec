// Input validation behind PM_VALIDATE=1: a device scan that flags, per limb,
// whether any word of the limb's span is not canonical (>= its modulus).
// grid: x = blocks over the limb's words (grid-stride), y = limb. A block
// ORs its threads' findings with a barrier reduction and, only if it found a
// word >= q, writes 1 to flags[limb] (flags are cleared by the caller).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pm_internal.hpp"

namespace pm {

template <typename W>
__global__ void __launch_bounds__(256)
k_canon(const W* __restrict__ x, size_t per_limb, const uint64_t* __restrict__ qs, uint32_t* __restrict__ flags) {
  const uint32_t limb = blockIdx.y;
  const W q = (W)qs[limb];
  const W* base = x + (size_t)limb * per_limb;
  int bad = 0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < per_limb; i += (size_t)gridDim.x * blockDim.x)
    bad |= base[i] >= q;
  bad = __syncthreads_or(bad);
  if (bad && threadIdx.x == 0) flags[limb] = 1u;
}

hipError_t launch_canon(const void* x, int word_bytes, size_t per_limb, uint32_t limbs, const uint64_t* qs_dev,
                        uint32_t* flags_dev, hipStream_t s) {
  const size_t blocks = (per_limb + 255) / 256;
  dim3 grid((uint32_t)(blocks < 1024 ? (blocks ? blocks : 1) : 1024), limbs);
  if (word_bytes == 8)
    hipLaunchKernelGGL(k_canon<uint64_t>, grid, dim3(256), 0, s, (const uint64_t*)x, per_limb, qs_dev, flags_dev);
  else
    hipLaunchKernelGGL(k_canon<uint32_t>, grid, dim3(256), 0, s, (const uint32_t*)x, per_limb, qs_dev, flags_dev);
  return hipGetLastError();
}

}  // namespace pm
