// Barrett variant study (Sec. II-B): the classical reduction (Alg. 2), the
// Dhem-Quisquater instantiation alpha = N+3, beta = -2 (Alg. 3), the proposed
// alpha = N+1, beta = -2 (Alg. 4) and the built-in '%', on 32-bit words
// (moduli up to 30 bits; Alg. 3 up to 28) and on 64-bit words (up to 62 bits;
// Alg. 3 up to 60). Each reduction also reports how many correctional
// subtractions it took, so the device reproduces the correction statistics.
//
//   k_reduce_apply   c[i] = a[i]*b[i] mod q and a per-workgroup histogram of
//                    corrections (0, 1, 2) written to hist[block][3]
//   k_reduce_chain   throughput: each thread runs 8 independent chains of
//                    x <- reduce(x * y) for `iters` steps
//
// These kernels serve the study only; the hot path uses modarith.hpp.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pm_internal.hpp"

namespace pm {

enum { RV_MOD = 0, RV_ALG2 = 2, RV_ALG3 = 3, RV_ALG4 = 4 };

// ---------------------------------------------------------------- 32-bit --
template <int V>
__device__ __forceinline__ uint32_t red32(uint64_t x, const RedParams& P, uint32_t& corr) {
  const uint32_t q = (uint32_t)P.q, mu = (uint32_t)P.mu, m = P.m;
  if (V == RV_MOD) {
    corr = 0;
    return (uint32_t)(x % q);
  }
  uint32_t quot;
  if (V == RV_ALG2) {
    const uint32_t c = (uint32_t)(x >> (m - 1));
    quot = (uint32_t)(((uint64_t)c * mu) >> (m + 1));
  } else if (V == RV_ALG3) {
    const uint32_t c = (uint32_t)(x >> (m - 2));
    quot = (uint32_t)(((uint64_t)c * mu) >> (m + 5));
  } else {
    const uint32_t c = (uint32_t)(x >> (m - 2));
    quot = (uint32_t)(((uint64_t)c * mu) >> (m + 3));
  }
  uint32_t r = (uint32_t)x - quot * q;
  uint32_t k = 0;
  if (r >= q) { r -= q; ++k; }
  if (V == RV_ALG2 && r >= q) { r -= q; ++k; }
  corr = k;
  return r;
}

// ---------------------------------------------------------------- 64-bit --
typedef unsigned __int128 u128;

template <int V>
__device__ __forceinline__ uint64_t red64(u128 x, const RedParams& P, uint32_t& corr) {
  const uint64_t q = P.q, mu = P.mu;
  const uint32_t m = P.m;
  if (V == RV_MOD) {
    corr = 0;
    return (uint64_t)(x % q);
  }
  uint64_t quot;
  if (V == RV_ALG2) quot = (uint64_t)((((u128)(uint64_t)(x >> (m - 1))) * mu) >> (m + 1));
  else if (V == RV_ALG3) quot = (uint64_t)((((u128)(uint64_t)(x >> (m - 2))) * mu) >> (m + 5));
  else quot = (uint64_t)((((u128)(uint64_t)(x >> (m - 2))) * mu) >> (m + 3));
  uint64_t r = (uint64_t)x - quot * q;
  uint32_t k = 0;
  if (r >= q) { r -= q; ++k; }
  if (V == RV_ALG2 && r >= q) { r -= q; ++k; }
  corr = k;
  return r;
}

template <int V, int W>
__global__ void __launch_bounds__(256) k_reduce_apply(const uint64_t* __restrict__ a, const uint64_t* __restrict__ b,
                                                      uint64_t* __restrict__ c, uint32_t* __restrict__ hist, size_t n,
                                                      RedParams P) {
  __shared__ uint32_t h[3];
  if (threadIdx.x < 3) h[threadIdx.x] = 0;
  __syncthreads();
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    uint32_t k;
    uint64_t r;
    if (W == 32) r = red32<V>((uint64_t)a[i] * b[i], P, k);
    else r = red64<V>((u128)a[i] * b[i], P, k);
    c[i] = r;
    atomicAdd(&h[k], 1u);
  }
  __syncthreads();
  if (threadIdx.x < 3) hist[(size_t)blockIdx.x * 3 + threadIdx.x] = h[threadIdx.x];
}

template <int V, int W>
__global__ void __launch_bounds__(256) k_reduce_chain(uint64_t* __restrict__ out, uint64_t y, int iters, RedParams P) {
  uint64_t acc[8];
  const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
#pragma unroll
  for (int j = 0; j < 8; ++j) acc[j] = (tid * 8 + j + 1) % P.q;
  uint32_t k = 0;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      uint32_t kk;
      if (W == 32) acc[j] = red32<V>((uint64_t)acc[j] * y, P, kk);
      else acc[j] = red64<V>((u128)acc[j] * y, P, kk);
      k += kk;
    }
  }
  uint64_t r = k;
#pragma unroll
  for (int j = 0; j < 8; ++j) r ^= acc[j];
  out[tid] = r;
}

#define PM_RED_DISPATCH(KERNEL, V, W, ...)                                                                  \
  do {                                                                                                    \
    if (W == 32) {                                                                                        \
      if (V == RV_MOD) hipLaunchKernelGGL((KERNEL<RV_MOD, 32>), __VA_ARGS__);                             \
      else if (V == RV_ALG2) hipLaunchKernelGGL((KERNEL<RV_ALG2, 32>), __VA_ARGS__);                      \
      else if (V == RV_ALG3) hipLaunchKernelGGL((KERNEL<RV_ALG3, 32>), __VA_ARGS__);                      \
      else hipLaunchKernelGGL((KERNEL<RV_ALG4, 32>), __VA_ARGS__);                                        \
    } else {                                                                                              \
      if (V == RV_MOD) hipLaunchKernelGGL((KERNEL<RV_MOD, 64>), __VA_ARGS__);                             \
      else if (V == RV_ALG2) hipLaunchKernelGGL((KERNEL<RV_ALG2, 64>), __VA_ARGS__);                      \
      else if (V == RV_ALG3) hipLaunchKernelGGL((KERNEL<RV_ALG3, 64>), __VA_ARGS__);                      \
      else hipLaunchKernelGGL((KERNEL<RV_ALG4, 64>), __VA_ARGS__);                                        \
    }                                                                                                     \
  } while (0)

hipError_t launch_reduce_apply(int variant, int word_bits, const uint64_t* a, const uint64_t* b, uint64_t* c,
                               uint32_t* hist, size_t n, const RedParams& P, hipStream_t s) {
  const dim3 grid((uint32_t)((n + 255) / 256));
  PM_RED_DISPATCH(k_reduce_apply, variant, word_bits, grid, dim3(256), 0, s, a, b, c, hist, n, P);
  return hipGetLastError();
}

hipError_t launch_reduce_chain(int variant, int word_bits, uint64_t* out, size_t threads, uint64_t y, int iters,
                               const RedParams& P, hipStream_t s) {
  const dim3 grid((uint32_t)(threads / 256));
  PM_RED_DISPATCH(k_reduce_chain, variant, word_bits, grid, dim3(256), 0, s, out, y, iters, P);
  return hipGetLastError();
}

}  // namespace pm
