// Modular arithmetic on 32-bit words (moduli of up to 30 bits), the word
// size of the paper's 30-bit NTT timings (Sec. VII, comparison table) and of Alg. 4 with
// beta = 32: m = len(q) <= beta - 2 = 30, mu = floor(2^(2m+1)/q) < 2^32.
//
//   x = a*b is one 32x32->64 multiply; c = x >> (m-2) is one funnel shift
//   (c < 2^(m+2) <= 2^32); quot = (c*mu) >> (m+3) is the high word of
//   c*mu' with mu' = mu << (29-m) for m <= 29 (the same integer, as for
//   64-bit words), and the high word shifted once more for m = 30;
//   r = x - quot*q in 32 bits (Alg. 4: r < 2q < 2^31); the correction is
//   min(r, r - q) as unsigned words (r - q wraps above r exactly when r < q).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pm {

struct Mod32 {
  uint32_t q;      // odd modulus, len(q) = m <= 30
  uint32_t mu;     // mu' as above
  uint32_t half;   // (q + 1) / 2
  uint32_t s;      // m - 2
  uint32_t t;      // 1 if m == 30, else 0
  uint32_t pad;
};
static_assert(sizeof(Mod32) == 24, "Mod32 layout");

__device__ __forceinline__ uint32_t addmod(uint32_t a, uint32_t b, uint32_t q) {
  const uint32_t s = a + b;            // < 2q < 2^31
  return min(s, s - q);
}

__device__ __forceinline__ uint32_t submod(uint32_t a, uint32_t b, uint32_t q) {
  const uint32_t d = a - b;
  return min(d, d + q);
}

__device__ __forceinline__ uint32_t halfmod(uint32_t x, uint32_t half) {
  return (x >> 1) + ((x & 1) ? half : 0u);
}

template <int KIND>
__device__ __forceinline__ uint32_t mulmod(uint32_t a, uint32_t b, const Mod32& M) {
  const uint64_t x = (uint64_t)a * b;
  const uint32_t c = __builtin_amdgcn_alignbit((uint32_t)(x >> 32), (uint32_t)x, M.s);
  uint32_t quot = __umulhi(c, M.mu);
  if (KIND != 0) quot >>= M.t;         // KIND_WIDE (0): every modulus has m <= 29
  const uint32_t r = (uint32_t)x - quot * M.q;
  return min(r, r - M.q);
}

template <int KIND>
__device__ __forceinline__ void ct_bfly(uint32_t& u, uint32_t& v, uint32_t xi, const Mod32& M) {
  const uint32_t w = mulmod<KIND>(v, xi, M);
  const uint32_t s = addmod(u, w, M.q);
  v = submod(u, w, M.q);
  u = s;
}

template <int KIND>
__device__ __forceinline__ void gs_bfly_half(uint32_t& u, uint32_t& v, uint32_t xi, const Mod32& M) {
  const uint32_t s = addmod(u, v, M.q);
  const uint32_t d = submod(u, v, M.q);
  u = halfmod(s, M.half);
  v = mulmod<KIND>(halfmod(d, M.half), xi, M);
}

// xi/2 mod q, for gs_bfly_htw.
__device__ __forceinline__ uint32_t half_tw(uint32_t xi, const Mod32& M) { return halfmod(xi, M.half); }

// gs_bfly_half with the twiddle halved beforehand (xh = xi/2 mod q):
// (u, v) -> ((u+v)/2, (u-v) xh); in Z_q, (u-v) xh = xi (u-v)/2.
template <int KIND>
__device__ __forceinline__ void gs_bfly_htw(uint32_t& u, uint32_t& v, uint32_t xh, const Mod32& M) {
  const uint32_t s = addmod(u, v, M.q);
  const uint32_t d = submod(u, v, M.q);
  u = halfmod(s, M.half);
  v = mulmod<KIND>(d, xh, M);
}

}  // namespace pm
