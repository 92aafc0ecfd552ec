// Word-level modular arithmetic on 64-bit words for gfx950 (CDNA4).
//
// Every routine takes canonical operands in [0, q) and returns a canonical
// result; q is odd with bit length m = len(q) <= 62. 64-bit products are
// assembled from 32x32->64 multiplies (v_mad_u64_u32, v_mul_hi_u32); the VALU
// has no 64-bit multiplier. On gfx950 these multiplies issue at (close to)
// full rate, so the cost of a routine is its instruction count.
//
//   addmod   modular addition with one correctional subtraction (Alg. 1)
//   submod   a - b, plus q on borrow (the difference of the GS butterfly)
//   halfmod  x/2 mod q = (x >> 1) + (x & 1) * ((q + 1) >> 1); it merges the
//            1/N scaling into the GS butterflies (Sec. III-A, Eq. 2)
//   mulmod   a*b mod q by the proposed Barrett reduction (Alg. 4):
//            m = len(q), mu = floor(2^(2m+1) / q), c = x >> (m-2),
//            quot = (c*mu) >> (m+3), r = x - quot*q, at most one r -= q.
//
// How the steps of Alg. 4 map onto 32-bit operations:
//   * x = a*b is formed from four partial products; the two cross products
//     are summed in one multiply-add (a, b < 2^62 keeps the sum below 2^63).
//   * c = x >> (m-2) is a funnel shift (v_alignbit_b32) over three 32-bit
//     words of x: words 1..3 with shift m-34 when m >= 34, else words 0..2
//     with shift m-2.
//   * quot = (c*mu) >> (m+3) is taken as the high 64 bits of c*mu', where the
//     host stores mu' = mu << (61-m) for m <= 61. It is the same integer:
//     c*mu*2^(61-m) / 2^64 = c*mu / 2^(m+3). For m = 62 the host stores
//     mu' = mu and the high word is shifted right once more.
//   * r = x - quot*q is formed modulo 2^64 as x + quot*(2^64 - q); Alg. 4
//     guarantees 0 <= r < 2q, so one subtraction of q, kept unless it
//     borrows, makes r canonical.
//
// Two instantiations:
//   KIND_WIDE  every modulus of the launch has 34 <= m <= 61 (all 60-bit NTT
//              primes); the cross sums of c*mu' then fit 64 bits.
//   KIND_ANY   any 2 <= m <= 62: window and final shift chosen per modulus,
//              carries of c*mu' kept explicitly.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pm {

// Per-modulus constants, computed on the host (pm_params.cpp).
struct Mod {
  uint64_t q;      // odd modulus, len(q) = m <= 62
  uint64_t mu;     // mu' as described above
  uint64_t half;   // (q + 1) / 2
  uint32_t s1;     // funnel shift for c: m-34 if m >= 34, else m-2
  uint16_t wide;   // 1 if the c window is words 1..3 (m >= 34)
  uint16_t t;      // extra right shift of hi64(c*mu'): 1 if m == 62
};
static_assert(sizeof(Mod) == 32, "Mod layout");

enum { KIND_WIDE = 0, KIND_ANY = 1 };

__device__ __forceinline__ uint32_t lo32(uint64_t x) { return (uint32_t)x; }
__device__ __forceinline__ uint32_t hi32(uint64_t x) { return (uint32_t)(x >> 32); }

__device__ __forceinline__ uint64_t pack64(uint32_t lo, uint32_t hi) { return ((uint64_t)hi << 32) | lo; }

// The single correctional subtraction: s - q unless that borrows (s < q).
// The select reads the borrow of the 64-bit subtraction itself, so no
// separate comparison is issued.
__device__ __forceinline__ uint64_t csub(uint64_t s, uint64_t q) {
  unsigned b0, b1;
  const uint32_t d0 = __builtin_subc(lo32(s), lo32(q), 0u, &b0);
  const uint32_t d1 = __builtin_subc(hi32(s), hi32(q), b0, &b1);
  return b1 ? s : pack64(d0, d1);
}

// (a + b) mod q (Alg. 1): a + b < 2q, one correctional subtraction.
__device__ __forceinline__ uint64_t addmod(uint64_t a, uint64_t b, uint64_t q) {
  return csub(a + b, q);
}

// (a - b) mod q: plus q when the subtraction borrows (a < b).
__device__ __forceinline__ uint64_t submod(uint64_t a, uint64_t b, uint64_t q) {
  unsigned b0, b1;
  const uint32_t d0 = __builtin_subc(lo32(a), lo32(b), 0u, &b0);
  const uint32_t d1 = __builtin_subc(hi32(a), hi32(b), b0, &b1);
  const uint64_t d = pack64(d0, d1);
  return b1 ? d + q : d;
}

// x/2 mod q for x in [0, q), q odd.
__device__ __forceinline__ uint64_t halfmod(uint64_t x, uint64_t half) {
  return (x >> 1) + ((x & 1) ? half : 0);
}

template <int KIND>
__device__ __forceinline__ uint64_t mulmod(uint64_t a, uint64_t b, const Mod& M) {
  const uint32_t a0 = lo32(a), a1 = hi32(a), b0 = lo32(b), b1 = hi32(b);
  // x = a*b = P00 + mid*2^32 + P11*2^64 as words x0..x3
  const uint64_t P00 = (uint64_t)a0 * b0;
  const uint64_t mid = (uint64_t)a1 * b0 + (uint64_t)a0 * b1;
  const uint64_t P11 = (uint64_t)a1 * b1;
  unsigned cy1, cy2;
  const uint32_t x0 = lo32(P00);
  const uint32_t x1 = __builtin_addc(hi32(P00), lo32(mid), 0u, &cy1);
  const uint32_t x2 = __builtin_addc(lo32(P11), hi32(mid), cy1, &cy2);
  const uint32_t x3 = hi32(P11) + cy2;

  // c = x >> (m-2)
  uint32_t y0 = x1, y1 = x2, y2 = x3;
  if (KIND != KIND_WIDE && !M.wide) { y0 = x0; y1 = x1; y2 = x2; }
  const uint32_t c0 = __builtin_amdgcn_alignbit(y1, y0, M.s1);
  const uint32_t c1 = __builtin_amdgcn_alignbit(y2, y1, M.s1);

  // quot = (c*mu) >> (m+3) = hi64(c*mu') [>> 1 when m == 62]
  const uint32_t m0 = lo32(M.mu), m1 = hi32(M.mu);
  uint64_t quot;
  if (KIND == KIND_WIDE) {
    const uint64_t e = (uint64_t)c0 * m1 + (uint64_t)__umulhi(c0, m0);
    const uint64_t f = (uint64_t)c1 * m0 + e;          // < 2^64: c1, m1 < 2^31
    quot = (uint64_t)c1 * m1 + hi32(f);
  } else {
    const uint64_t e = (uint64_t)c0 * m1 + (uint64_t)__umulhi(c0, m0);
    const uint64_t f = (uint64_t)c1 * m0 + lo32(e);
    quot = (uint64_t)c1 * m1 + ((uint64_t)hi32(e) + hi32(f));
    quot >>= M.t;
  }

  // r = x - quot*q  (mod 2^64), then at most one correctional subtraction.
  // The cross products of quot*(2^64 - q) only reach the high word: they are
  // summed in 32 bits and added to it directly.
  const uint64_t nq = 0 - M.q;
  const uint32_t k0 = lo32(quot), k1 = hi32(quot);
  const uint64_t r0 = (uint64_t)k0 * lo32(nq) + (((uint64_t)x1 << 32) | x0);
  const uint32_t cross = lo32((uint64_t)k1 * lo32(nq) + (uint32_t)(k0 * hi32(nq)));
  return csub(pack64(lo32(r0), hi32(r0) + cross), M.q);
}

// CT butterfly of the merged forward NTT (Alg. 5):
//   (u, v) -> (u + xi*v, u - xi*v) mod q
template <int KIND>
__device__ __forceinline__ void ct_bfly(uint64_t& u, uint64_t& v, uint64_t xi, const Mod& M) {
  const uint64_t w = mulmod<KIND>(v, xi, M);
  const uint64_t s = addmod(u, w, M.q);
  v = submod(u, w, M.q);
  u = s;
}

// GS butterfly of the merged inverse NTT (Alg. 6) with both outputs halved
// (Eq. 2): (u, v) -> ((u+v)/2, xi*(u-v)/2) mod q. The difference is halved
// before the product; in Z_q the order of the two factors is immaterial.
template <int KIND>
__device__ __forceinline__ void gs_bfly_half(uint64_t& u, uint64_t& v, uint64_t xi, const Mod& M) {
  const uint64_t s = addmod(u, v, M.q);
  const uint64_t d = submod(u, v, M.q);
  u = halfmod(s, M.half);
  v = mulmod<KIND>(halfmod(d, M.half), xi, M);
}

// xi/2 mod q, for gs_bfly_htw.
__device__ __forceinline__ uint64_t half_tw(uint64_t xi, const Mod& M) { return halfmod(xi, M.half); }

// gs_bfly_half with the twiddle halved beforehand (xh = xi/2 mod q):
// (u, v) -> ((u+v)/2, (u-v) xh); in Z_q, (u-v) xh = xi (u-v)/2. Where one
// twiddle serves several butterflies, its halving is paid once instead of
// once per butterfly.
template <int KIND>
__device__ __forceinline__ void gs_bfly_htw(uint64_t& u, uint64_t& v, uint64_t xh, const Mod& M) {
  const uint64_t s = addmod(u, v, M.q);
  const uint64_t d = submod(u, v, M.q);
  u = halfmod(s, M.half);
  v = mulmod<KIND>(d, xh, M);
}

// Unhalved GS butterfly (Alg. 6 as printed): (u, v) -> (u+v, xi*(u-v)).
template <int KIND>
__device__ __forceinline__ void gs_bfly(uint64_t& u, uint64_t& v, uint64_t xi, const Mod& M) {
  const uint64_t s = addmod(u, v, M.q);
  const uint64_t d = submod(u, v, M.q);
  u = s;
  v = mulmod<KIND>(d, xi, M);
}

}  // namespace pm
