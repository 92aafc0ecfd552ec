// Device building blocks of the merged NTTs (Alg. 5 and Alg. 6) on gfx950.
//
// Decomposition. A polynomial of N = R*C coefficients is viewed as an R x C
// row-major matrix (R = 2^s rows, C = 2^c columns). Unrolling the loops of
// Alg. 5 shows that a butterfly at stride k pairs j and j+k inside group
// i = j / (2k) of stage m = N / (2k), with twiddle psi_br[m + i]:
//   * strides k >= C (the first s stages) pair rows of one column; every
//     column runs the same R-point merged NTT with twiddles psi_br[1..R);
//   * strides k < C (the last c stages) stay inside one row r; with
//     mm = C / (2k) groups per row the twiddle index is (R + r)*mm + i_row,
//     i_row = (column index) / (2k).
// Alg. 6 has the same (m, k, i) structure, run in the opposite stage order,
// so the inverse uses the same indices on psi_inv_br. No transposition and no
// extra twiddle table is needed. R = 1 is the single-pass case.
//
// Row pass. A row of C = 2^c words is held by T = C/16 threads, 16 words per
// thread in registers. The c stages are taken in rounds of four from the top
// (largest stride first): a round whose butterfly bits are [p, p+4) gives
// each thread the 16 words whose index bits [p, p+4) vary, so the round's
// four stages are radix-16 in registers. Rounds exchange data through LDS.
// The last round always holds bits [0, 4) (16 consecutive words per thread);
// when c is not a multiple of 4 it runs only the remaining c mod 4 stages.
//
// Column pass. One thread per column holds the R = 2^s words of that column
// in registers and runs the s column stages; twiddles are uniform per launch.
#pragma once
#include "modarith.hpp"
#include "modarith32.hpp"

namespace pm {

template <int LOGC>
struct RowGeom {
  static constexpr int EB = LOGC < 4 ? LOGC : 4;      // log2(words per thread)
  static constexpr int E = 1 << EB;
  static constexpr int LOGT = LOGC - EB;
  static constexpr int T = 1 << LOGT;                  // threads per row
  static constexpr int NR = LOGC <= 4 ? 1 : (LOGC + 3) / 4;   // rounds
  static constexpr int WG = T < 256 ? 256 : T;         // threads per workgroup
  static constexpr int ROWS = WG / T;                  // rows per workgroup
  static constexpr int LDS_ROW = (1 << LOGC) + ((1 << LOGC) >> 4);  // padded words
  static constexpr int LDS_WORDS = NR > 1 ? ROWS * LDS_ROW : 1;
  // register-bit base p and butterfly bits [lo, hi) of round rho (forward order)
  static constexpr int hi(int rho) { return LOGC - 4 * rho; }
  static constexpr int lo(int rho) { return hi(rho) - 4 > 0 ? hi(rho) - 4 : 0; }
  static constexpr int p(int rho) { return rho == NR - 1 ? 0 : hi(rho) - 4; }
};

// Index inside the row of register j of thread t when the register bits are [p, p+EB).
template <int P, int EB>
__device__ __forceinline__ uint32_t reg_index(uint32_t t, uint32_t j) {
  return ((t >> P) << (P + EB)) | (j << P) | (t & ((1u << P) - 1u));
}

// Scheduling fence between stages: stops the compiler from hoisting the
// twiddle loads and butterflies of later stages, which bounds register use.
#ifndef PM_STAGE_FENCE
#define PM_STAGE_FENCE 1
#endif
__device__ __forceinline__ void stage_fence() {
#if PM_STAGE_FENCE
  __builtin_amdgcn_sched_barrier(0);
#endif
}

// LDS slot of row word idx is idx + idx/16: one pad word per 16 keeps strided
// 64-bit accesses spread over the banks. With idx = th*2^(P+4) + j*2^P + tl
// (tl < 2^P) the slot splits into a per-thread base plus a per-register
// constant, so every LDS access is one instruction with an immediate offset:
//   slot = [th*(2^(P+4) + 2^P) + tl + tl/16] + [j*2^P + (j*2^P)/16]
// (for P < 4, tl/16 = 0 and (j*2^P + tl)/16 = (j*2^P)/16 since tl < 2^P).
template <int P>
__device__ __forceinline__ uint32_t lds_base(uint32_t t) {
  const uint32_t th = t >> P, tl = t & ((1u << P) - 1u);
  return th * ((16u << P) + (1u << P)) + tl + (tl >> 4);
}
template <int P>
__device__ __forceinline__ constexpr uint32_t lds_off(uint32_t j) {
  return (j << P) + ((j << P) >> 4);
}
// Row offset of register j: per-thread base plus a per-register constant.
template <int P>
__device__ __forceinline__ uint32_t row_base(uint32_t t) {
  return ((t >> P) << (P + 4)) | (t & ((1u << P) - 1u));
}

// Forward (CT) stages of round RHO on registers x. tw = psi_br of this limb,
// Rr = R + r for row r of an R-row split.
// TRUNC drops the stride-1 stage (the last of Alg. 5): the truncated CT NTT
// of the fused product (Sec. III-B).
template <int LOGC, int RHO, int KIND, bool TRUNC = false, typename W, typename MT>
__device__ __forceinline__ void fwd_round(W (&x)[RowGeom<LOGC>::E], uint32_t t, const W* __restrict__ tw,
                                          uint32_t Rr, const MT& M) {
  using G = RowGeom<LOGC>;
  constexpr int P = G::p(RHO), HI = G::hi(RHO), LO = (TRUNC && G::lo(RHO) == 0) ? 1 : G::lo(RHO), EB = G::EB;
  const uint32_t th = t >> P;
#pragma unroll
  for (int b = HI - 1; b >= LO; --b) {
    const int jb = b - P;                          // register bit paired at this stage
    const uint32_t mm = 1u << (LOGC - b - 1);      // groups per row at this stage
    const uint32_t base = Rr * mm + (th << (P + EB - b - 1));
#pragma unroll
    for (int g = 0; g < (G::E >> (jb + 1)); ++g) {
      const W xi = tw[base + g];
#pragma unroll
      for (int s = 0; s < (1 << jb); ++s) {
        const int j = (g << (jb + 1)) | s;
        ct_bfly<KIND>(x[j], x[j | (1 << jb)], xi, M);
      }
    }
    stage_fence();
  }
}

// Inverse (GS, halved) stages of round RHO, smallest stride first. TRUNC drops
// the stride-1 stage (the first of Alg. 6): the truncated GS NTT of the fused
// product, whose first stage and its 1/2 are folded into Alg. 7.
template <int LOGC, int RHO, int KIND, bool TRUNC = false, typename W, typename MT>
__device__ __forceinline__ void inv_round(W (&x)[RowGeom<LOGC>::E], uint32_t t, const W* __restrict__ tw,
                                          uint32_t Rr, const MT& M) {
  using G = RowGeom<LOGC>;
  constexpr int P = G::p(RHO), HI = G::hi(RHO), LO = (TRUNC && G::lo(RHO) == 0) ? 1 : G::lo(RHO), EB = G::EB;
  const uint32_t th = t >> P;
#pragma unroll
  for (int b = LO; b < HI; ++b) {
    const int jb = b - P;
    const uint32_t mm = 1u << (LOGC - b - 1);
    const uint32_t base = Rr * mm + (th << (P + EB - b - 1));
#pragma unroll
    for (int g = 0; g < (G::E >> (jb + 1)); ++g) {
      const W xi = tw[base + g];
#pragma unroll
      for (int s = 0; s < (1 << jb); ++s) {
        const int j = (g << (jb + 1)) | s;
        gs_bfly_half<KIND>(x[j], x[j | (1 << jb)], xi, M);
      }
    }
    stage_fence();
  }
}

// LDS and global accesses below only run for rows with at least two rounds
// (LOGC > 4), where every round's register bits are 4 wide (EB = 4); for
// LOGC <= 4 the single round has P = 0 and EB = LOGC, and the same formulas
// hold with 2^(P+4) replaced by 2^EB, which row_base/lds_base never need
// because th = 0 there (one thread per row).
template <int LOGC, int RHO, typename W>
__device__ __forceinline__ void lds_put(W* lds, const W (&x)[RowGeom<LOGC>::E], uint32_t t) {
  using G = RowGeom<LOGC>;
  constexpr int P = G::p(RHO);
  W* b = lds + lds_base<P>(t);
#pragma unroll
  for (int j = 0; j < G::E; ++j) b[lds_off<P>(j)] = x[j];
}

template <int LOGC, int RHO, typename W>
__device__ __forceinline__ void lds_get(const W* lds, W (&x)[RowGeom<LOGC>::E], uint32_t t) {
  using G = RowGeom<LOGC>;
  constexpr int P = G::p(RHO);
  const W* b = lds + lds_base<P>(t);
#pragma unroll
  for (int j = 0; j < G::E; ++j) x[j] = b[lds_off<P>(j)];
}

template <int LOGC, int RHO, typename W>
__device__ __forceinline__ void gmem_get(const W* __restrict__ row, W (&x)[RowGeom<LOGC>::E], uint32_t t) {
  using G = RowGeom<LOGC>;
  constexpr int P = G::p(RHO);
  const uint32_t tb = (G::NR > 1) ? row_base<P>(t) : (t << G::EB);
#pragma unroll
  for (int j = 0; j < G::E; ++j) x[j] = (row + (j << P))[tb];
}

template <int LOGC, int RHO, typename W>
__device__ __forceinline__ void gmem_put(W* __restrict__ row, const W (&x)[RowGeom<LOGC>::E], uint32_t t) {
  using G = RowGeom<LOGC>;
  constexpr int P = G::p(RHO);
  const uint32_t tb = (G::NR > 1) ? row_base<P>(t) : (t << G::EB);
#pragma unroll
  for (int j = 0; j < G::E; ++j) (row + (j << P))[tb] = x[j];
}

// Move registers from round FROM's layout to round TO's layout through LDS.
// All threads of the workgroup must call it (it holds two barriers).
template <int LOGC, int FROM, int TO, typename W>
__device__ __forceinline__ void exchange(W* lds, W (&x)[RowGeom<LOGC>::E], uint32_t t) {
  __syncthreads();
  lds_put<LOGC, FROM>(lds, x, t);
  __syncthreads();
  lds_get<LOGC, TO>(lds, x, t);
}

// All row stages of the forward transform: rounds 0..NR-1. On return x holds
// the row in the last round's layout (16 consecutive words per thread).
template <int LOGC, int KIND, int RHO = 0, bool TRUNC = false, typename W, typename MT>
__device__ __forceinline__ void fwd_rounds(W* lds, W (&x)[RowGeom<LOGC>::E], uint32_t t, const W* __restrict__ tw,
                                           uint32_t Rr, const MT& M) {
  fwd_round<LOGC, RHO, KIND, TRUNC>(x, t, tw, Rr, M);
  if constexpr (RHO + 1 < RowGeom<LOGC>::NR) {
    exchange<LOGC, RHO, RHO + 1>(lds, x, t);
    fwd_rounds<LOGC, KIND, RHO + 1, TRUNC>(lds, x, t, tw, Rr, M);
  }
}

// All row stages of the inverse transform, from the last round's layout back
// to round 0's layout.
template <int LOGC, int KIND, int RHO = RowGeom<LOGC>::NR - 1, bool TRUNC = false, typename W, typename MT>
__device__ __forceinline__ void inv_rounds(W* lds, W (&x)[RowGeom<LOGC>::E], uint32_t t, const W* __restrict__ tw,
                                           uint32_t Rr, const MT& M) {
  inv_round<LOGC, RHO, KIND, TRUNC>(x, t, tw, Rr, M);
  if constexpr (RHO > 0) {
    exchange<LOGC, RHO, RHO - 1>(lds, x, t);
    inv_rounds<LOGC, KIND, RHO - 1, TRUNC>(lds, x, t, tw, Rr, M);
  }
}

// Alg. 7 on the 8 adjacent pairs (2i, 2i+1) of a thread's 16 consecutive words
// (last-round layout): with u = a0 b0, v = a1 b1, w = (a0+a1)(b0+b1),
//   c1 = w - u - v,  c0 = u + alpha^2 v,
// alpha^2 = (-1)^i psi_br[N/4 + i/2] (Alg. 8): the square of the stride-1
// twiddle is the stride-2 twiddle of the same word, index (R+r)*C/4 + idx/4,
// and the sign is fixed per register because 16t and r*C are multiples of 4.
// Needs C >= 4. Results overwrite x.
template <int LOGC, typename W>
struct FusedTw {
  W v[RowGeom<LOGC>::E / 4 > 0 ? RowGeom<LOGC>::E / 4 : 1];
};

// The alpha^2 twiddles of a thread's pairs, loaded ahead of use.
template <int LOGC, typename W>
__device__ __forceinline__ FusedTw<LOGC, W> fused_twiddles(uint32_t t, const W* __restrict__ tw, uint32_t Rr) {
  using G = RowGeom<LOGC>;
  static_assert(LOGC >= 2, "the fused product needs rows of at least 4 words");
  FusedTw<LOGC, W> f;
  const uint32_t base = Rr * (1u << (LOGC - 2)) + (t << (G::EB - 2));
#pragma unroll
  for (int g = 0; g < G::E / 4; ++g) f.v[g] = tw[base + g];
  return f;
}

template <int LOGC, int KIND, typename W, typename MT>
__device__ __forceinline__ void fused_hadamard(W (&x)[RowGeom<LOGC>::E], const W (&y)[RowGeom<LOGC>::E],
                                               const FusedTw<LOGC, W>& f, const MT& M) {
  using G = RowGeom<LOGC>;
#pragma unroll
  for (int j = 0; j < G::E; j += 2) {
    const W xi = f.v[j >> 2];
    const W u = mulmod<KIND>(x[j], y[j], M);
    const W v = mulmod<KIND>(x[j + 1], y[j + 1], M);
    const W w = mulmod<KIND>(addmod(x[j], x[j + 1], M.q), addmod(y[j], y[j + 1], M.q), M);
    const W z = mulmod<KIND>(v, xi, M);
    x[j + 1] = submod(submod(w, u, M.q), v, M.q);
    x[j] = (j & 2) ? submod(u, z, M.q) : addmod(u, z, M.q);
  }
}

// Column pass: R = 2^LOGR words of one column (stride C) in registers.
template <int LOGR, int KIND, typename W, typename MT>
__device__ __forceinline__ void col_fwd(W (&x)[1 << LOGR], const W* __restrict__ tw, const MT& M) {
  constexpr int R = 1 << LOGR;
#pragma unroll
  for (int lm = 0; lm < LOGR; ++lm) {
    const int m = 1 << lm, k = R >> (lm + 1);
#pragma unroll
    for (int g = 0; g < m; ++g) {
      const W xi = tw[m + g];
#pragma unroll
      for (int s = 0; s < k; ++s) ct_bfly<KIND>(x[2 * g * k + s], x[2 * g * k + s + k], xi, M);
    }
  }
}

template <int LOGR, int KIND, typename W, typename MT>
__device__ __forceinline__ void col_inv(W (&x)[1 << LOGR], const W* __restrict__ tw, const MT& M) {
  constexpr int R = 1 << LOGR;
#pragma unroll
  for (int lm = LOGR - 1; lm >= 0; --lm) {
    const int m = 1 << lm, k = R >> (lm + 1);
#pragma unroll
    for (int g = 0; g < m; ++g) {
      const W xi = tw[m + g];
#pragma unroll
      for (int s = 0; s < k; ++s) gs_bfly_half<KIND>(x[2 * g * k + s], x[2 * g * k + s + k], xi, M);
    }
  }
}

// The same radix-2^LOGR block at any depth of Alg. 5 / Alg. 6. A block of
// stages s0..s0+LOGR-1 touches 2^LOGR words at stride N >> (s0+LOGR) that
// share the index bits above bit log2(N) - s0; with h those high bits and
// rb = 2^s0 + h, stage s0+j's group g (within the block) uses the twiddle at
// (rb << j) + g. col_fwd / col_inv are the case rb = 1.
template <int LOGR, int KIND, typename W, typename MT>
__device__ __forceinline__ void blk_fwd(W (&x)[1 << LOGR], const W* __restrict__ tw, uint32_t rb, const MT& M) {
  constexpr int R = 1 << LOGR;
#pragma unroll
  for (int lm = 0; lm < LOGR; ++lm) {
    const int m = 1 << lm, k = R >> (lm + 1);
    const W* t = tw + (rb << lm);
#pragma unroll
    for (int g = 0; g < m; ++g) {
      const W xi = t[g];
#pragma unroll
      for (int s = 0; s < k; ++s) ct_bfly<KIND>(x[2 * g * k + s], x[2 * g * k + s + k], xi, M);
    }
  }
}

template <int LOGR, int KIND, typename W, typename MT>
__device__ __forceinline__ void blk_inv(W (&x)[1 << LOGR], const W* __restrict__ tw, uint32_t rb, const MT& M) {
  constexpr int R = 1 << LOGR;
#pragma unroll
  for (int lm = LOGR - 1; lm >= 0; --lm) {
    const int m = 1 << lm, k = R >> (lm + 1);
    const W* t = tw + (rb << lm);
#pragma unroll
    for (int g = 0; g < m; ++g) {
      const W xi = t[g];
#pragma unroll
      for (int s = 0; s < k; ++s) gs_bfly_half<KIND>(x[2 * g * k + s], x[2 * g * k + s + k], xi, M);
    }
  }
}

}  // namespace pm
