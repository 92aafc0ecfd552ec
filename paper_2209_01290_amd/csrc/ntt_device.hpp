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
// The small-batch geometry does the same with rounds of two stages and 4
// words per thread: four times the threads per row, for batches too small
// to fill the GPU with 16-word threads.
//
// Column pass. One thread per column holds the R = 2^s words of that column
// in registers and runs the s column stages; twiddles are uniform per launch.
// In the software-pipelined kernels a 32-word column (s = 5) is held by two
// lanes of one wave instead, 16 words each (col32_fwd_pair below), so that the
// column code needs no more registers than the row code beside it.
#pragma once
#include "modarith.hpp"
#include "modarith32.hpp"

namespace pm {

// Row geometry code GEO: bits [0, 5) = c (row of 2^c words); bit 5 set =
// rounds of two stages with 4 words per thread (the small-batch geometry,
// more threads per row), clear = rounds of four stages with 16 words per
// thread. For the 16-word geometry GEO = c.
constexpr int row_geo(int logc, int ebx) { return logc | (ebx == 2 ? 32 : 0); }

template <int GEO>
struct RowGeom {
  static constexpr int LC = GEO & 31;                  // log2(row length)
  static constexpr int EBX = (GEO & 32) ? 2 : 4;       // index bits per round
  static constexpr int EB = LC < EBX ? LC : EBX;       // log2(words per thread)
  static constexpr int E = 1 << EB;
  static constexpr int LOGT = LC - EB;
  static constexpr int T = 1 << LOGT;                  // threads per row
  static constexpr int NR = LC <= EBX ? 1 : (LC + EBX - 1) / EBX;   // rounds
  static constexpr int WGMIN = EBX == 4 ? 256 : 64;
  static constexpr int WG = T < WGMIN ? WGMIN : T;     // threads per workgroup
  static constexpr int ROWS = WG / T;                  // rows per workgroup
  static constexpr int LDS_ROW = (1 << LC) + ((1 << LC) >> 4);  // padded words
  static constexpr int LDS_WORDS = NR > 1 ? ROWS * LDS_ROW : 1;
  // register-bit base p and butterfly bits [lo, hi) of round rho (forward order)
  static constexpr int hi(int rho) { return LC - EBX * rho; }
  static constexpr int lo(int rho) { return hi(rho) - EBX > 0 ? hi(rho) - EBX : 0; }
  static constexpr int p(int rho) { return rho == NR - 1 ? 0 : hi(rho) - EBX; }
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
// 64-bit accesses spread over the banks. With idx = th*2^(P+EB) + j*2^P + tl
// (tl < 2^P, j < 2^EB) the slot splits into a per-thread base plus a
// per-register constant, so every LDS access is one instruction with an
// immediate offset:
//   slot = [a + a/16 + tl + tl/16] + [j*2^P + (j*2^P)/16],  a = th*2^(P+EB)
// (exact for every round of both geometries: the low part j*2^P + tl never
// carries into the next multiple of 16 above a). For EB = 4, a + a/16 =
// th*(2^(P+4) + 2^P).
template <int P, int EB>
__device__ __forceinline__ uint32_t lds_base(uint32_t t) {
  const uint32_t th = t >> P, tl = t & ((1u << P) - 1u);
  if constexpr (EB == 4) {
    return th * ((16u << P) + (1u << P)) + tl + (tl >> 4);
  } else {
    const uint32_t a = th << (P + EB);
    return a + (a >> 4) + tl + (tl >> 4);
  }
}
template <int P>
__device__ __forceinline__ constexpr uint32_t lds_off(uint32_t j) {
  return (j << P) + ((j << P) >> 4);
}
// Row offset of register j: per-thread base plus a per-register constant.
template <int P, int EB>
__device__ __forceinline__ uint32_t row_base(uint32_t t) {
  return ((t >> P) << (P + EB)) | (t & ((1u << P) - 1u));
}

// Forward (CT) stages of round RHO on registers x. tw = psi_br of this limb,
// Rr = R + r for row r of an R-row split.
// TRUNC drops the stride-1 stage (the last of Alg. 5): the truncated CT NTT
// of the fused product (Sec. III-B).
template <int GEO, int RHO, int KIND, bool TRUNC = false, typename W, typename MT>
__device__ __forceinline__ void fwd_round(W (&x)[RowGeom<GEO>::E], uint32_t t, const W* __restrict__ tw,
                                          uint32_t Rr, const MT& M) {
  using G = RowGeom<GEO>;
  constexpr int P = G::p(RHO), HI = G::hi(RHO), LO = (TRUNC && G::lo(RHO) == 0) ? 1 : G::lo(RHO), EB = G::EB;
  const uint32_t th = t >> P;
#pragma unroll
  for (int b = HI - 1; b >= LO; --b) {
    const int jb = b - P;                          // register bit paired at this stage
    const uint32_t mm = 1u << (G::LC - b - 1);      // groups per row at this stage
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
template <int GEO, int RHO, int KIND, bool TRUNC = false, typename W, typename MT>
__device__ __forceinline__ void inv_round(W (&x)[RowGeom<GEO>::E], uint32_t t, const W* __restrict__ tw,
                                          uint32_t Rr, const MT& M) {
  using G = RowGeom<GEO>;
  constexpr int P = G::p(RHO), HI = G::hi(RHO), LO = (TRUNC && G::lo(RHO) == 0) ? 1 : G::lo(RHO), EB = G::EB;
  const uint32_t th = t >> P;
#pragma unroll
  for (int b = LO; b < HI; ++b) {
    const int jb = b - P;
    const uint32_t mm = 1u << (G::LC - b - 1);
    const uint32_t base = Rr * mm + (th << (P + EB - b - 1));
#pragma unroll
    for (int g = 0; g < (G::E >> (jb + 1)); ++g) {
      const W xh = half_tw(tw[base + g], M);     // halved once for its 2^jb butterflies
#pragma unroll
      for (int s = 0; s < (1 << jb); ++s) {
        const int j = (g << (jb + 1)) | s;
        gs_bfly_htw<KIND>(x[j], x[j | (1 << jb)], xh, M);
      }
    }
    stage_fence();
  }
}

// LDS exchanges only run for rows of at least two rounds, where every round's
// register bits are EB = EBX wide; a single-round row (c <= EBX) has P = 0
// and one thread per row, so its global accesses use t << EB directly.
template <int GEO, int RHO, typename W>
__device__ __forceinline__ void lds_put(W* lds, const W (&x)[RowGeom<GEO>::E], uint32_t t) {
  using G = RowGeom<GEO>;
  constexpr int P = G::p(RHO);
  W* b = lds + lds_base<P, G::EB>(t);
#pragma unroll
  for (int j = 0; j < G::E; ++j) b[lds_off<P>(j)] = x[j];
}

template <int GEO, int RHO, typename W>
__device__ __forceinline__ void lds_get(const W* lds, W (&x)[RowGeom<GEO>::E], uint32_t t) {
  using G = RowGeom<GEO>;
  constexpr int P = G::p(RHO);
  const W* b = lds + lds_base<P, G::EB>(t);
#pragma unroll
  for (int j = 0; j < G::E; ++j) x[j] = b[lds_off<P>(j)];
}

template <int GEO, int RHO, typename W>
__device__ __forceinline__ void gmem_get(const W* __restrict__ row, W (&x)[RowGeom<GEO>::E], uint32_t t) {
  using G = RowGeom<GEO>;
  constexpr int P = G::p(RHO);
  const uint32_t tb = (G::NR > 1) ? row_base<P, G::EB>(t) : (t << G::EB);
#pragma unroll
  for (int j = 0; j < G::E; ++j) x[j] = (row + (j << P))[tb];
}

template <int GEO, int RHO, typename W>
__device__ __forceinline__ void gmem_put(W* __restrict__ row, const W (&x)[RowGeom<GEO>::E], uint32_t t) {
  using G = RowGeom<GEO>;
  constexpr int P = G::p(RHO);
  const uint32_t tb = (G::NR > 1) ? row_base<P, G::EB>(t) : (t << G::EB);
#pragma unroll
  for (int j = 0; j < G::E; ++j) (row + (j << P))[tb] = x[j];
}

// Move registers from round FROM's layout to round TO's layout through LDS.
// All threads of the workgroup must call it (it holds two barriers).
template <int GEO, int FROM, int TO, typename W>
__device__ __forceinline__ void exchange(W* lds, W (&x)[RowGeom<GEO>::E], uint32_t t) {
  __syncthreads();
#if PM_POISON_LDS
  // Debug build: fill the row's LDS with words above every modulus before
  // each exchange, so a slot read without being written in this exchange (a
  // missing barrier or an indexing error) corrupts the result.
  for (uint32_t i = t; i < (uint32_t)RowGeom<GEO>::LDS_ROW; i += RowGeom<GEO>::T) lds[i] = ~(W)0;
  __syncthreads();
#endif
  lds_put<GEO, FROM>(lds, x, t);
  __syncthreads();
  lds_get<GEO, TO>(lds, x, t);
}

// All row stages of the forward transform: rounds 0..NR-1. On return x holds
// the row in the last round's layout (E consecutive words per thread).
template <int GEO, int KIND, int RHO = 0, bool TRUNC = false, typename W, typename MT>
__device__ __forceinline__ void fwd_rounds(W* lds, W (&x)[RowGeom<GEO>::E], uint32_t t, const W* __restrict__ tw,
                                           uint32_t Rr, const MT& M) {
  fwd_round<GEO, RHO, KIND, TRUNC>(x, t, tw, Rr, M);
  if constexpr (RHO + 1 < RowGeom<GEO>::NR) {
    exchange<GEO, RHO, RHO + 1>(lds, x, t);
    fwd_rounds<GEO, KIND, RHO + 1, TRUNC>(lds, x, t, tw, Rr, M);
  }
}

// All row stages of the inverse transform, from the last round's layout back
// to round 0's layout.
template <int GEO, int KIND, int RHO = RowGeom<GEO>::NR - 1, bool TRUNC = false, typename W, typename MT>
__device__ __forceinline__ void inv_rounds(W* lds, W (&x)[RowGeom<GEO>::E], uint32_t t, const W* __restrict__ tw,
                                           uint32_t Rr, const MT& M) {
  inv_round<GEO, RHO, KIND, TRUNC>(x, t, tw, Rr, M);
  if constexpr (RHO > 0) {
    exchange<GEO, RHO, RHO - 1>(lds, x, t);
    inv_rounds<GEO, KIND, RHO - 1, TRUNC>(lds, x, t, tw, Rr, M);
  }
}

// Alg. 7 on the 8 adjacent pairs (2i, 2i+1) of a thread's 16 consecutive words
// (last-round layout): with u = a0 b0, v = a1 b1, w = (a0+a1)(b0+b1),
//   c1 = w - u - v,  c0 = u + alpha^2 v,
// alpha^2 = (-1)^i psi_br[N/4 + i/2] (Alg. 8): the square of the stride-1
// twiddle is the stride-2 twiddle of the same word, index (R+r)*C/4 + idx/4,
// and the sign is fixed per register because 16t and r*C are multiples of 4.
// Needs C >= 4. Results overwrite x.
template <int GEO, typename W>
struct FusedTw {
  W v[RowGeom<GEO>::E / 4 > 0 ? RowGeom<GEO>::E / 4 : 1];
};

// The alpha^2 twiddles of a thread's pairs, loaded ahead of use.
template <int GEO, typename W>
__device__ __forceinline__ FusedTw<GEO, W> fused_twiddles(uint32_t t, const W* __restrict__ tw, uint32_t Rr) {
  using G = RowGeom<GEO>;
  static_assert(G::LC >= 2, "the fused product needs rows of at least 4 words");
  FusedTw<GEO, W> f;
  const uint32_t base = Rr * (1u << (G::LC - 2)) + (t << (G::EB - 2));
#pragma unroll
  for (int g = 0; g < G::E / 4; ++g) f.v[g] = tw[base + g];
  return f;
}

template <int GEO, int KIND, typename W, typename MT>
__device__ __forceinline__ void fused_hadamard(W (&x)[RowGeom<GEO>::E], const W (&y)[RowGeom<GEO>::E],
                                               const FusedTw<GEO, W>& f, const MT& M) {
  using G = RowGeom<GEO>;
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
      const W xh = half_tw(tw[m + g], M);
#pragma unroll
      for (int s = 0; s < k; ++s) gs_bfly_htw<KIND>(x[2 * g * k + s], x[2 * g * k + s + k], xh, M);
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
      const W xh = half_tw(t[g], M);
#pragma unroll
      for (int s = 0; s < k; ++s) gs_bfly_htw<KIND>(x[2 * g * k + s], x[2 * g * k + s + k], xh, M);
    }
  }
}

// Exchange between the two halves of a wave (v_permlane32_swap, gfx950).
// Afterwards lanes 32..63 hold in p what lanes 0..31 held in q, and lanes
// 0..31 hold in q what lanes 32..63 held in p; lanes 0..31 keep p and lanes
// 32..63 keep q. Every lane of the wave must be active.
__device__ __forceinline__ void half_swap(uint32_t& p, uint32_t& q) {
  const auto r = __builtin_amdgcn_permlane32_swap(p, q, false, false);
  p = r[0];
  q = r[1];
}

__device__ __forceinline__ void half_swap(uint64_t& p, uint64_t& q) {
  uint32_t p0 = lo32(p), p1 = hi32(p), q0 = lo32(q), q1 = hi32(q);
  half_swap(p0, q0);
  half_swap(p1, q1);
  p = pack64(p0, p1);
  q = pack64(q0, q1);
}

// Column pass of R = 32 words held by the lanes l and l + 32 of one wave
// (h = 0 and 1), 16 words each. The first stage of Alg. 5 (stride 16 rows)
// pairs row i with row i + 16, so half h starts with rows
// col32_split_row(j, h) = (j & 7) + 8h + 16 (j >> 3) in y[j]: y[k] and y[8+k]
// are the pairs of that stage. One exchange of eight words (y[8+k] of h = 0
// with y[k] of h = 1) then leaves half h with rows 16h + j in y[j], the block
// of rows whose last four column stages use the twiddles of blk_fwd with
// rb = 2 + h. The inverse (Alg. 6, halved) runs the same steps in reverse
// order: the block's four stages, the same exchange, then the stride-16 stage.
__device__ __forceinline__ uint32_t col32_split_row(int j, uint32_t h) { return (j & 7) + 8 * h + 16 * (j >> 3); }
__device__ __forceinline__ uint32_t col32_block_row(int j, uint32_t h) { return 16 * h + j; }

template <int KIND, typename W, typename MT>
__device__ __forceinline__ void col32_fwd_pair(W (&y)[16], const W* __restrict__ tw, uint32_t h, const MT& M) {
  const W xi = tw[1];
#pragma unroll
  for (int k = 0; k < 8; ++k) ct_bfly<KIND>(y[k], y[8 + k], xi, M);
#pragma unroll
  for (int k = 0; k < 8; ++k) half_swap(y[k], y[8 + k]);
  blk_fwd<4, KIND>(y, tw, 2 + h, M);
}

template <int KIND, typename W, typename MT>
__device__ __forceinline__ void col32_inv_pair(W (&y)[16], const W* __restrict__ tw, uint32_t h, const MT& M) {
  blk_inv<4, KIND>(y, tw, 2 + h, M);
#pragma unroll
  for (int k = 0; k < 8; ++k) half_swap(y[k], y[8 + k]);
  const W xh = half_tw(tw[1], M);
#pragma unroll
  for (int k = 0; k < 8; ++k) gs_bfly_htw<KIND>(y[k], y[8 + k], xh, M);
}

}  // namespace pm
