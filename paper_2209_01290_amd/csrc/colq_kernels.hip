// Column pass with four words per thread, for calls too small to fill the
// GPU with one thread per column.
//
// The first log2 R stages of Alg. 5 (the last of Alg. 6) pair rows of one
// column of the R x C view; every column runs the same R-point merged
// transform with twiddles psi_br[1..R). Forward stage s (0-based) pairs rows
// r and r + h, h = R >> (s+1), in group r / (2h) of 2^s groups, twiddle
// index 2^s + group. Here a column is spread over TPC = R/4 threads. The
// stages run in rounds of two: in the round of stages (s, s+1), thread t
// holds the rows b + {0, q, 2q, 3q} with q = R >> (s+2) and
// b = (t / q) * 4q + t % q, so stage s pairs registers (0,2), (1,3) in group
// t / q and stage s+1 pairs (0,1), (2,3) in groups 2(t / q) and 2(t / q) + 1.
// When log2 R is odd, stage 0 runs alone in the first forward round (the
// last inverse round) with q = R/4. The inverse runs the rounds backwards,
// each round's stages in reverse order, with the halved GS butterflies of
// Eq. 2. Rounds exchange registers through LDS; the two exchange buffers
// alternate, so one barrier per exchange suffices.
//
// grid: x = block of CPW columns, y = poly, z = limb * nops + op;
// block = TPC * CPW threads, thread = t * CPW + j (column j of the block).
// Neighbouring lanes take neighbouring columns, so each global access of a
// wave covers CPW consecutive words in each of 64 / CPW rows.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ntt_device.hpp"
#include "pm_colq.hpp"

namespace pm {
namespace {

constexpr int COLQ_WG = 256;   // largest block: 4 * COLQ_WG words of LDS per buffer

template <int LOGR>
struct ColqGeom {
  static constexpr int R = 1 << LOGR;
  static constexpr int TPC = R / 4;                  // threads per column
  static constexpr int NRND = (LOGR + 1) / 2;        // rounds
  // first stage and length of round rho (forward order)
  static constexpr int stage(int rho) { return (LOGR & 1) ? (rho == 0 ? 0 : 2 * rho - 1) : 2 * rho; }
  static constexpr int len(int rho) { return ((LOGR & 1) && rho == 0) ? 1 : 2; }
  // log2 q of round rho
  static constexpr int lq(int rho) { return LOGR - stage(rho) - 2; }
};

// Row of register k of thread t in a round with quarter q = 2^LQ.
template <int LQ>
__device__ __forceinline__ uint32_t colq_row(uint32_t t, int k) {
  return ((t >> LQ) << (LQ + 2)) + (t & ((1u << LQ) - 1u)) + ((uint32_t)k << LQ);
}

template <int LQ_FROM, int LQ_TO, typename W>
__device__ __forceinline__ void colq_exchange(W* buf, W (&x)[4], uint32_t t, uint32_t j, uint32_t logcpw) {
#if PM_POISON_LDS
  // Debug build: fill the buffer with words above every modulus first, so a
  // slot read without being written in this exchange corrupts the result.
  for (int k = 0; k < 4; ++k) buf[k * blockDim.x + threadIdx.x] = ~(W)0;
  __syncthreads();
#endif
#pragma unroll
  for (int k = 0; k < 4; ++k) buf[(colq_row<LQ_FROM>(t, k) << logcpw) + j] = x[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 4; ++k) x[k] = buf[(colq_row<LQ_TO>(t, k) << logcpw) + j];
}

template <int LOGR, int KIND, int INV, typename W>
__global__ void __launch_bounds__(COLQ_WG)
k_colq(const W* src0, W* dst0, const W* src1, W* dst1, const W* __restrict__ tw, uint32_t log2n, uint32_t polys,
       uint32_t nops, uint32_t logcpw, LimbSetT<W> ls) {
  using G = ColqGeom<LOGR>;
  __shared__ W lds[2][4 * COLQ_WG];
  const uint32_t limb = blockIdx.z / nops, op = blockIdx.z - limb * nops;
  const uint32_t j = threadIdx.x & ((1u << logcpw) - 1u);
  const uint32_t t = threadIdx.x >> logcpw;
  const size_t N = (size_t)1 << log2n, C = N >> LOGR;
  const size_t off = ((size_t)limb * polys + blockIdx.y) * N + ((size_t)blockIdx.x << logcpw) + j;
  const W* src = (op ? src1 : src0) + off;
  W* dst = (op ? dst1 : dst0) + off;
  const W* tl = tw + (size_t)limb * N;
  const typename ModOf<W>::type M = ls.mod[limb];

  // every twiddle this thread needs, fetched before the data arrives
  W ta[G::NRND], tb[G::NRND], tc[G::NRND];
#pragma unroll
  for (int rho = 0; rho < G::NRND; ++rho) {
    const uint32_t m = 1u << G::stage(rho), g = t >> G::lq(rho);
    ta[rho] = tl[m + g];
    if (G::len(rho) == 2) {
      tb[rho] = tl[2 * m + 2 * g];
      tc[rho] = tl[2 * m + 2 * g + 1];
    }
  }

  W x[4];
  if (!INV) {
    constexpr int LQ0 = G::lq(0);
#pragma unroll
    for (int k = 0; k < 4; ++k) x[k] = src[(size_t)colq_row<LQ0>(t, k) * C];
    ct_bfly<KIND>(x[0], x[2], ta[0], M);
    ct_bfly<KIND>(x[1], x[3], ta[0], M);
    if (G::len(0) == 2) {
      ct_bfly<KIND>(x[0], x[1], tb[0], M);
      ct_bfly<KIND>(x[2], x[3], tc[0], M);
    }
    if constexpr (G::NRND > 1) {
      colq_exchange<G::lq(0), G::lq(1)>(lds[0], x, t, j, logcpw);
      ct_bfly<KIND>(x[0], x[2], ta[1], M);
      ct_bfly<KIND>(x[1], x[3], ta[1], M);
      ct_bfly<KIND>(x[0], x[1], tb[1], M);
      ct_bfly<KIND>(x[2], x[3], tc[1], M);
    }
    if constexpr (G::NRND > 2) {
      colq_exchange<G::lq(1), G::lq(2)>(lds[1], x, t, j, logcpw);
      ct_bfly<KIND>(x[0], x[2], ta[2], M);
      ct_bfly<KIND>(x[1], x[3], ta[2], M);
      ct_bfly<KIND>(x[0], x[1], tb[2], M);
      ct_bfly<KIND>(x[2], x[3], tc[2], M);
    }
    if constexpr (G::NRND > 3) {
      colq_exchange<G::lq(2), G::lq(3)>(lds[0], x, t, j, logcpw);
      ct_bfly<KIND>(x[0], x[2], ta[3], M);
      ct_bfly<KIND>(x[1], x[3], ta[3], M);
      ct_bfly<KIND>(x[0], x[1], tb[3], M);
      ct_bfly<KIND>(x[2], x[3], tc[3], M);
    }
    constexpr int LQL = G::lq(G::NRND - 1);
#pragma unroll
    for (int k = 0; k < 4; ++k) dst[(size_t)colq_row<LQL>(t, k) * C] = x[k];
  } else {
    constexpr int LQL = G::lq(G::NRND - 1);
#pragma unroll
    for (int k = 0; k < 4; ++k) x[k] = src[(size_t)colq_row<LQL>(t, k) * C];
    if constexpr (G::NRND > 3) {
      gs_bfly_half<KIND>(x[0], x[1], tb[3], M);
      gs_bfly_half<KIND>(x[2], x[3], tc[3], M);
      gs_bfly_half<KIND>(x[0], x[2], ta[3], M);
      gs_bfly_half<KIND>(x[1], x[3], ta[3], M);
      colq_exchange<G::lq(3), G::lq(2)>(lds[0], x, t, j, logcpw);
    }
    if constexpr (G::NRND > 2) {
      gs_bfly_half<KIND>(x[0], x[1], tb[2], M);
      gs_bfly_half<KIND>(x[2], x[3], tc[2], M);
      gs_bfly_half<KIND>(x[0], x[2], ta[2], M);
      gs_bfly_half<KIND>(x[1], x[3], ta[2], M);
      colq_exchange<G::lq(2), G::lq(1)>(lds[1], x, t, j, logcpw);
    }
    if constexpr (G::NRND > 1) {
      gs_bfly_half<KIND>(x[0], x[1], tb[1], M);
      gs_bfly_half<KIND>(x[2], x[3], tc[1], M);
      gs_bfly_half<KIND>(x[0], x[2], ta[1], M);
      gs_bfly_half<KIND>(x[1], x[3], ta[1], M);
      colq_exchange<G::lq(1), G::lq(0)>(lds[0], x, t, j, logcpw);
    }
    if (G::len(0) == 2) {
      gs_bfly_half<KIND>(x[0], x[1], tb[0], M);
      gs_bfly_half<KIND>(x[2], x[3], tc[0], M);
    }
    gs_bfly_half<KIND>(x[0], x[2], ta[0], M);
    gs_bfly_half<KIND>(x[1], x[3], ta[0], M);
    constexpr int LQ0 = G::lq(0);
#pragma unroll
    for (int k = 0; k < 4; ++k) dst[(size_t)colq_row<LQ0>(t, k) * C] = x[k];
  }
}

template <int LOGR, int KIND, typename W>
void colq_launch(const ColArgsT<W>& a, bool inv, hipStream_t s) {
  using G = ColqGeom<LOGR>;
  const uint32_t logc = a.log2n - LOGR;
  uint32_t logcpw = 0;
  while ((G::TPC << (logcpw + 1)) <= COLQ_WG && logcpw + 1 <= logc) ++logcpw;
  dim3 grid(1u << (logc - logcpw), a.polys, a.limbs * a.nops);
  dim3 block(G::TPC << logcpw);
  if (inv)
    hipLaunchKernelGGL((k_colq<LOGR, KIND, 1, W>), grid, block, 0, s, a.src0, a.dst0, a.src1, a.dst1, a.tw,
                       a.log2n, a.polys, a.nops, logcpw, *a.ls);
  else
    hipLaunchKernelGGL((k_colq<LOGR, KIND, 0, W>), grid, block, 0, s, a.src0, a.dst0, a.src1, a.dst1, a.tw,
                       a.log2n, a.polys, a.nops, logcpw, *a.ls);
}

template <int LOGR, typename W>
void colq_launch_kind(const ColArgsT<W>& a, int kind, bool inv, hipStream_t s) {
  if (kind == KIND_WIDE) colq_launch<LOGR, KIND_WIDE>(a, inv, s);
  else colq_launch<LOGR, KIND_ANY>(a, inv, s);
}

template <typename W>
hipError_t launch_colq_any(int logr, int kind, bool inv, const ColArgsT<W>& a, hipStream_t s) {
  if (logr < (int)PM_COLQ_MIN_LOGR || logr > (int)PM_COLQ_MAX_LOGR || (uint32_t)logr > a.log2n)
    return hipErrorInvalidValue;
  switch (logr) {
    case 2: colq_launch_kind<2>(a, kind, inv, s); break;
    case 3: colq_launch_kind<3>(a, kind, inv, s); break;
    case 4: colq_launch_kind<4>(a, kind, inv, s); break;
    case 5: colq_launch_kind<5>(a, kind, inv, s); break;
    case 6: colq_launch_kind<6>(a, kind, inv, s); break;
    case 7: colq_launch_kind<7>(a, kind, inv, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_colq(int logr, int kind, bool inv, const ColArgs& a, hipStream_t s) {
  return launch_colq_any(logr, kind, inv, a, s);
}

hipError_t launch_colq(int logr, int kind, bool inv, const ColArgsT<uint32_t>& a, hipStream_t s) {
  return launch_colq_any(logr, kind, inv, a, s);
}

}  // namespace pm
