// Software-pipelined Eq. 2 (and the fused product of Alg. 8) over chunks of
// the batch's products: the throughput plan with rows of 2^12 words after a
// column pass of 2^3..2^5 rows (N = 2^15..2^17), 64- or 32-bit words.
//
// The column passes are bound by memory and the row pass by the VALU. With
// the batch split into G chunks of products, launch j runs three independent
// kinds of workgroup: the row pass of chunk j-1 (forward rows of a and b,
// product, inverse rows; one forward row transform when a = b), the forward
// column pass of chunk j and the inverse column pass of chunk j-2. Their data are disjoint, and every dependency (a
// chunk's rows after its forward columns, its inverse columns after its rows)
// is between consecutive launches on one stream, so no workgroup ever waits
// for another. The rows come first in each launch and the short column
// workgroups after them, so the column work fills the CUs that the long row
// workgroups leave idle as they finish. (An order that interleaved the kinds
// finely in the grid measured about 1.5x slower.) G + 2 launches per batch.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ntt_row.hpp"
#include "pm_internal.hpp"
#include "pm_pipe.hpp"

namespace pm {
namespace {

constexpr int PIPE_LC = 12;                        // row length 2^12 (16 words per thread)
using PG = RowGeom<PIPE_LC>;
static_assert(PG::WG == 256 && PG::ROWS == 1, "one 2^12-word row per workgroup of 256 threads");
static_assert(pipe_col_blocks(3) == (1u << PIPE_LC) / 256 && pipe_col_blocks(5) == (1u << PIPE_LC) / 128,
              "column blocks of 256 columns, of 128 columns for a 32-word column on two lanes");

// grid: nr row workgroups, then nf forward-column and ni inverse-column ones.
// A chunk is a range of products (limb-major: product p = limb * polys + poly,
// stored at p * N), so a chunk may end inside a limb. Every kind of work
// item fits the row modes' register budget (RowWaves): a column of 8 or 16
// words is held by one thread, one of 32 words by two lanes.
template <typename W, int LOGR, int KIND, int MODE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(RowWaves<MODE>::value, 8)))
k_pipe(PipeArgsT<W> a, LimbSetT<W> ls) {
  __shared__ W lds[PG::LDS_WORDS];
  constexpr uint32_t R = 1u << LOGR;
  constexpr uint32_t CB = pipe_col_blocks(LOGR);
  const size_t N = (size_t)1 << (PIPE_LC + LOGR), C = (size_t)1 << PIPE_LC;
  const uint32_t t = threadIdx.x, b = blockIdx.x;
  if (b < a.nr) {
    const uint32_t prod = a.r0 + b / R, row = b % R;
    const uint32_t limb = prod / a.polys;
    const size_t off = (size_t)prod * N + ((size_t)row << PIPE_LC);
    const typename ModOf<W>::type M = ls.mod[limb];
    const W* Bp = (MODE == ROW_SQR) ? nullptr : (a.nops == 1 ? a.C : a.WS) + off;
    row_task<PIPE_LC, KIND, MODE>(a.C + off, Bp, a.C + off, a.twf + (size_t)limb * N, a.twi + (size_t)limb * N,
                                  R + row, true, M, lds, t);
    return;
  }
  // column workgroups: forward (a -> C, b -> WS) or inverse (C in place)
  const bool fwd = b < a.nr + a.nf;
  const uint32_t idx = fwd ? b - a.nr : b - a.nr - a.nf;
  const uint32_t nops = fwd ? a.nops : 1u;
  const uint32_t cb = idx % CB;
  const uint32_t rest = idx / CB;
  const uint32_t op = rest % nops;
  const uint32_t prod = (fwd ? a.f0 : a.i0) + rest / nops;
  const uint32_t limb = prod / a.polys;
  const typename ModOf<W>::type M = ls.mod[limb];
  const W* tw = (fwd ? a.twf : a.twi) + (size_t)limb * N;
  if constexpr (LOGR == 5) {
    // lanes l and l + 32 of a wave share a column
    const uint32_t lane = t & 63, h = lane >> 5;
    const size_t off = (size_t)prod * N + (size_t)cb * 128 + (t >> 6) * 32 + (lane & 31);
    const W* src = fwd ? (op ? a.B : a.A) + off : a.C + off;
    W* dst = fwd ? (op ? a.WS : a.C) + off : a.C + off;
    W y[16];
    if (fwd) {
#pragma unroll
      for (int j = 0; j < 16; ++j) y[j] = src[col32_split_row(j, h) * C];
      col32_fwd_pair<KIND>(y, tw, h, M);
#pragma unroll
      for (int j = 0; j < 16; ++j) dst[col32_block_row(j, h) * C] = y[j];
    } else {
#pragma unroll
      for (int j = 0; j < 16; ++j) y[j] = src[col32_block_row(j, h) * C];
      col32_inv_pair<KIND>(y, tw, h, M);
#pragma unroll
      for (int j = 0; j < 16; ++j) dst[col32_split_row(j, h) * C] = y[j];
    }
  } else {
    const size_t off = (size_t)prod * N + (size_t)cb * 256 + t;
    const W* src = fwd ? (op ? a.B : a.A) + off : a.C + off;
    W* dst = fwd ? (op ? a.WS : a.C) + off : a.C + off;
    W x[R];
#pragma unroll
    for (uint32_t i = 0; i < R; ++i) x[i] = src[i * C];
    if (fwd) col_fwd<LOGR, KIND>(x, tw, M);
    else col_inv<LOGR, KIND>(x, tw, M);
#pragma unroll
    for (uint32_t i = 0; i < R; ++i) dst[i * C] = x[i];
  }
}

template <typename W, int LOGR, int MODE>
void pipe_launch(const PipeArgsT<W>& a, const LimbSetT<W>& ls, int kind, hipStream_t s) {
  const uint32_t blocks = a.nr + a.nf + a.ni;
  if (kind == KIND_WIDE)
    hipLaunchKernelGGL((k_pipe<W, LOGR, KIND_WIDE, MODE>), dim3(blocks), dim3(256), 0, s, a, ls);
  else
    hipLaunchKernelGGL((k_pipe<W, LOGR, KIND_ANY, MODE>), dim3(blocks), dim3(256), 0, s, a, ls);
}

template <typename W, int MODE>
hipError_t pipe_launch_logr(int logr, const PipeArgsT<W>& a, const LimbSetT<W>& ls, int kind, hipStream_t s) {
  switch (logr) {
    case 3: pipe_launch<W, 3, MODE>(a, ls, kind, s); break;
    case 4: pipe_launch<W, 4, MODE>(a, ls, kind, s); break;
    case 5: pipe_launch<W, 5, MODE>(a, ls, kind, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename W>
hipError_t launch_pipe_any(int logr, int mode, const PipeArgsT<W>& a, const LimbSetT<W>& ls, int kind,
                           hipStream_t s) {
  if (a.nops < 1 || a.nops > 2) return hipErrorInvalidValue;
  if (a.nr + a.nf + a.ni == 0) return hipSuccess;
  switch (mode) {
    case ROW_MUL: return pipe_launch_logr<W, ROW_MUL>(logr, a, ls, kind, s);
    case ROW_FMUL: return pipe_launch_logr<W, ROW_FMUL>(logr, a, ls, kind, s);
    case ROW_SQR: return pipe_launch_logr<W, ROW_SQR>(logr, a, ls, kind, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_pipe(int logr, int mode, const PipeArgsT<uint64_t>& a, const LimbSetT<uint64_t>& ls, int kind,
                       hipStream_t s) {
  return launch_pipe_any(logr, mode, a, ls, kind, s);
}

hipError_t launch_pipe(int logr, int mode, const PipeArgsT<uint32_t>& a, const LimbSetT<uint32_t>& ls, int kind,
                       hipStream_t s) {
  return launch_pipe_any(logr, mode, a, ls, kind, s);
}

}  // namespace pm
