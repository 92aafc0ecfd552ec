// Software-pipelined Eq. 2 and fused product (pipe_kernels.hip): one launch
// runs the row pass of one chunk of products, the forward column pass of the
// next chunk and the inverse column pass of the chunk before.
#pragma once
#include "pm_internal.hpp"

namespace pm {

// One pipelined launch over a batch [limb][poly][N] of 64- or 32-bit words,
// N = 2^(12 + logr), rows of 2^12 words. A chunk is a range of products p =
// limb * polys + poly (indices within the launch group): r0 / f0 / i0 = first
// product of the row, forward-column and inverse-column chunk; nr / nf / ni =
// workgroups of each kind (0 when absent): nr = 2^logr per product (one per
// row), nf = nops * pipe_col_blocks(logr) per product (nops operands),
// ni = pipe_col_blocks(logr) per product. nops = 1 when a = b (squaring): the forward
// column pass transforms a alone into C, and the rows read C for both.
template <typename W>
struct PipeArgsT {
  const W* A;
  const W* B;
  W* C;                        // output; holds a's column-pass result in between
  W* WS;                       // workspace: b's column-pass result (nops = 2)
  const W* twf;                // psi_br [limbs][N]
  const W* twi;                // psi_inv_br [limbs][N]
  uint32_t polys;
  uint32_t r0, f0, i0;
  uint32_t nr, nf, ni;
  uint32_t nops;
};

// logr in 3..5; mode: ROW_MUL (Eq. 2), ROW_FMUL (Alg. 8's rows) or ROW_SQR
// (Eq. 2 with a = b, one forward row transform).
hipError_t launch_pipe(int logr, int mode, const PipeArgsT<uint64_t>& a, const LimbSetT<uint64_t>& ls, int kind,
                       hipStream_t s);
hipError_t launch_pipe(int logr, int mode, const PipeArgsT<uint32_t>& a, const LimbSetT<uint32_t>& ls, int kind,
                       hipStream_t s);

}  // namespace pm
