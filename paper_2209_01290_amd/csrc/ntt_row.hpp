// One row task of the row pass (see ntt_device.hpp), shared by the batch
// kernels (row_kernel.inc) and the job-table kernels (pm_jobs.hip).
//
//   ROW_FWD  the last c stages of Alg. 5 on one row, in place
//   ROW_INV  the first c stages of Alg. 6 (halved butterflies), in place
//   ROW_MUL  the row of a forward, the row of b forward, pointwise product
//            mod q, inverse; with R = 1 this is all of Eq. 2 for one pair
//   ROW_SQR  as ROW_MUL with b = a (one forward transform)
//   ROW_FMUL the fused product of Sec. III-B (Alg. 8): truncated rows of a and
//            b, Alg. 7 on adjacent pairs, truncated inverse rows
#pragma once
#include "ntt_device.hpp"
#include "pm_internal.hpp"

namespace pm {

template <int GEO, int KIND, int MODE, typename W, typename MT>
__device__ __forceinline__ void row_task(const W* A, const W* B, W* Cout, const W* tf, const W* ti, uint32_t Rr,
                                         bool active, const MT& M, W* lds, uint32_t t) {
  using G = RowGeom<GEO>;
  W x[G::E];
#pragma unroll
  for (int j = 0; j < G::E; ++j) x[j] = 0;
  if constexpr (MODE == ROW_FWD) {
    if (active) gmem_get<GEO, 0>(A, x, t);
    fwd_rounds<GEO, KIND>(lds, x, t, tf, Rr, M);
    if (active) gmem_put<GEO, G::NR - 1>(Cout, x, t);
  } else if constexpr (MODE == ROW_INV) {
    if (active) gmem_get<GEO, G::NR - 1>(A, x, t);
    inv_rounds<GEO, KIND>(lds, x, t, ti, Rr, M);
    if (active) gmem_put<GEO, 0>(Cout, x, t);
  } else if constexpr (MODE == ROW_MUL) {
    if (active) gmem_get<GEO, 0>(A, x, t);
    fwd_rounds<GEO, KIND>(lds, x, t, tf, Rr, M);
    // keep the scheduler from overlapping the two transforms (register pressure)
    __builtin_amdgcn_sched_barrier(0);
    W y[G::E];
#pragma unroll
    for (int j = 0; j < G::E; ++j) y[j] = 0;
    if (active) gmem_get<GEO, 0>(B, y, t);
    fwd_rounds<GEO, KIND>(lds, y, t, tf, Rr, M);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < G::E; ++j) x[j] = mulmod<KIND>(x[j], y[j], M);
    inv_rounds<GEO, KIND>(lds, x, t, ti, Rr, M);
    if (active) gmem_put<GEO, 0>(Cout, x, t);
  } else if constexpr (MODE == ROW_FMUL) {
    // fused product (Alg. 8): truncated forward rows of a and b, Alg. 7 on
    // adjacent pairs, truncated inverse rows
    if (active) gmem_get<GEO, 0>(A, x, t);
    fwd_rounds<GEO, KIND, 0, true>(lds, x, t, tf, Rr, M);
    __builtin_amdgcn_sched_barrier(0);
    W y[G::E];
#pragma unroll
    for (int j = 0; j < G::E; ++j) y[j] = 0;
    if (active) gmem_get<GEO, 0>(B, y, t);
    const FusedTw<GEO, W> ftw = fused_twiddles<GEO>(t, tf, Rr);   // in flight during b's rows
    fwd_rounds<GEO, KIND, 0, true>(lds, y, t, tf, Rr, M);
    __builtin_amdgcn_sched_barrier(0);
    fused_hadamard<GEO, KIND>(x, y, ftw, M);
    inv_rounds<GEO, KIND, G::NR - 1, true>(lds, x, t, ti, Rr, M);
    if (active) gmem_put<GEO, 0>(Cout, x, t);
  } else {  // ROW_SQR: a == b, one forward transform
    if (active) gmem_get<GEO, 0>(A, x, t);
    fwd_rounds<GEO, KIND>(lds, x, t, tf, Rr, M);
#pragma unroll
    for (int j = 0; j < G::E; ++j) x[j] = mulmod<KIND>(x[j], x[j], M);
    inv_rounds<GEO, KIND>(lds, x, t, ti, Rr, M);
    if (active) gmem_put<GEO, 0>(Cout, x, t);
  }
}

// Register budget: transforms keep 4 waves per SIMD (<= 128 VGPRs); the fused
// product holds a second row of 16 words and gets 3 waves per SIMD. (The
// 4-word geometry needs far fewer registers; the bound is only a floor.)
template <int MODE>
struct RowWaves {
  static constexpr int value = (MODE == ROW_MUL || MODE == ROW_FMUL) ? 3 : 4;   // two rows held
};

}  // namespace pm
