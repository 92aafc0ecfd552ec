// Interleaved (coefficient-major) batch layout, the storage of the paper's
// throughput-optimised multi-block design (Sec. V-C): within a limb the batch
// is an N x P matrix with coefficient j of polynomial p at [j * P + p], so the
// lanes of a wave, which hold consecutive polynomials, read and write
// consecutive words at every stage.
//
// Each thread runs one radix-2^LOGR block of stages (blk_fwd / blk_inv) of one
// polynomial with its 2^LOGR words in registers; a transform is a short
// sequence of such passes over HBM. A block of stages s0..s0+LOGR-1 is one
// grid row (blockIdx.y), so its twiddles are uniform across the workgroup.
//
//   IL_FWD  stages of Alg. 5 on one or two operands (A -> C, B -> D)
//   IL_INV  stages of Alg. 6 with halved butterflies (A -> C)
//   IL_MUL  the last block of Alg. 5 on A and on B, the pointwise product and
//           the first block of Alg. 6 (A, B -> C): Eq. 2's middle, fused
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ntt_device.hpp"
#include "pm_internal.hpp"

namespace pm {

template <int LOGR> struct IlWaves { static constexpr int value = LOGR >= 5 ? 2 : 4; };

template <int LOGR, int KIND, int MODE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(IlWaves<LOGR>::value + (MODE != IL_MUL), 8)))
k_il(const uint64_t* A, const uint64_t* B, uint64_t* C, uint64_t* D, const uint64_t* __restrict__ twf,
     const uint64_t* __restrict__ twi, uint32_t log2n, uint32_t s0, uint32_t polys, uint32_t nops, LimbSet ls) {
  constexpr int R = 1 << LOGR;
  const uint32_t p0 = blockIdx.x * blockDim.x;    // first polynomial of the workgroup
  const uint32_t lane = threadIdx.x;
  if (p0 + lane >= polys) return;
  const uint32_t limb = (MODE == IL_FWD) ? blockIdx.z / nops : blockIdx.z;
  const uint32_t op = (MODE == IL_FWD) ? blockIdx.z - limb * nops : 0;
  const uint32_t lk = log2n - s0 - LOGR;          // log2 of the block's stride
  const uint32_t h = blockIdx.y >> lk, lo = blockIdx.y & ((1u << lk) - 1);
  const size_t N = (size_t)1 << log2n;
  // everything but the lane index is uniform: word i of the block sits at
  // base + i * step + lane
  const size_t base = (size_t)limb * N * polys + ((((size_t)h << (log2n - s0)) | lo) * polys) + p0;
  const size_t step = ((size_t)polys) << lk;
  const uint32_t rb = (1u << s0) + h;
  const Mod M = ls.mod[limb];
  uint64_t x[R];
  if constexpr (MODE == IL_FWD) {
    const uint64_t* src = (op ? B : A) + base;
    uint64_t* dst = (op ? D : C) + base;
#pragma unroll
    for (int i = 0; i < R; ++i) x[i] = (src + i * step)[lane];
    blk_fwd<LOGR, KIND>(x, twf + (size_t)limb * N, rb, M);
#pragma unroll
    for (int i = 0; i < R; ++i) (dst + i * step)[lane] = x[i];
  } else if constexpr (MODE == IL_INV) {
    const uint64_t* src = A + base;
    uint64_t* dst = C + base;
#pragma unroll
    for (int i = 0; i < R; ++i) x[i] = (src + i * step)[lane];
    blk_inv<LOGR, KIND>(x, twi + (size_t)limb * N, rb, M);
#pragma unroll
    for (int i = 0; i < R; ++i) (dst + i * step)[lane] = x[i];
  } else {
    const uint64_t* tf = twf + (size_t)limb * N;
    const uint64_t* sa = A + base;
    const uint64_t* sb = B + base;
    uint64_t* dst = C + base;
#pragma unroll
    for (int i = 0; i < R; ++i) x[i] = (sa + i * step)[lane];
    blk_fwd<LOGR, KIND>(x, tf, rb, M);
    uint64_t y[R];
#pragma unroll
    for (int i = 0; i < R; ++i) y[i] = (sb + i * step)[lane];
    blk_fwd<LOGR, KIND>(y, tf, rb, M);
#pragma unroll
    for (int i = 0; i < R; ++i) x[i] = mulmod<KIND>(x[i], y[i], M);
    blk_inv<LOGR, KIND>(x, twi + (size_t)limb * N, rb, M);
#pragma unroll
    for (int i = 0; i < R; ++i) (dst + i * step)[lane] = x[i];
  }
}

template <int LOGR, int KIND, int MODE>
static void il_launch(const IlArgs& a, hipStream_t s) {
  const uint32_t bs = a.polys >= 256 ? 256u : ((a.polys + 63) / 64) * 64;
  const uint32_t nz = (MODE == IL_FWD) ? a.limbs * a.nops : a.limbs;
  dim3 grid((a.polys + bs - 1) / bs, 1u << (a.log2n - LOGR), nz);
  hipLaunchKernelGGL((k_il<LOGR, KIND, MODE>), grid, dim3(bs), 0, s, a.A, a.B, a.C, a.D, a.twf, a.twi, a.log2n,
                     a.s0, a.polys, a.nops, *a.ls);
}

template <int LOGR, int KIND>
static void il_launch_mode(const IlArgs& a, int mode, hipStream_t s) {
  if (mode == IL_FWD) il_launch<LOGR, KIND, IL_FWD>(a, s);
  else if (mode == IL_INV) il_launch<LOGR, KIND, IL_INV>(a, s);
  else if constexpr (LOGR <= IL_MUL_MAXR) il_launch<LOGR, KIND, IL_MUL>(a, s);
}

template <int LOGR>
static void il_launch_kind(const IlArgs& a, int kind, int mode, hipStream_t s) {
  if (kind == KIND_WIDE) il_launch_mode<LOGR, KIND_WIDE>(a, mode, s);
  else il_launch_mode<LOGR, KIND_ANY>(a, mode, s);
}

hipError_t launch_il(int logr, int kind, int mode, const IlArgs& a, hipStream_t s) {
  if (logr < 1 || logr > IL_MAXR || (mode == IL_MUL && logr > IL_MUL_MAXR)) return hipErrorInvalidValue;
  if (a.s0 + (uint32_t)logr > a.log2n) return hipErrorInvalidValue;
  switch (logr) {
    case 1: il_launch_kind<1>(a, kind, mode, s); break;
    case 2: il_launch_kind<2>(a, kind, mode, s); break;
    case 3: il_launch_kind<3>(a, kind, mode, s); break;
    case 4: il_launch_kind<4>(a, kind, mode, s); break;
    case 5: il_launch_kind<5>(a, kind, mode, s); break;
    default: il_launch_kind<6>(a, kind, mode, s); break;
  }
  return hipGetLastError();
}

}  // namespace pm
