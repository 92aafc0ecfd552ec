// HIP kernels for gfx950 and their host-side launchers.
//
//   k_mulmod    elementwise a*b mod q (Alg. 4), one modulus
//   k_row       (row_kernel.inc, one file per row length) row pass of the
//               merged NTTs: forward, inverse, or the fused polymul row step
//   k_col       column pass (first / last log2 R stages), forward or inverse
//   k_stage     one radix-2 stage per launch straight from HBM (the plain
//               per-stage path: one launch per stage of Alg. 5 / Alg. 6)
//   k_pointwise a[i]*b[i] mod q over whole polynomials (the plain path)
//
// Batch layout everywhere: [limb][poly][N] uint64 words, limb l uses modulus
// mods[l] and twiddle tables tw + l*N.
#include "pm_internal.hpp"
#include "ntt_device.hpp"

namespace pm {

// ---------------------------------------------------------------- mulmod --
// c may alias a or b (each word is read and written by the same thread), so
// no pointer is marked __restrict__.
template <int KIND>
__global__ void __launch_bounds__(256) k_mulmod(const uint64_t* a, const uint64_t* b, uint64_t* c, size_t n, Mod M) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) c[i] = mulmod<KIND>(a[i], b[i], M);
}

// ---------------------------------------------------------------- column --
// grid: x = block of 256 columns, y = poly, z = limb * nops + op.
template <int LOGR, int KIND, int INV, typename W>
__global__ void __launch_bounds__(256)
k_col(const W* src0, W* dst0, const W* src1, W* dst1, const W* __restrict__ tw, uint32_t log2n, uint32_t polys,
      uint32_t nops, LimbSetT<W> ls) {
  constexpr int R = 1 << LOGR;
  const uint32_t limb = blockIdx.z / nops, op = blockIdx.z - limb * nops;
  const uint32_t poly = blockIdx.y;
  const size_t N = (size_t)1 << log2n, C = N >> LOGR;
  const size_t col = (size_t)blockIdx.x * 256 + threadIdx.x;
  const size_t off = ((size_t)limb * polys + poly) * N + col;
  const W* src = (op ? src1 : src0) + off;
  W* dst = (op ? dst1 : dst0) + off;
  const W* t = tw + (size_t)limb * N;
  const typename ModOf<W>::type M = ls.mod[limb];
  W x[R];
#pragma unroll
  for (int i = 0; i < R; ++i) x[i] = src[i * C];
  if (INV) col_inv<LOGR, KIND>(x, t, M);
  else col_fwd<LOGR, KIND>(x, t, M);
#pragma unroll
  for (int i = 0; i < R; ++i) dst[i * C] = x[i];
}

// ------------------------------------------------------- plain per-stage --
// One butterfly per thread for the stage with m groups of stride k = N/(2m).
// grid: x = block of 256 butterflies, y = poly, z = limb * nops + op.
template <int KIND, int INV>
__global__ void __launch_bounds__(256)
k_stage(const uint64_t* src0, uint64_t* dst0, const uint64_t* src1, uint64_t* dst1,
        const uint64_t* __restrict__ tw, uint32_t log2n, uint32_t log2m, uint32_t polys, uint32_t nops,
        LimbSet ls) {
  const uint32_t limb = blockIdx.z / nops, op = blockIdx.z - limb * nops;
  const uint32_t poly = blockIdx.y;
  const size_t N = (size_t)1 << log2n;
  const uint32_t bidx = blockIdx.x * 256 + threadIdx.x;
  if (bidx >= (N >> 1)) return;
  const uint32_t log2k = log2n - 1 - log2m;
  const uint32_t i = bidx >> log2k, s = bidx & ((1u << log2k) - 1);
  const size_t j = ((size_t)i << (log2k + 1)) + s;
  const size_t off = ((size_t)limb * polys + poly) * N;
  const uint64_t* src = (op ? src1 : src0) + off;
  uint64_t* dst = (op ? dst1 : dst0) + off;
  const Mod M = ls.mod[limb];
  const uint64_t xi = tw[(size_t)limb * N + (1u << log2m) + i];
  uint64_t u = src[j], v = src[j + ((size_t)1 << log2k)];
  if (INV) gs_bfly_half<KIND>(u, v, xi, M);
  else ct_bfly<KIND>(u, v, xi, M);
  dst[j] = u;
  dst[j + ((size_t)1 << log2k)] = v;
}

// grid: x = block of 256 words, y = poly, z = limb.
template <int KIND>
__global__ void __launch_bounds__(256)
k_pointwise(const uint64_t* A, const uint64_t* B, uint64_t* Cout, uint32_t log2n, uint32_t polys, LimbSet ls) {
  const size_t N = (size_t)1 << log2n;
  const size_t w = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (w >= N) return;
  const size_t off = ((size_t)blockIdx.z * polys + blockIdx.y) * N + w;
  const Mod M = ls.mod[blockIdx.z];
  Cout[off] = mulmod<KIND>(A[off], B[off], M);
}

// =============================================================== launchers ==

hipError_t launch_mulmod(const uint64_t* a, const uint64_t* b, uint64_t* c, size_t n, const Mod& M,
                         int kind, hipStream_t s) {
  size_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (kind == KIND_WIDE) hipLaunchKernelGGL((k_mulmod<KIND_WIDE>), dim3(blocks), dim3(256), 0, s, a, b, c, n, M);
  else hipLaunchKernelGGL((k_mulmod<KIND_ANY>), dim3(blocks), dim3(256), 0, s, a, b, c, n, M);
  return hipGetLastError();
}

template <typename A>
static hipError_t launch_row_any(int logc, int kind, int mode, int ebx, const A& a, hipStream_t s) {
  switch (logc) {
#define PM_ROW_CASE(L) case L: return launch_row_##L(kind, mode, ebx, a, s);
    PM_ROW_CASE(1) PM_ROW_CASE(2) PM_ROW_CASE(3) PM_ROW_CASE(4) PM_ROW_CASE(5) PM_ROW_CASE(6)
    PM_ROW_CASE(7) PM_ROW_CASE(8) PM_ROW_CASE(9) PM_ROW_CASE(10) PM_ROW_CASE(11) PM_ROW_CASE(12)
    PM_ROW_CASE(13) PM_ROW_CASE(14)
#undef PM_ROW_CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_row(int logc, int kind, int mode, const RowArgs& a, hipStream_t s, int ebx) {
  return launch_row_any(logc, kind, mode, ebx, a, s);
}

hipError_t launch_row(int logc, int kind, int mode, const RowArgsT<uint32_t>& a, hipStream_t s, int ebx) {
  return launch_row_any(logc, kind, mode, ebx, a, s);
}

template <int LOGR, int KIND, typename W>
static void col_launch(const ColArgsT<W>& a, bool inv, hipStream_t s) {
  const size_t C = ((size_t)1 << a.log2n) >> LOGR;
  dim3 grid((uint32_t)(C / 256), a.polys, a.limbs * a.nops);
  if (inv)
    hipLaunchKernelGGL((k_col<LOGR, KIND, 1, W>), grid, dim3(256), 0, s, a.src0, a.dst0, a.src1, a.dst1, a.tw,
                       a.log2n, a.polys, a.nops, *a.ls);
  else
    hipLaunchKernelGGL((k_col<LOGR, KIND, 0, W>), grid, dim3(256), 0, s, a.src0, a.dst0, a.src1, a.dst1, a.tw,
                       a.log2n, a.polys, a.nops, *a.ls);
}

template <int LOGR, typename W>
static void col_launch_kind(const ColArgsT<W>& a, int kind, bool inv, hipStream_t s) {
  if (kind == KIND_WIDE) col_launch<LOGR, KIND_WIDE>(a, inv, s);
  else col_launch<LOGR, KIND_ANY>(a, inv, s);
}

template <typename W>
static hipError_t launch_col_any(int logr, int kind, bool inv, const ColArgsT<W>& a, hipStream_t s) {
  switch (logr) {
    case 1: col_launch_kind<1>(a, kind, inv, s); break;
    case 2: col_launch_kind<2>(a, kind, inv, s); break;
    case 3: col_launch_kind<3>(a, kind, inv, s); break;
    case 4: col_launch_kind<4>(a, kind, inv, s); break;
    case 5: col_launch_kind<5>(a, kind, inv, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_col(int logr, int kind, bool inv, const ColArgs& a, hipStream_t s) {
  return launch_col_any(logr, kind, inv, a, s);
}

hipError_t launch_col(int logr, int kind, bool inv, const ColArgsT<uint32_t>& a, hipStream_t s) {
  return launch_col_any(logr, kind, inv, a, s);
}

hipError_t launch_stage(int kind, bool inv, const ColArgs& a, uint32_t log2m, hipStream_t s) {
  const size_t half = ((size_t)1 << a.log2n) >> 1;
  dim3 grid((uint32_t)((half + 255) / 256), a.polys, a.limbs * a.nops);
#define PM_STAGE(K, I) hipLaunchKernelGGL((k_stage<K, I>), grid, dim3(256), 0, s, a.src0, a.dst0, a.src1, a.dst1, \
                                          a.tw, a.log2n, log2m, a.polys, a.nops, *a.ls)
  if (kind == KIND_WIDE) { if (inv) PM_STAGE(KIND_WIDE, 1); else PM_STAGE(KIND_WIDE, 0); }
  else { if (inv) PM_STAGE(KIND_ANY, 1); else PM_STAGE(KIND_ANY, 0); }
#undef PM_STAGE
  return hipGetLastError();
}

hipError_t launch_pointwise(int kind, const uint64_t* A, const uint64_t* B, uint64_t* C, uint32_t log2n,
                            uint32_t polys, uint32_t limbs, const LimbSet& ls, hipStream_t s) {
  const size_t N = (size_t)1 << log2n;
  dim3 grid((uint32_t)((N + 255) / 256), polys, limbs);
  if (kind == KIND_WIDE) hipLaunchKernelGGL((k_pointwise<KIND_WIDE>), grid, dim3(256), 0, s, A, B, C, log2n, polys, ls);
  else hipLaunchKernelGGL((k_pointwise<KIND_ANY>), grid, dim3(256), 0, s, A, B, C, log2n, polys, ls);
  return hipGetLastError();
}

}  // namespace pm
