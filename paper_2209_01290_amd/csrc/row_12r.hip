// Row pass of the product (Eq. 2 and the fused Alg. 8 rows) for rows of
// 2^12 words, 64-bit words and moduli of 34..61 bits (KIND_WIDE, every
// 60-bit NTT prime), with the column radix R = 2^LOGR of the split
// (N = R * 2^12) fixed at compile time. With R, N and the row's twiddle
// offsets known to the compiler, the product's row code fits 4 waves per
// SIMD without spills (114-128 VGPRs), where the generic k_row<12> for any R
// takes 159 and runs 3. One row per workgroup of 256 threads; grid x = row
// task (poly * R + r), y = limb.
#include "ntt_row.hpp"
#include "pm_internal.hpp"

namespace pm {
namespace {

using RG = RowGeom<12>;
static_assert(RG::WG == 256 && RG::ROWS == 1, "one 2^12-word row per workgroup of 256 threads");

template <int KIND, int MODE, int LOGR>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8)))
k_row_r(const uint64_t* A, const uint64_t* B, uint64_t* Cout, const uint64_t* twf, const uint64_t* twi,
        uint32_t polys, LimbSet ls) {
  __shared__ uint64_t lds[RG::LDS_WORDS];
  constexpr uint32_t R = 1u << LOGR;
  constexpr size_t N = (size_t)1 << (12 + LOGR);
  const uint32_t limb = blockIdx.y, task = blockIdx.x, t = threadIdx.x;
  const uint32_t r = task & (R - 1);
  const size_t off = (size_t)limb * polys * N + ((size_t)task << 12);
  const Mod M = ls.mod[limb];
  row_task<12, KIND, MODE>(A + off, B + off, Cout + off, twf + limb * N, twi + limb * N, R + r, true, M, lds, t);
}

template <int KIND, int MODE, int LOGR>
void launch_r(const RowArgs& a, hipStream_t s) {
  dim3 grid(a.polys << LOGR, a.limbs);
  hipLaunchKernelGGL((k_row_r<KIND, MODE, LOGR>), grid, dim3(256), 0, s, a.A, a.B, a.C, a.twf, a.twi, a.polys,
                     *a.ls);
}

template <int KIND, int MODE>
bool launch_mode(const RowArgs& a, hipStream_t s) {
  switch (a.log2n) {
    case 12: launch_r<KIND, MODE, 0>(a, s); return true;
    case 13: launch_r<KIND, MODE, 1>(a, s); return true;
    case 14: launch_r<KIND, MODE, 2>(a, s); return true;
    case 15: launch_r<KIND, MODE, 3>(a, s); return true;
    case 16: launch_r<KIND, MODE, 4>(a, s); return true;
    case 17: launch_r<KIND, MODE, 5>(a, s); return true;
    default: return false;
  }
}

}  // namespace

bool launch_row12_fixed(int kind, int mode, const RowArgs& a, hipStream_t s) {
  if (kind != KIND_WIDE || a.log2n < 12 || a.log2n > 17 || a.R != (1u << (a.log2n - 12)) ||
      (uint64_t)a.polys * a.R >= (1ull << 31))
    return false;
  if (mode == ROW_MUL) return launch_mode<KIND_WIDE, ROW_MUL>(a, s);
  if (mode == ROW_FMUL) return launch_mode<KIND_WIDE, ROW_FMUL>(a, s);
  return false;
}

}  // namespace pm
