// Job-table kernels: the three passes of Eq. 2 over a batch of jobs with
// mixed N and moduli, one launch per pass (blockIdx.x = work item).
//
//   k_jobs_col<FWD>  first log2 R stages of Alg. 5 on the columns of a and b
//   k_jobs_row<12>   rows of up to 2^12 words: rows of the R x 2^12 split,
//                    or several whole small polynomials per workgroup
//   k_jobs_row<13|14> rows of 2^13 / 2^14 words (tuned splits only)
//   k_jobs_col<INV>  last log2 R stages of Alg. 6 on the columns of c
//   k_jobs_pipe      the software-pipelined form: rows of 2^12 words of one
//                    chunk of products beside the column passes of its
//                    neighbours, any N = 2^12..2^17 in one launch
#include "ntt_row.hpp"
#include "pm_jobs.hpp"

namespace pm {

template <int LOGR, int KIND, int INV>
__device__ __forceinline__ void col_task(const uint64_t* src, uint64_t* dst, size_t C, const uint64_t* __restrict__ tw,
                                         const Mod& M) {
  constexpr int R = 1 << LOGR;
  uint64_t x[R];
#pragma unroll
  for (int i = 0; i < R; ++i) x[i] = src[i * C];
  if (INV) col_inv<LOGR, KIND>(x, tw, M);
  else col_fwd<LOGR, KIND>(x, tw, M);
#pragma unroll
  for (int i = 0; i < R; ++i) dst[i * C] = x[i];
}

template <int KIND, int INV>
__global__ void __launch_bounds__(256) k_jobs_col(const JobDev* __restrict__ jobs, const uint32_t* __restrict__ item_job) {
  const uint32_t item = blockIdx.x;
  const JobDev& J = jobs[item_job[item]];
  const uint32_t local = item - J.first[INV ? PH_COLI : PH_COLF];
  const uint32_t cbs = 1u << (J.logc - 8);            // blocks of 256 columns per polynomial
  const uint32_t cb = local & (cbs - 1), rest = local >> (J.logc - 8);
  const uint32_t poly = rest % J.count, op = rest / J.count;
  const size_t N = (size_t)1 << J.log2n, C = (size_t)1 << J.logc;
  const size_t off = (size_t)poly * N + (size_t)cb * 256 + threadIdx.x;
  const uint64_t* src = INV ? J.c : (op ? J.b : J.a);
  uint64_t* dst = INV ? J.c : (op ? J.wb : J.c);
  const uint64_t* tw = INV ? J.ti : J.tf;
  switch (J.logr) {
    case 1: col_task<1, KIND, INV>(src + off, dst + off, C, tw, J.mod); break;
    case 2: col_task<2, KIND, INV>(src + off, dst + off, C, tw, J.mod); break;
    case 3: col_task<3, KIND, INV>(src + off, dst + off, C, tw, J.mod); break;
    case 4: col_task<4, KIND, INV>(src + off, dst + off, C, tw, J.mod); break;
    case 5: col_task<5, KIND, INV>(src + off, dst + off, C, tw, J.mod); break;
    default: break;
  }
}

// One work item = one group of ROWS row tasks of one job.
template <int LOGC, int KIND>
__device__ __forceinline__ void job_row(const JobDev& J, uint32_t group, uint64_t* lds_all) {
  using G = RowGeom<LOGC>;
  const uint32_t sub = threadIdx.x >> G::LOGT;
  const uint32_t t = threadIdx.x & (G::T - 1);
  const uint32_t R = 1u << J.logr;
  const uint32_t task = group * G::ROWS + sub;
  const bool active = task < J.count * R;
  const uint32_t r = task & (R - 1);
  const size_t off = (size_t)task << LOGC;
  const uint64_t* A = (R > 1) ? J.c : J.a;
  const uint64_t* B = (R > 1) ? J.wb : J.b;
  row_task<LOGC, KIND, ROW_MUL>(A + off, B + off, J.c + off, J.tf, J.ti, R + r, active, J.mod,
                                lds_all + (G::NR > 1 ? sub * G::LDS_ROW : 0), t);
}

template <int KIND, int MAXLOGC>
__global__ void __launch_bounds__(RowGeom<MAXLOGC>::WG) __attribute__((amdgpu_waves_per_eu(3, 8)))
k_jobs_row(const JobDev* __restrict__ jobs, const uint32_t* __restrict__ item_job) {
  __shared__ uint64_t lds[RowGeom<MAXLOGC>::LDS_WORDS];
  const uint32_t item = blockIdx.x;
  const JobDev& J = jobs[item_job[item]];
  const uint32_t group = item - J.first[PH_ROW];
  if constexpr (MAXLOGC == 12) {
    switch (J.logc) {
#define PM_JR(L) case L: job_row<L, KIND>(J, group, lds); break;
      PM_JR(1) PM_JR(2) PM_JR(3) PM_JR(4) PM_JR(5) PM_JR(6) PM_JR(7) PM_JR(8) PM_JR(9) PM_JR(10) PM_JR(11)
      PM_JR(12)
#undef PM_JR
      default: break;
    }
  } else {
    job_row<MAXLOGC, KIND>(J, group, lds);
  }
}

// Column work item of the pipelined table: radix R = 2^logr chosen per job.
template <int KIND, int INV>
__device__ __forceinline__ void pipe_col(const JobDev& J, uint32_t local, uint32_t t) {
  const uint32_t cb = local & 15, rest = local >> 4;    // 16 blocks of 256 columns per operand
  const uint32_t nops = INV ? 1u : J.nops;
  const uint32_t poly = rest / nops, op = rest % nops;  // product-major: a product's operands stay together
  const size_t off = ((size_t)poly << J.log2n) + (size_t)cb * 256 + t;
  const uint64_t* src = INV ? J.c : (op ? J.b : J.a);
  uint64_t* dst = INV ? J.c : (op ? J.wb : J.c);
  const uint64_t* tw = INV ? J.ti : J.tf;
  constexpr size_t C = 4096;
  switch (J.logr) {
    case 1: col_task<1, KIND, INV>(src + off, dst + off, C, tw, J.mod); break;
    case 2: col_task<2, KIND, INV>(src + off, dst + off, C, tw, J.mod); break;
    case 3: col_task<3, KIND, INV>(src + off, dst + off, C, tw, J.mod); break;
    case 4: col_task<4, KIND, INV>(src + off, dst + off, C, tw, J.mod); break;
    case 5: col_task<5, KIND, INV>(src + off, dst + off, C, tw, J.mod); break;
    default: break;
  }
}

// The software-pipelined job table (see pipe_kernels.hip for the schedule):
// every job here has N = 2^12..2^17 and is split into R = N / 2^12 rows of
// 2^12 words. One launch runs, in this order of workgroups, the rows of one
// chunk of products (forward rows of a and b, product, inverse rows), the
// forward column pass of the next chunk and the inverse column pass of the
// chunk before; chunks are ranges of the table's products, whose row and
// column items are contiguous in the maps. All rows run the same code, so a
// launch mixes sizes and moduli freely.
template <int KIND>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8)))
k_jobs_pipe(const JobDev* __restrict__ jobs, const uint32_t* __restrict__ map_row,
            const uint32_t* __restrict__ map_colf, const uint32_t* __restrict__ map_coli, JobsPipeLaunch L) {
  using G = RowGeom<12>;
  static_assert(G::WG == 256 && G::ROWS == 1, "one 2^12-word row per workgroup of 256 threads");
  __shared__ uint64_t lds[G::LDS_WORDS];
  const uint32_t b = blockIdx.x, t = threadIdx.x;
  if (b < L.nr) {
    const uint32_t item = L.r0 + b;
    const JobDev& J = jobs[map_row[item]];
    const uint32_t local = item - J.first[PH_ROW];
    const uint32_t R = 1u << J.logr;
    const uint32_t poly = local >> J.logr, row = local & (R - 1);
    const size_t off = ((size_t)poly << J.log2n) + ((size_t)row << 12);
    const uint64_t* A = (R > 1) ? J.c : J.a;
    const uint64_t* B = (R > 1) ? J.wb : J.b;
    row_task<12, KIND, ROW_MUL>(A + off, B + off, J.c + off, J.tf, J.ti, R + row, true, J.mod, lds, t);
    return;
  }
  if (b < L.nr + L.nf) {
    const uint32_t item = L.f0 + (b - L.nr);
    const JobDev& J = jobs[map_colf[item]];
    pipe_col<KIND, 0>(J, item - J.first[PH_COLF], t);
  } else {
    const uint32_t item = L.i0 + (b - L.nr - L.nf);
    const JobDev& J = jobs[map_coli[item]];
    pipe_col<KIND, 1>(J, item - J.first[PH_COLI], t);
  }
}

hipError_t launch_jobs_pipe(int kind, const JobDev* jobs, const uint32_t* map_row, const uint32_t* map_colf,
                            const uint32_t* map_coli, const JobsPipeLaunch& L, hipStream_t s) {
  const uint32_t blocks = L.nr + L.nf + L.ni;
  if (blocks == 0) return hipSuccess;
  if (kind == KIND_WIDE)
    hipLaunchKernelGGL((k_jobs_pipe<KIND_WIDE>), dim3(blocks), dim3(256), 0, s, jobs, map_row, map_colf, map_coli, L);
  else
    hipLaunchKernelGGL((k_jobs_pipe<KIND_ANY>), dim3(blocks), dim3(256), 0, s, jobs, map_row, map_colf, map_coli, L);
  return hipGetLastError();
}

hipError_t launch_jobs(int phase, int maxlogc, int kind, const JobDev* jobs, const uint32_t* item_job,
                       uint32_t nitems, hipStream_t s) {
  if (nitems == 0) return hipSuccess;
  dim3 grid(nitems);
  const bool w = kind == KIND_WIDE;
  if (phase == PH_COLF || phase == PH_COLI) {
    const bool inv = phase == PH_COLI;
    if (w && !inv) hipLaunchKernelGGL((k_jobs_col<KIND_WIDE, 0>), grid, dim3(256), 0, s, jobs, item_job);
    else if (w) hipLaunchKernelGGL((k_jobs_col<KIND_WIDE, 1>), grid, dim3(256), 0, s, jobs, item_job);
    else if (!inv) hipLaunchKernelGGL((k_jobs_col<KIND_ANY, 0>), grid, dim3(256), 0, s, jobs, item_job);
    else hipLaunchKernelGGL((k_jobs_col<KIND_ANY, 1>), grid, dim3(256), 0, s, jobs, item_job);
  } else if (maxlogc == 12) {
    if (w) hipLaunchKernelGGL((k_jobs_row<KIND_WIDE, 12>), grid, dim3(256), 0, s, jobs, item_job);
    else hipLaunchKernelGGL((k_jobs_row<KIND_ANY, 12>), grid, dim3(256), 0, s, jobs, item_job);
  } else if (maxlogc == 13) {
    if (w) hipLaunchKernelGGL((k_jobs_row<KIND_WIDE, 13>), grid, dim3(512), 0, s, jobs, item_job);
    else hipLaunchKernelGGL((k_jobs_row<KIND_ANY, 13>), grid, dim3(512), 0, s, jobs, item_job);
  } else if (maxlogc == 14) {
    if (w) hipLaunchKernelGGL((k_jobs_row<KIND_WIDE, 14>), grid, dim3(1024), 0, s, jobs, item_job);
    else hipLaunchKernelGGL((k_jobs_row<KIND_ANY, 14>), grid, dim3(1024), 0, s, jobs, item_job);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace pm
