// Job-table kernels: the three passes of Eq. 2 over a batch of jobs with
// mixed N and moduli, one launch per pass (blockIdx.x = work item).
//
//   k_jobs_col<FWD>  first log2 R stages of Alg. 5 on the columns of a and b
//   k_jobs_row<11>   rows of up to 2^11 words: rows of a split, or several
//                    whole small polynomials per workgroup
//   k_jobs_row<12>   rows of 2^12 words (the R x 2^12 split, or N = 2^12)
//   k_jobs_row<13|14> rows of 2^13 / 2^14 words (tuned splits only)
//   k_jobs_col<INV>  last log2 R stages of Alg. 6 on the columns of c
//   k_jobs_pipe      the software-pipelined form: rows of 2^12 words of one
//                    chunk of products beside the column passes of its
//                    neighbours, any N = 2^12..2^17 in one launch
#include "ntt_row.hpp"
#include "pm_jobs.hpp"

namespace pm {

// The pointers of a job record address global memory, but loaded from the
// table they are generic pointers, which the compiler can only dereference
// with flat instructions: 64-bit addresses in VGPRs, and every flat load
// also counts against the LDS wait counter, so each LDS exchange of the row
// code would wait for the loads in flight. Rebuilt from their integer value
// in the global address space they get global loads and stores with a
// scalar base and a 32-bit lane offset.
template <typename T>
__device__ __forceinline__ T* gmem(T* p) {
  return (T*)(__attribute__((address_space(1))) T*)(uintptr_t)p;
}

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
  const uint64_t* src = INV ? gmem(J.c) : (op ? gmem(J.b) : gmem(J.a));
  uint64_t* dst = INV ? gmem(J.c) : (op ? gmem(J.wb) : gmem(J.c));
  const uint64_t* tw = INV ? gmem(J.ti) : gmem(J.tf);
  switch (J.logr) {
    case 1: col_task<1, KIND, INV>(src + off, dst + off, C, tw, J.mod); break;
    case 2: col_task<2, KIND, INV>(src + off, dst + off, C, tw, J.mod); break;
    case 3: col_task<3, KIND, INV>(src + off, dst + off, C, tw, J.mod); break;
    case 4: col_task<4, KIND, INV>(src + off, dst + off, C, tw, J.mod); break;
    case 5: col_task<5, KIND, INV>(src + off, dst + off, C, tw, J.mod); break;
    default: break;
  }
}

// One work item = one group of ROWS row tasks of one job. LOGR >= 0 fixes
// the job's column radix at compile time (rows of 2^12 words).
template <int LOGC, int KIND, int LOGR = -1>
__device__ __forceinline__ void job_row(const JobDev& J, uint32_t group, uint64_t* lds_all) {
  using G = RowGeom<LOGC>;
  const uint32_t sub = threadIdx.x >> G::LOGT;
  const uint32_t t = threadIdx.x & (G::T - 1);
  const uint32_t R = LOGR >= 0 ? (1u << LOGR) : (1u << J.logr);
  const uint32_t task = group * G::ROWS + sub;
  // one row per workgroup: the map lists exactly the job's row tasks
  const bool active = G::ROWS == 1 || task < J.count * R;
  const uint32_t r = task & (R - 1);
  const size_t off = (size_t)task << LOGC;
  const uint64_t* A = (R > 1) ? gmem(J.c) : gmem(J.a);
  const uint64_t* B = (R > 1) ? gmem(J.wb) : gmem(J.b);
  uint64_t* Cp = gmem(J.c);
  const uint64_t* tf = gmem(J.tf);
  const uint64_t* ti = gmem(J.ti);
  const Mod M = J.mod;
  row_task<LOGC, KIND, ROW_MUL>(A + off, B + off, Cp + off, tf, ti, R + r, active, M,
                                lds_all + (G::NR > 1 ? sub * G::LDS_ROW : 0), t);
}

// Row kernels per map group: MAXLOGC = 11 takes every row length up to 2^11
// (several rows or whole small polynomials per workgroup), 12 exactly rows of
// 2^12 words with the radix dispatched to compile-time instances (which fit
// 4 waves per SIMD), 13 and 14 the tuned long rows.
template <int MAXLOGC>
struct JobRowGeo {
  static constexpr int geo = MAXLOGC == 11 ? 12 : MAXLOGC;   // sizes the workgroup and its LDS
  static constexpr int waves = MAXLOGC == 12 ? 4 : 3;
};

template <int KIND, int MAXLOGC>
__global__ void __launch_bounds__(RowGeom<JobRowGeo<MAXLOGC>::geo>::WG)
__attribute__((amdgpu_waves_per_eu(JobRowGeo<MAXLOGC>::waves, 8)))
k_jobs_row(const JobDev* __restrict__ jobs, const uint32_t* __restrict__ item_job) {
  __shared__ uint64_t lds[RowGeom<JobRowGeo<MAXLOGC>::geo>::LDS_WORDS];
  const uint32_t item = blockIdx.x;
  const JobDev& J = jobs[item_job[item]];
  const uint32_t group = item - J.first[PH_ROW];
  if constexpr (MAXLOGC == 11) {
    switch (J.logc) {
#define PM_JR(L) case L: job_row<L, KIND>(J, group, lds); break;
      PM_JR(1) PM_JR(2) PM_JR(3) PM_JR(4) PM_JR(5) PM_JR(6) PM_JR(7) PM_JR(8) PM_JR(9) PM_JR(10) PM_JR(11)
#undef PM_JR
      default: break;
    }
  } else if constexpr (MAXLOGC == 12) {
    switch (J.logr) {
#define PM_JR(R) case R: job_row<12, KIND, R>(J, group, lds); break;
      PM_JR(0) PM_JR(1) PM_JR(2) PM_JR(3) PM_JR(4) PM_JR(5)
#undef PM_JR
      default: break;
    }
  } else {
    job_row<MAXLOGC, KIND>(J, group, lds);
  }
}

// Row work item of the pipelined table: row `local` of the job's products,
// the radix fixed at compile time (R = 2^LOGR, rows of 2^12 words).
template <int KIND, int LOGR>
__device__ __forceinline__ void pipe_row(const JobDev& J, uint32_t local, uint64_t* lds, uint32_t t) {
  constexpr uint32_t R = 1u << LOGR;
  const uint32_t poly = local >> LOGR, row = local & (R - 1);
  const size_t off = ((size_t)poly << (12 + LOGR)) + ((size_t)row << 12);
  const uint64_t* A = (R > 1) ? gmem(J.c) : gmem(J.a);
  const uint64_t* B = (R > 1) ? gmem(J.wb) : gmem(J.b);
  uint64_t* Cp = gmem(J.c);
  const uint64_t* tf = gmem(J.tf);
  const uint64_t* ti = gmem(J.ti);
  const Mod M = J.mod;
  row_task<12, KIND, ROW_MUL>(A + off, B + off, Cp + off, tf, ti, R + row, true, M, lds, t);
}

// Column work item of the pipelined table: radix R = 2^logr chosen per job;
// pipe_col_blocks(logr) items per operand of a product (a 32-word column is
// held by the lanes l and l + 32 of a wave, 16 words each).
template <int KIND, int INV>
__device__ __forceinline__ void pipe_col32(const JobDev& J, uint32_t local, uint32_t t) {
  const uint32_t cb = local % pipe_col_blocks(5), rest = local / pipe_col_blocks(5);
  const uint32_t nops = INV ? 1u : J.nops;
  const uint32_t poly = rest / nops, op = rest % nops;
  const uint32_t lane = t & 63, h = lane >> 5;
  const size_t off = ((size_t)poly << J.log2n) + (size_t)cb * 128 + (t >> 6) * 32 + (lane & 31);
  const uint64_t* src = (INV ? gmem(J.c) : (op ? gmem(J.b) : gmem(J.a))) + off;
  uint64_t* dst = (INV ? gmem(J.c) : (op ? gmem(J.wb) : gmem(J.c))) + off;
  const uint64_t* tw = INV ? gmem(J.ti) : gmem(J.tf);
  const Mod M = J.mod;
  constexpr size_t C = 4096;
  uint64_t y[16];
  if (INV) {
#pragma unroll
    for (int j = 0; j < 16; ++j) y[j] = src[col32_block_row(j, h) * C];
    col32_inv_pair<KIND>(y, tw, h, M);
#pragma unroll
    for (int j = 0; j < 16; ++j) dst[col32_split_row(j, h) * C] = y[j];
  } else {
#pragma unroll
    for (int j = 0; j < 16; ++j) y[j] = src[col32_split_row(j, h) * C];
    col32_fwd_pair<KIND>(y, tw, h, M);
#pragma unroll
    for (int j = 0; j < 16; ++j) dst[col32_block_row(j, h) * C] = y[j];
  }
}

template <int KIND, int INV>
__device__ __forceinline__ void pipe_col(const JobDev& J, uint32_t local, uint32_t t) {
  if (J.logr == 5) {
    pipe_col32<KIND, INV>(J, local, t);
    return;
  }
  const uint32_t cb = local & 15, rest = local >> 4;    // 16 blocks of 256 columns per operand
  const uint32_t nops = INV ? 1u : J.nops;
  const uint32_t poly = rest / nops, op = rest % nops;  // product-major: a product's operands stay together
  const size_t off = ((size_t)poly << J.log2n) + (size_t)cb * 256 + t;
  const uint64_t* src = INV ? gmem(J.c) : (op ? gmem(J.b) : gmem(J.a));
  uint64_t* dst = INV ? gmem(J.c) : (op ? gmem(J.wb) : gmem(J.c));
  const uint64_t* tw = INV ? gmem(J.ti) : gmem(J.tf);
  constexpr size_t C = 4096;
  static_assert(pipe_col_blocks(4) == 16, "16 blocks of 256 columns per operand");
  switch (J.logr) {
    case 1: col_task<1, KIND, INV>(src + off, dst + off, C, tw, J.mod); break;
    case 2: col_task<2, KIND, INV>(src + off, dst + off, C, tw, J.mod); break;
    case 3: col_task<3, KIND, INV>(src + off, dst + off, C, tw, J.mod); break;
    case 4: col_task<4, KIND, INV>(src + off, dst + off, C, tw, J.mod); break;
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
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8)))
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
    switch (J.logr) {
#define PM_PR(R) case R: pipe_row<KIND, R>(J, local, lds, t); break;
      PM_PR(0) PM_PR(1) PM_PR(2) PM_PR(3) PM_PR(4) PM_PR(5)
#undef PM_PR
      default: break;
    }
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
  } else if (maxlogc == 11) {
    if (w) hipLaunchKernelGGL((k_jobs_row<KIND_WIDE, 11>), grid, dim3(256), 0, s, jobs, item_job);
    else hipLaunchKernelGGL((k_jobs_row<KIND_ANY, 11>), grid, dim3(256), 0, s, jobs, item_job);
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
