// Job table of the batched entry points (pm_plan_*, pm_polymul_jobs): one
// device record per job (a group of polynomial pairs sharing N and q), plus
// per-phase maps from work item to job.
#pragma once
#include <hip/hip_runtime.h>

#include "modarith.hpp"

namespace pm {

enum { PH_COLF = 0, PH_ROW = 1, PH_COLI = 2 };

struct JobDev {
  const uint64_t* a;       // count x N input words
  const uint64_t* b;       // count x N input words (may equal a)
  uint64_t* c;             // count x N output words (also a's column output)
  uint64_t* wb;            // b's column output (R > 1; equals c when b == a), else nullptr
  const uint64_t* tf;      // psi_br (N words)
  const uint64_t* ti;      // psi_inv_br (N words)
  Mod mod;
  uint32_t log2n, count, logc, logr;
  uint32_t nops, pad;      // operands of the forward column pass (1 or 2)
  uint32_t first[4];       // first work item of the job in each phase's numbering
};

// One launch of the software-pipelined job table (k_jobs_pipe): nr row work
// items from r0 of the row map, then nf forward-column items from f0 and ni
// inverse-column items from i0 of the column maps.
struct JobsPipeLaunch {
  uint32_t r0, nr, f0, nf, i0, ni;
};

hipError_t launch_jobs_pipe(int kind, const JobDev* jobs, const uint32_t* map_row, const uint32_t* map_colf,
                            const uint32_t* map_coli, const JobsPipeLaunch& L, hipStream_t s);

}  // namespace pm
