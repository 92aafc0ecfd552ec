// Job table of the batched entry points (pm_plan_*, pm_polymul_jobs): one
// device record per job (a group of polynomial pairs sharing N and q), plus
// per-phase maps from work item to job.
#pragma once
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

}  // namespace pm
