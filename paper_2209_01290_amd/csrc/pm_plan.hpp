// Pass plan per transform size: how an N-point transform is split into a
// column pass (R = 2^logr rows) and a row pass (rows of C = 2^logc words).
// R = 1 means a single row pass holds the whole polynomial. The defaults can
// be replaced per (operation, N) at run time (pm_tune_set), which is how the
// autotuner installs its choices.
#pragma once
#include <stdint.h>

namespace pm {

constexpr unsigned PM_MAX_LOG2N = 17;
constexpr unsigned PM_MAX_LOGC = 14;     // largest row held in one workgroup's LDS
constexpr unsigned PM_MAX_LOGR = 5;      // largest column radix held in registers

enum { OP_NTT_FWD = 0, OP_NTT_INV = 1, OP_POLYMUL = 2, OP_COUNT = 3 };

struct PassPlan {
  uint32_t logc, logr, R;
};

PassPlan plan_for(int op, unsigned log2n);
// Returns false if (op, log2n, logc) is not a valid split.
bool plan_set(int op, unsigned log2n, unsigned logc);

}  // namespace pm
