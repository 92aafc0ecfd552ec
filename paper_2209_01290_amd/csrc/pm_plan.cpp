// Pass-plan table (see pm_plan.hpp).
#include "pm_plan.hpp"

#include <atomic>

#include "../../include/pm.h"

namespace pm {

namespace {

// logc per (op, log2n); 0 = use the default rule.
std::atomic<uint32_t> g_logc[OP_COUNT][PM_MAX_LOG2N + 1];

uint32_t default_logc(int op, unsigned log2n) {
  // Rows of 2^12 words (32 KiB of LDS, 256 threads) keep four workgroups per
  // CU; a whole polynomial up to 2^13 words (fused product) or 2^14 words
  // (single transform) fits one workgroup's LDS.
  const unsigned single_max = (op == OP_POLYMUL) ? 13 : 14;
  if (log2n <= single_max) return log2n;
  return 12;
}

}  // namespace

bool plan_set(int op, unsigned log2n, unsigned logc) {
  if (op < 0 || op >= OP_COUNT || log2n < 1 || log2n > PM_MAX_LOG2N) return false;
  if (logc == 0) { g_logc[op][log2n].store(0); return true; }
  if (logc > log2n || logc > PM_MAX_LOGC || log2n - logc > PM_MAX_LOGR) return false;
  if (logc < log2n && logc < 8) return false;   // column pass needs >= 256 columns
  g_logc[op][log2n].store(logc);
  return true;
}

PassPlan plan_for(int op, unsigned log2n) {
  uint32_t logc = g_logc[op][log2n].load();
  if (logc == 0) logc = default_logc(op, log2n);
  PassPlan p;
  p.logc = logc;
  p.logr = log2n - logc;
  p.R = 1u << p.logr;
  return p;
}

}  // namespace pm

extern "C" int pm_tune_set(int op, unsigned log2n, unsigned logc) {
  return pm::plan_set(op, log2n, logc) ? PM_OK : PM_EINVAL;
}

extern "C" int pm_tune_get(int op, unsigned log2n) {
  if (op < 0 || op >= pm::OP_COUNT || log2n < 1 || log2n > pm::PM_MAX_LOG2N) return PM_EINVAL;
  return (int)pm::plan_for(op, log2n).logc;
}
