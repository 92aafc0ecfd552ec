// Pass-plan table (see pm_plan.hpp).
#include "pm_plan.hpp"

#include <atomic>

#include "../../include/pm.h"

namespace pm {

namespace {

// logc per (op, log2n); 0 = use the default rule.
std::atomic<uint32_t> g_logc[OP_COUNT][PM_MAX_LOG2N + 1];
// small-batch plans: logc | ebx << 8 per (op, log2n); 0 = none installed
std::atomic<uint32_t> g_small[OP_COUNT][PM_MAX_LOG2N + 1];
std::atomic<size_t> g_small_words{0};
// per (op, log2n) batch limit of the small-batch plan; 0 = g_small_words
std::atomic<size_t> g_small_limit[OP_COUNT][PM_MAX_LOG2N + 1];
std::atomic<int> g_pipe{-1};

bool valid_split(unsigned log2n, unsigned logc) {
  if (logc > log2n || logc > PM_MAX_LOGC || log2n - logc > PM_MAX_LOGR) return false;
  if (logc < log2n && logc < 8) return false;   // column pass needs >= 256 columns
  return true;
}

// The small-batch geometry: rows of 2^5..2^12 words; a column pass of
// 2^2..2^7 rows runs with four words per thread (any number of columns), a
// column pass of 2 rows with one thread per column (>= 256 columns).
bool valid_small_split(unsigned log2n, unsigned logc) {
  if (logc < 5 || logc > 12 || logc > log2n) return false;
  const unsigned logr = log2n - logc;
  if (logr == 1) return logc >= 8;
  return logr <= PM_COLQ_MAX_LOGR;
}

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
  if (!valid_split(log2n, logc)) return false;
  g_logc[op][log2n].store(logc);
  return true;
}

bool plan_small_set(int op, unsigned log2n, unsigned logc, unsigned ebx) {
  if (op < 0 || op >= OP_COUNT || log2n < 1 || log2n > PM_MAX_LOG2N) return false;
  if (logc == 0) { g_small[op][log2n].store(0); return true; }
  if (ebx != 2 && ebx != 4) return false;
  if (ebx == 4 && !valid_split(log2n, logc)) return false;
  if (ebx == 2 && !valid_small_split(log2n, logc)) return false;
  g_small[op][log2n].store(logc | (ebx << 8));
  return true;
}

bool plan_small_get(int op, unsigned log2n, unsigned* logc, unsigned* ebx) {
  if (op < 0 || op >= OP_COUNT || log2n < 1 || log2n > PM_MAX_LOG2N) return false;
  const uint32_t v = g_small[op][log2n].load();
  *logc = v & 0xff;
  *ebx = v ? v >> 8 : 0;
  return true;
}

void plan_small_threshold_set(size_t words) { g_small_words.store(words); }
size_t plan_small_threshold() { return g_small_words.load(); }

bool plan_small_limit_set(int op, unsigned log2n, size_t words) {
  if (op < 0 || op >= OP_COUNT || log2n < 1 || log2n > PM_MAX_LOG2N) return false;
  g_small_limit[op][log2n].store(words);
  return true;
}

void plan_pipe_set(int chunks) { g_pipe.store(chunks < 0 ? -1 : chunks); }
int plan_pipe() { return g_pipe.load(); }

namespace {
// built-in thresholds, from a sweep of batch sizes on MI355X (2^15..2^17):
// at 2^17 the three passes are the faster form at every batch size
constexpr size_t PIPE_MIN_ROWS_DEFAULT[3] = {2048, 2048, SIZE_MAX};
std::atomic<size_t> g_pipe_rows[3] = {{0}, {0}, {0}};
}  // namespace

bool plan_pipe_rows_set(unsigned logr, size_t min_rows) {
  if (logr < 3 || logr > 5) return false;
  g_pipe_rows[logr - 3].store(min_rows);
  return true;
}

size_t plan_pipe_rows(unsigned logr) {
  if (logr < 3 || logr > 5) return 0;
  const size_t v = g_pipe_rows[logr - 3].load();
  return v ? v : PIPE_MIN_ROWS_DEFAULT[logr - 3];
}

size_t plan_small_limit(int op, unsigned log2n) {
  if (op < 0 || op >= OP_COUNT || log2n < 1 || log2n > PM_MAX_LOG2N) return 0;
  return g_small_limit[op][log2n].load();
}

PassPlan plan_for(int op, unsigned log2n) {
  uint32_t logc = g_logc[op][log2n].load();
  if (logc == 0) logc = default_logc(op, log2n);
  PassPlan p;
  p.logc = logc;
  p.logr = log2n - logc;
  p.R = 1u << p.logr;
  p.ebx = 4;
  return p;
}

PassPlan plan_for(int op, unsigned log2n, size_t batch_words) {
  const size_t limit = g_small_limit[op][log2n].load();
  if (batch_words <= (limit ? limit : g_small_words.load())) {
    const uint32_t v = g_small[op][log2n].load();
    if (v) {
      PassPlan p;
      p.logc = v & 0xff;
      p.logr = log2n - p.logc;
      p.R = 1u << p.logr;
      p.ebx = v >> 8;
      return p;
    }
  }
  return plan_for(op, log2n);
}

}  // namespace pm

extern "C" int pm_tune_set(int op, unsigned log2n, unsigned logc) {
  return pm::plan_set(op, log2n, logc) ? PM_OK : PM_EINVAL;
}

extern "C" int pm_tune_get(int op, unsigned log2n) {
  if (op < 0 || op >= pm::OP_COUNT || log2n < 1 || log2n > pm::PM_MAX_LOG2N) return PM_EINVAL;
  return (int)pm::plan_for(op, log2n).logc;
}

extern "C" int pm_tune_set_small(int op, unsigned log2n, unsigned logc, unsigned words_per_thread) {
  const unsigned ebx = words_per_thread == 4 ? 2 : words_per_thread == 16 ? 4 : 0;
  if (logc != 0 && ebx == 0) return PM_EINVAL;
  return pm::plan_small_set(op, log2n, logc, ebx) ? PM_OK : PM_EINVAL;
}

extern "C" int pm_tune_get_small(int op, unsigned log2n, unsigned* logc, unsigned* words_per_thread) {
  unsigned l, e;
  if (!logc || !words_per_thread || !pm::plan_small_get(op, log2n, &l, &e)) return PM_EINVAL;
  *logc = l;
  *words_per_thread = e ? (1u << e) : 0;
  return PM_OK;
}

extern "C" int pm_tune_set_small_batch(size_t max_words) {
  pm::plan_small_threshold_set(max_words);
  return PM_OK;
}

extern "C" size_t pm_tune_get_small_batch(void) { return pm::plan_small_threshold(); }

extern "C" int pm_tune_set_small_limit(int op, unsigned log2n, size_t max_words) {
  return pm::plan_small_limit_set(op, log2n, max_words) ? PM_OK : PM_EINVAL;
}

extern "C" size_t pm_tune_get_small_limit(int op, unsigned log2n) { return pm::plan_small_limit(op, log2n); }

extern "C" int pm_tune_set_pipeline(int chunks) {
  pm::plan_pipe_set(chunks);
  return PM_OK;
}

extern "C" int pm_tune_get_pipeline(void) { return pm::plan_pipe(); }

extern "C" int pm_tune_set_pipeline_rows(unsigned logr, size_t min_rows) {
  return pm::plan_pipe_rows_set(logr, min_rows) ? PM_OK : PM_EINVAL;
}

extern "C" size_t pm_tune_get_pipeline_rows(unsigned logr) { return pm::plan_pipe_rows(logr); }
