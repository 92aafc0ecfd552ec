// Pass plan per transform size: how an N-point transform is split into a
// column pass (R = 2^logr rows) and a row pass (rows of C = 2^logc words).
// R = 1 means a single row pass holds the whole polynomial. The defaults can
// be replaced per (operation, N) at run time (pm_tune_set), which is how the
// autotuner installs its choices.
#pragma once
#include <stddef.h>
#include <stdint.h>

namespace pm {

constexpr unsigned PM_MAX_LOG2N = 17;
constexpr unsigned PM_MAX_LOGC = 14;     // largest row held in one workgroup's LDS
constexpr unsigned PM_MAX_LOGR = 5;      // largest column radix held in registers
// column radices of the four-word column pass (small-batch plans)
constexpr unsigned PM_COLQ_MIN_LOGR = 2;
constexpr unsigned PM_COLQ_MAX_LOGR = 7;

enum { OP_NTT_FWD = 0, OP_NTT_INV = 1, OP_POLYMUL = 2, OP_COUNT = 3 };

struct PassPlan {
  uint32_t logc, logr, R;
  uint32_t ebx;    // row pass: log2 words per thread (4, or 2 for the small-batch geometry)
};

// The throughput plan (16 words per thread).
PassPlan plan_for(int op, unsigned log2n);
// The plan for a call over batch_words = N * limbs * polys words: the
// small-batch plan of (op, log2n) if one is installed and batch_words is at
// most its limit (the per-(op, log2n) limit if set, else the global
// small-batch threshold), else the throughput plan.
PassPlan plan_for(int op, unsigned log2n, size_t batch_words);
// Returns false if (op, log2n, logc) is not a valid split.
bool plan_set(int op, unsigned log2n, unsigned logc);
// Small-batch plan: logc = 0 removes it; ebx in {2, 4}. ebx = 4 takes the
// throughput splits; ebx = 2 needs 5 <= logc <= 12 and a column radix of
// 2^2..2^7 (2^1 with >= 256 columns). Returns false for an invalid split.
bool plan_small_set(int op, unsigned log2n, unsigned logc, unsigned ebx);
bool plan_small_get(int op, unsigned log2n, unsigned* logc, unsigned* ebx);
void plan_small_threshold_set(size_t words);
size_t plan_small_threshold();
// Per (op, log2n) batch limit of the small-batch plan (0 = the global
// threshold above); false for an invalid (op, log2n).
bool plan_small_limit_set(int op, unsigned log2n, size_t words);
size_t plan_small_limit(int op, unsigned log2n);
// Limb chunks of the software-pipelined product: -1 = the built-in choice,
// 0 or 1 = never pipelined, G >= 2 = G chunks (at most the launch group's limbs).
void plan_pipe_set(int chunks);
int plan_pipe();
// Rows of 2^12 words from which the default pipelines a launch group, per
// column radix 2^logr (3..5); 0 = the built-in value. False for other logr.
bool plan_pipe_rows_set(unsigned logr, size_t min_rows);
size_t plan_pipe_rows(unsigned logr);     // the threshold in effect

}  // namespace pm
