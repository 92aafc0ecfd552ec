/*
 * pm.h - exact negacyclic polynomial multiplication in Z_q[x]/(x^N + 1) on
 * AMD MI355X (gfx950), C ABI.
 *
 * Method (Sec. III-A of the paper, Eq. 2): c = a (*) b is computed as
 *     c = GS'_{psi^-1}( CT_psi(a) . CT_psi(b) )
 * where CT_psi is the merged Cooley-Tukey NTT (Alg. 5: normal order in,
 * bit-reversed order out, powers of psi folded into the twiddles), "." is the
 * pointwise product mod q, and GS'_{psi^-1} is the merged Gentleman-Sande NTT
 * (Alg. 6: bit-reversed in, normal out) whose butterflies halve both outputs,
 * which merges the 1/N scaling. Every product is reduced with the paper's
 * Barrett variant (Alg. 4, constant mu = floor(2^(2m+1)/q), m = len(q),
 * at most one correctional subtraction). Arithmetic is exact: every output
 * word is the canonical residue in [0, q).
 *
 * Conventions for every entry point:
 *   - Array pointers marked "device" are caller-owned device memory (e.g.
 *     torch tensors). The library never frees them. uint64 words, 8-byte
 *     aligned. Pointers marked "host" are read on the host during the call.
 *   - Batch layout is [limb][poly][N]: `limbs` moduli, each with
 *     `polys_per_limb` polynomials of N contiguous coefficients. Limb l uses
 *     modulus q[l] and twiddle tables psi_br + l*N, psi_inv_br + l*N.
 *   - Coefficient domain is normal order. The NTT domain is bit-reversed
 *     order: position p holds the value at psi^(2*br(p)+1), br over log2 N bits.
 *   - Twiddle tables: psi_br[i] = psi^br(i) and psi_inv_br[i] = psi^-br(i) for
 *     a primitive 2N-th root of unity psi (psi^N = q-1); entry 0 is never read.
 *     pm_make_tables() builds them.
 *   - Inputs must be canonical (< q); non-canonical input gives unspecified
 *     (but memory-safe) output. With the environment variable PM_VALIDATE
 *     set (to anything but "0"), every entry point that takes coefficients or
 *     twiddle tables also checks, on the device, that each input word is below
 *     its limb's modulus and that each table's entry N/2 (psi, or psi^-1 for
 *     an inverse table) satisfies psi^N = q - 1, and returns PM_EINVAL
 *     otherwise, before any output is written. These checks allocate a little
 *     device memory and synchronise the stream (a debugging aid; not for use
 *     under graph capture). pm_plan_create checks the tables, pm_plan_launch
 *     the inputs.
 *   - Calls are stream-ordered and asynchronous: `stream` is a hipStream_t
 *     (NULL = the default stream). Argument errors are reported before any
 *     work is enqueued.
 *   - Return value: PM_OK (0) or a negative PM_E* code; pm_last_error()
 *     returns a message for the calling thread. No C++ exception crosses the ABI.
 *   - Limits: N a power of two with 2 <= N <= 2^17; q odd with
 *     3 <= q < 2^62 (Alg. 4 needs len(q) <= word size - 2) and 2N | q - 1
 *     (the NTT setup of Sec. III-A).
 */
#ifndef PM_H
#define PM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PM_OK 0
#define PM_EINVAL (-1)        /* bad argument: size, modulus, pointer, alignment */
#define PM_EUNSUPPORTED (-2)  /* valid request outside what this build implements */
#define PM_ENOMEM (-3)        /* a device allocation made by the library failed */
#define PM_EHIP (-4)          /* the HIP runtime reported an error */

typedef void *pm_stream_t;    /* a hipStream_t */

/* Message describing the last error on the calling thread ("" if none). */
const char *pm_last_error(void);

/*
 * c[i] = a[i] * b[i] mod q for i < n, by Alg. 4 (Sec. II-B).
 * a, b, c: device, n words each (c may alias a or b). q: 2 <= q < 2^62.
 * Errors: PM_EINVAL for n == 0, a null or misaligned pointer, or q out of range.
 */
int pm_barrett_mulmod(const uint64_t *a, const uint64_t *b, uint64_t *c, size_t n, uint64_t q,
                      pm_stream_t stream);

/*
 * In-place forward merged CT NTT (Alg. 5) of limbs*polys_per_limb polynomials.
 * x: device [limbs][polys_per_limb][N], normal order in, bit-reversed out.
 * q: host [limbs]. psi_br: device [limbs][N].
 */
int pm_ntt_fwd(uint64_t *x, size_t N, size_t limbs, size_t polys_per_limb, const uint64_t *q,
               const uint64_t *psi_br, pm_stream_t stream);

/*
 * In-place inverse: merged GS NTT (Alg. 6) with each butterfly output halved
 * (Eq. 2), so the result includes the 1/N factor and pm_ntt_inv(pm_ntt_fwd(x))
 * = x. x: device, bit-reversed in, normal out. psi_inv_br: device [limbs][N].
 */
int pm_ntt_inv(uint64_t *x, size_t N, size_t limbs, size_t polys_per_limb, const uint64_t *q,
               const uint64_t *psi_inv_br, pm_stream_t stream);

/*
 * c = a (*) b (negacyclic) for every polynomial pair of the batch, by Eq. 2.
 * a, b, c: device [limbs][polys_per_limb][N]; c may alias a or b.
 * workspace: device, at least pm_polymul_workspace_bytes(N, limbs,
 * polys_per_limb) bytes (may be NULL when that is 0); not preserved.
 */
int pm_polymul(const uint64_t *a, const uint64_t *b, uint64_t *c, size_t N, size_t limbs,
               size_t polys_per_limb, const uint64_t *q, const uint64_t *psi_br,
               const uint64_t *psi_inv_br, void *workspace, pm_stream_t stream);

/*
 * The fused polynomial multiplication of Sec. III-B (Alg. 8): truncated merged
 * CT NTTs of a and b (last stage omitted), the last CT stages, the pointwise
 * product and the first GS stage fused into Alg. 7 on adjacent pairs (four
 * products per pair, twiddle alpha^2 = (-1)^i psi_br[N/4 + i/2]), truncated
 * merged GS NTT (first stage omitted) with halved butterflies. Same result,
 * arguments and workspace as pm_polymul; N = 2 runs the unfused product.
 */
int pm_polymul_fused(const uint64_t *a, const uint64_t *b, uint64_t *c, size_t N, size_t limbs,
                     size_t polys_per_limb, const uint64_t *q, const uint64_t *psi_br,
                     const uint64_t *psi_inv_br, void *workspace, pm_stream_t stream);

/* Workspace bytes pm_polymul and pm_polymul_fused need for this shape (0 if none). */
size_t pm_polymul_workspace_bytes(size_t N, size_t limbs, size_t polys_per_limb);

/*
 * pm_polymul without a workspace argument and without any device allocation,
 * for callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments (minus workspace), result, aliasing rules and kernels as
 * pm_polymul. The workspace lives in a fixed device array of this library,
 * PM_NOALLOC_SCRATCH_BYTES (64 MiB) per GPU, created when the library is
 * loaded on that GPU and held until the process ends; its address is looked
 * up on the first call for each device (the stream's device).
 * Limit: batches with pm_polymul_workspace_bytes(N, limbs, polys_per_limb)
 * above PM_NOALLOC_SCRATCH_BYTES return PM_EINVAL before any work is queued
 * (e.g. at most 128 products of N = 2^16, or 64 of N = 2^17, per call; batches
 * needing no workspace have no limit).
 * Every call on one GPU shares that GPU's array: calls that may overlap on one
 * GPU (several streams or threads) race and must be serialised by the caller.
 * The PM_VALIDATE scans (which allocate) and the event timer (pm_prof_*) do
 * not apply to this entry point.
 */
#define PM_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int pm_polymul_noalloc(const uint64_t *a, const uint64_t *b, uint64_t *c, size_t N, size_t limbs,
                       size_t polys_per_limb, const uint64_t *q, const uint64_t *psi_br,
                       const uint64_t *psi_inv_br, pm_stream_t stream);

/*
 * The plain per-stage path (the paper's global-memory radix-2 baseline):
 * same result and arguments as pm_polymul, computed with one kernel launch per
 * NTT stage (each launch covers a and b of every limb), one pointwise launch
 * and one launch per inverse stage, every word read from and written to HBM
 * at every stage. workspace: pm_polymul_stagewise_workspace_bytes() bytes.
 */
int pm_polymul_stagewise(const uint64_t *a, const uint64_t *b, uint64_t *c, size_t N, size_t limbs,
                         size_t polys_per_limb, const uint64_t *q, const uint64_t *psi_br,
                         const uint64_t *psi_inv_br, void *workspace, pm_stream_t stream);
size_t pm_polymul_stagewise_workspace_bytes(size_t N, size_t limbs, size_t polys_per_limb);

/* --------------------------------------------------- interleaved layout
 * The storage of the paper's throughput-optimised multi-block design
 * (Sec. V-C): the batch of one limb is an N x P matrix held coefficient-major,
 * coefficient j of polynomial p at [j * P + p] (P = polys_per_limb), so that
 * consecutive lanes read consecutive words at every stage. x, a, b, c: device
 * [limbs][N][polys_per_limb]. Same transforms, product, tables, limits,
 * aliasing, stream and error rules as pm_ntt_fwd, pm_ntt_inv and pm_polymul;
 * with polys_per_limb = 1 the layouts coincide. pm_polymul_il's workspace:
 * pm_polymul_il_workspace_bytes() bytes (NULL when 0 or when a == b).
 */
int pm_ntt_fwd_il(uint64_t *x, size_t N, size_t limbs, size_t polys_per_limb, const uint64_t *q,
                  const uint64_t *psi_br, pm_stream_t stream);
int pm_ntt_inv_il(uint64_t *x, size_t N, size_t limbs, size_t polys_per_limb, const uint64_t *q,
                  const uint64_t *psi_inv_br, pm_stream_t stream);
int pm_polymul_il(const uint64_t *a, const uint64_t *b, uint64_t *c, size_t N, size_t limbs,
                  size_t polys_per_limb, const uint64_t *q, const uint64_t *psi_br,
                  const uint64_t *psi_inv_br, void *workspace, pm_stream_t stream);
size_t pm_polymul_il_workspace_bytes(size_t N, size_t limbs, size_t polys_per_limb);

/* --------------------------------------------------------- 32-bit words
 * The paper's 30-bit NTT timings (Sec. VII, comparison table) use 32-bit words:
 * Alg. 4 with beta = 32 needs len(q) <= 30. These calls are pm_ntt_fwd,
 * pm_ntt_inv, pm_polymul and pm_polymul_fused on 32-bit words (the fused and
 * squaring rows included), with the same layouts, aliasing,
 * stream and error rules, for moduli q odd with 3 <= q < 2^30 and 2N | q - 1.
 * x, a, b, c, psi_br, psi_inv_br: device arrays of uint32_t, 4-byte aligned;
 * q: host array of limbs moduli. pm_make_tables_u32 writes the twiddle tables
 * as 32-bit words (host arrays of N words).
 */
int pm_ntt_fwd_u32(uint32_t *x, size_t N, size_t limbs, size_t polys_per_limb, const uint32_t *q,
                   const uint32_t *psi_br, pm_stream_t stream);
int pm_ntt_inv_u32(uint32_t *x, size_t N, size_t limbs, size_t polys_per_limb, const uint32_t *q,
                   const uint32_t *psi_inv_br, pm_stream_t stream);
int pm_polymul_u32(const uint32_t *a, const uint32_t *b, uint32_t *c, size_t N, size_t limbs,
                   size_t polys_per_limb, const uint32_t *q, const uint32_t *psi_br,
                   const uint32_t *psi_inv_br, void *workspace, pm_stream_t stream);
/* The fused product (Alg. 8) on 32-bit words: as pm_polymul_fused. */
int pm_polymul_fused_u32(const uint32_t *a, const uint32_t *b, uint32_t *c, size_t N, size_t limbs,
                         size_t polys_per_limb, const uint32_t *q, const uint32_t *psi_br,
                         const uint32_t *psi_inv_br, void *workspace, pm_stream_t stream);
/* Workspace bytes pm_polymul_u32 needs for this shape (0 if none). */
size_t pm_polymul_u32_workspace_bytes(size_t N, size_t limbs, size_t polys_per_limb);
int pm_make_tables_u32(uint32_t q, size_t N, uint32_t psi, uint32_t *psi_br, uint32_t *psi_inv_br);

/* ---------------------------------------------------------- batched jobs
 * A job is `count` polynomial pairs sharing N = 2^log2n and modulus q:
 * c[i] = a[i] (*) b[i] for i < count, each array count*N words (device).
 * A batch mixes jobs of any N (2..2^17) and modulus; an RNS product of L
 * limbs is L jobs. Each pass of Eq. 2 (forward columns, fused rows, inverse
 * columns) is one kernel launch over the work of all jobs of the batch.
 * Per job, c may alias a or b; buffers of different jobs must not overlap.
 */
typedef struct {
  uint32_t log2n;               /* N = 2^log2n, 1 <= log2n <= 17 */
  uint32_t count;               /* polynomial pairs of this job */
  uint64_t q;                   /* modulus, as for pm_polymul */
  const uint64_t *psi_br;       /* device, N words */
  const uint64_t *psi_inv_br;   /* device, N words */
  const uint64_t *a, *b;        /* device, count*N words each */
  uint64_t *c;                  /* device, count*N words */
} pm_job;

/*
 * One-shot form: validates the jobs, uploads a job table into `workspace`
 * (device, 256-byte aligned, at least pm_polymul_jobs_workspace_bytes()
 * bytes; it also holds intermediates) and enqueues the passes on `stream`.
 * The host job array may be reused as soon as the call returns.
 */
size_t pm_polymul_jobs_workspace_bytes(const pm_job *jobs, size_t njobs); /* 0 if invalid */
int pm_polymul_jobs(const pm_job *jobs, size_t njobs, void *workspace, size_t workspace_bytes,
                    pm_stream_t stream);

/*
 * Plan form: pm_plan_create validates the jobs, allocates the job table and
 * intermediates on the current device (pm_plan_device_bytes() bytes) and
 * captures the passes into a HIP graph; pm_plan_launch replays the graph on
 * `stream` (one graph launch per batch). The jobs' buffers must stay valid and
 * are read again at every launch. flags: PM_PLAN_NO_GRAPH launches the kernels
 * directly instead. Pass plans (pm_tune_set) are read at creation.
 */
typedef struct pm_plan pm_plan;
#define PM_PLAN_NO_GRAPH 1u
int pm_plan_create(pm_plan **plan, const pm_job *jobs, size_t njobs, unsigned flags);
int pm_plan_launch(pm_plan *plan, pm_stream_t stream);
int pm_plan_destroy(pm_plan *plan);   /* waits for the device before freeing */
size_t pm_plan_device_bytes(const pm_plan *plan);

/* ------------------------------------------------------ Barrett variant study
 * The reductions of Sec. II-B side by side: variant 2 = classical Barrett
 * (Alg. 2, up to two correctional subtractions), 3 = Dhem-Quisquater with
 * alpha = N+3, beta = -2 (Alg. 3), 4 = the proposed alpha = N+1, beta = -2
 * (Alg. 4), 0 = the built-in '%'. word_bits = 32 computes on 32-bit words
 * (len(q) <= 30; <= 28 for Alg. 3), 64 on 64-bit words (len(q) <= 62; <= 60
 * for Alg. 3). Inputs canonical (< q), stored as uint64 words either way.
 *
 * pm_reduce_apply: c[i] = a[i]*b[i] mod q and, per workgroup of 256 indices,
 * how many reductions took 0, 1 and 2 correctional subtractions:
 * hist[3*w + k] (device, 3 * ceil(n/256) uint32).
 * pm_reduce_chain: throughput probe; each of `threads` threads (a positive
 * multiple of 256) runs 8 independent chains x <- reduce(x*y) for `iters`
 * steps and writes one word to out (device, `threads` words); 0 < y < q.
 */
int pm_reduce_apply(int variant, unsigned word_bits, const uint64_t *a, const uint64_t *b, uint64_t *c,
                    uint32_t *hist, size_t n, uint64_t q, pm_stream_t stream);
int pm_reduce_chain(int variant, unsigned word_bits, uint64_t *out, size_t threads, uint64_t y, int iters,
                    uint64_t q, pm_stream_t stream);

/* ------------------------------------------------------------------- tuning
 * Pass plan per (operation, N): an N-point transform is a column pass of
 * R = N / 2^logc rows (in registers) followed by a row pass over rows of
 * 2^logc words (in LDS); logc = log2 N is a single pass. op: 0 = pm_ntt_fwd,
 * 1 = pm_ntt_inv, 2 = pm_polymul. logc = 0 restores the built-in default.
 * pm_tune_set returns PM_EINVAL for a split the kernels do not implement
 * (logc > 14, log2 N - logc > 5, or a column pass with fewer than 256 columns).
 * The setting is process-wide and is read when a call is made.
 */
int pm_tune_set(int op, unsigned log2n, unsigned logc);
int pm_tune_get(int op, unsigned log2n);   /* current logc, or PM_EINVAL */

/*
 * Small-batch plans: a batch too small to fill the GPU with 16-word threads
 * (a single transform or product is latency-bound: a row of 2^logc words
 * runs on one CU) can use a plan with 4 words per thread (rounds of two
 * stages, four times the threads) in both passes and shorter rows, spreading
 * one transform over more CUs; this is the role of the paper's
 * latency-optimised single- and multi-block kernels (Sec. V-A, V-B).
 * pm_tune_set_small installs (logc, words_per_thread) for (op, N):
 * words_per_thread 4 needs 5 <= logc <= 12 and N / 2^logc in 2^0, 2^2..2^7
 * (or 2 with logc >= 8; pm_polymul_fused keeps 16 words per thread in its
 * rows), 16 any valid split; logc = 0 removes the plan. A call over
 * N * limbs * polys_per_limb <= pm_tune_get_small_batch() words uses the
 * small-batch plan of its (op, N) if one is installed; the threshold is 0
 * (no small-batch plans used) until pm_tune_set_small_batch sets it.
 * pm_tune_set_small_limit sets a limit for one (op, N) that replaces the
 * global threshold there (the batch size up to which that plan wins varies
 * with N); max_words = 0 restores the global threshold;
 * pm_tune_get_small_limit returns 0 when none is set (or for an invalid
 * op / N). Results are identical under every plan; workspace sizes follow
 * the plan in use.
 */
int pm_tune_set_small(int op, unsigned log2n, unsigned logc, unsigned words_per_thread);
int pm_tune_get_small(int op, unsigned log2n, unsigned *logc, unsigned *words_per_thread);
int pm_tune_set_small_batch(size_t max_words);
size_t pm_tune_get_small_batch(void);
int pm_tune_set_small_limit(int op, unsigned log2n, size_t max_words);
size_t pm_tune_get_small_limit(int op, unsigned log2n);

/*
 * Software-pipelined product: pm_polymul and pm_polymul_fused (64-bit
 * words; a = b included) and their _u32 forms, under a throughput plan with rows of 2^12
 * words and a column radix of 2^3..2^5 (N = 2^15..2^17), split each launch
 * group's products (limb-major) into G chunks and run G + 2 launches; launch
 * j does the row pass of chunk j-1, the forward column pass of chunk j and
 * the inverse column pass of chunk j-2, so that the memory-bound column work
 * overlaps the VALU-bound rows. chunks = -1 (the default) pipelines a launch
 * group over 2 chunks when its row pass has at least 2048 rows (never at
 * N = 2^17; unless tuned: pm_tune_set_pipeline_rows), i.e. from 256 / 128
 * products at N = 2^15 / 2^16:
 * each chunk's rows add a phase to the critical path, which pays only for
 * batches that fill the GPU several times over; 0 or 1 never pipelines;
 * G >= 2 uses G chunks (at most 64 and at most the group's products; more
 * where a launch would exceed the grid limit). Results are identical either way.
 * Process-wide, read when a call is made; always PM_OK.
 */
int pm_tune_set_pipeline(int chunks);
int pm_tune_get_pipeline(void);

/*
 * The threshold of the default (chunks = -1) pipelining above, per column
 * radix 2^logr (logr = 3, 4, 5: N = 2^15, 2^16, 2^17 with rows of 2^12
 * words): a launch group is pipelined over 2 chunks when its row pass has
 * at least min_rows rows. min_rows = 0 restores the built-in value (2048;
 * SIZE_MAX for logr = 5); SIZE_MAX never pipelines that radix. The autotuner
 * measures it (tune.py --pipeline) and lib.apply_tune_db installs it.
 * Process-wide, read when a call is made. PM_EINVAL for logr outside 3..5;
 * pm_tune_get_pipeline_rows returns the threshold in effect (0 for an
 * invalid logr).
 */
int pm_tune_set_pipeline_rows(unsigned logr, size_t min_rows);
size_t pm_tune_get_pipeline_rows(unsigned logr);

/*
 * Software pipelining of job tables (pm_polymul_jobs, pm_plan_create): a
 * batch whose jobs of N >= 2^12 hold at least 2048 rows of 2^12 words runs
 * those jobs with rows of 2^12 words, their products split into G chunks of
 * about equal work (in job order; a boundary may fall inside a job, between
 * two of its products), in G + 2 launches; launch j does the row pass of
 * chunk j-1, the forward column pass of chunk j and the inverse column pass
 * of chunk j-2, with any mix of sizes and moduli in one launch. Jobs of
 * N < 2^12 run their single row pass in a launch before the pipeline.
 * chunks = -1 (the default): G = rows / 24576 within [2, 16]; 0 or 1: never
 * pipelined (three launches, one per pass of Eq. 2, with the tuned splits);
 * G >= 2: G chunks (at most 256; more where a launch would exceed the grid
 * limit), pipelined whenever the batch has such a job. Results are
 * identical either way. Process-wide, read when a table is built
 * (pm_polymul_jobs call, pm_plan_create); always PM_OK.
 */
int pm_tune_set_jobs_pipeline(int chunks);
int pm_tune_get_jobs_pipeline(void);

/* ------------------------------------------------------------- kernel timing
 * While enabled, every kernel the library launches is bracketed by two HIP
 * events recorded on the launch's own stream (the measurement a profiler
 * would make, taken live). pm_prof_read waits for the recorded events and
 * writes per-kernel totals (launch count and summed milliseconds) to out
 * (host, cap entries); *n receives the number of distinct kernels. reset != 0
 * discards the records afterwards. Recording costs two event records per
 * launch; leave it disabled outside measurements.
 */
typedef struct {
  char name[48];
  uint64_t launches;
  double total_ms;
} pm_prof_entry;
int pm_prof_enable(int on);
int pm_prof_read(pm_prof_entry *out, size_t cap, size_t *n, int reset);

/* ------------------------------------------------------ VALU issue-rate probe
 * A measurement helper, not part of the method: the lane-operations per
 * second the device issues for each class of VALU instruction the butterflies
 * are built from (v_mad_u64_u32, 32-bit multiplies, three-operand and carry
 * arithmetic, 64-bit shifted add, two-operand add / xor, move), each measured
 * with 32 independent register chains per thread and every CU busy, and the
 * shader clock under that load (*clock_mhz; core-clock counter against the
 * 100 MHz real-time counter). out (host, cap entries) receives one entry per
 * instruction, *n their number. Synchronous on the current device: allocates
 * a device buffer of 16 x 256 x 8 bytes per CU and frees it before returning.
 */
typedef struct {
  char name[24];
  double lane_ops_per_s;
} pm_probe_entry;
int pm_probe_valu(pm_probe_entry *out, size_t cap, size_t *n, double *clock_mhz);

/* ---------------------------------------------------------------- host helpers
 * Parameter generation on the host (no device work).
 *
 * pm_ntt_primes: the `count` largest primes q < 2^bits with q = 1 mod two_n, in
 * descending order, written to out (host). Returns how many were found.
 * pm_find_psi: psi = g^((q-1)/(2N)) for the smallest quadratic non-residue g
 * (so psi^N = q-1); 0 if 2N does not divide q-1.
 * pm_make_tables: psi_br[i] = psi^br(i), psi_inv_br[i] = psi^-br(i) (host arrays
 * of N words). Returns PM_EINVAL if psi^N != q-1.
 */
size_t pm_ntt_primes(uint64_t two_n, unsigned bits, size_t count, uint64_t *out);
uint64_t pm_find_psi(uint64_t q, size_t N);
int pm_make_tables(uint64_t q, size_t N, uint64_t psi, uint64_t *psi_br, uint64_t *psi_inv_br);

#ifdef __cplusplus
}
#endif

#endif /* PM_H */
