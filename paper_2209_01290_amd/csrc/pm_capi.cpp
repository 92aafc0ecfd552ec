// Host runtime behind the C ABI of include/pm.h: argument validation, the
// per-modulus Barrett constants of Alg. 4, the pass plan for each N, limb
// chunking and kernel launches. Parameter helpers (primes, psi, twiddle
// tables) are the library's own; they share nothing with the test oracle.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <initializer_list>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/pm.h"
#include "pm_colq.hpp"
#include "pm_pipe.hpp"
#include "pm_host.hpp"
#include "pm_internal.hpp"
#include "pm_plan.hpp"
#include "pm_prof.hpp"

using namespace pm;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(PM_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

typedef unsigned __int128 u128;

bool is_pow2(size_t n) { return n && !(n & (n - 1)); }

uint64_t mulmod_h(uint64_t a, uint64_t b, uint64_t m) { return (uint64_t)((u128)a * b % m); }

uint64_t powmod_h(uint64_t b, uint64_t e, uint64_t m) {
  uint64_t r = 1 % m;
  for (b %= m; e; e >>= 1, b = mulmod_h(b, b, m))
    if (e & 1) r = mulmod_h(r, b, m);
  return r;
}
unsigned log2u(size_t n) { unsigned l = 0; while (((size_t)1 << l) < n) ++l; return l; }

}  // namespace

namespace pm {

// Barrett constants of Alg. 4 for modulus q, in the form the kernels use
// (see modarith.hpp): mu' = floor(2^(2m+1)/q) << (61-m) for m <= 61.
bool make_mod(uint64_t q, Mod* M) {
  if (q < 2 || (q >> 62) != 0) return false;
  const int m = 64 - __builtin_clzll(q);
  const u128 mu = (((u128)1) << (2 * m + 1)) / q;       // < 2^(m+2)
  M->q = q;
  M->half = (q >> 1) + 1;                                // (q+1)/2 for odd q
  if (m <= 61) {
    M->mu = (uint64_t)(mu << (61 - m));
    M->t = 0;
  } else {
    M->mu = (uint64_t)mu;
    M->t = 1;
  }
  if (m >= 34) { M->wide = 1; M->s1 = (uint32_t)(m - 34); }
  else { M->wide = 0; M->s1 = (uint32_t)(m - 2); }
  return true;
}

int set_error(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int mod_kind(const Mod& M) {
  const int m = 64 - __builtin_clzll(M.q);
  return (m >= 34 && m <= 61) ? KIND_WIDE : KIND_ANY;
}

// Barrett constants of Alg. 4 with beta = 32 (see modarith32.hpp): for an odd
// q of m <= 30 bits, mu = floor(2^(2m+1)/q) < 2^(m+2) <= 2^32, kept as
// mu << (29-m) for m <= 29 and as mu with one extra final shift for m = 30.
bool make_mod32(uint32_t q, Mod32* M) {
  if (q < 3 || !(q & 1) || (q >> 30)) return false;
  const int m = 32 - __builtin_clz(q);
  const uint64_t mu = ((uint64_t)1 << (2 * m + 1)) / q;
  M->q = q;
  M->half = (q >> 1) + 1;
  M->s = (uint32_t)(m - 2);
  if (m <= 29) {
    M->mu = (uint32_t)(mu << (29 - m));
    M->t = 0;
  } else {
    M->mu = (uint32_t)mu;
    M->t = 1;
  }
  M->pad = 0;
  return true;
}

// KIND_WIDE on 32-bit words: every modulus has m <= 29 (no final shift).
int mod_kind32(const Mod32& M) { return M.t ? KIND_ANY : KIND_WIDE; }

// ------------------------------------------------------------ PM_VALIDATE --
// With PM_VALIDATE set (and not "0"), calls also check what the kernels take
// as preconditions: every input word is canonical (< q of its limb) and each
// twiddle table's psi = table[N/2] satisfies psi^N = q - 1 (for an inverse
// table, psi^-1 does too). The checks read device memory, allocate a little
// and synchronise the stream: a debugging aid, not for graph capture.
bool validate_enabled() {
  const char* v = std::getenv("PM_VALIDATE");
  return v && *v && std::strcmp(v, "0") != 0;
}

int validate_canonical(const void* x, int word_bytes, size_t per_limb, size_t limbs, const uint64_t* q,
                       const std::string& name, hipStream_t s) {
  if (per_limb == 0 || limbs == 0) return PM_OK;
  uint64_t* qd = nullptr;
  uint32_t* fd = nullptr;
  std::vector<uint32_t> flags(limbs, 0);
  hipError_t e = hipMalloc((void**)&qd, limbs * sizeof(uint64_t));
  if (e == hipSuccess) e = hipMalloc((void**)&fd, limbs * sizeof(uint32_t));
  if (e == hipSuccess) e = hipMemcpyAsync(qd, q, limbs * sizeof(uint64_t), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemsetAsync(fd, 0, limbs * sizeof(uint32_t), s);
  for (size_t l0 = 0; e == hipSuccess && l0 < limbs; l0 += 65535) {
    const size_t nl = std::min((size_t)65535, limbs - l0);
    e = launch_canon((const char*)x + l0 * per_limb * word_bytes, word_bytes, per_limb, (uint32_t)nl, qd + l0,
                     fd + l0, s);
  }
  if (e == hipSuccess) e = hipMemcpyAsync(flags.data(), fd, limbs * sizeof(uint32_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (qd) (void)hipFree(qd);
  if (fd) (void)hipFree(fd);
  if (e != hipSuccess) return hip_fail(e, "input validation");
  for (size_t l = 0; l < limbs; ++l)
    if (flags[l])
      return fail(PM_EINVAL, name + ": limb " + std::to_string(l) + " holds a word >= q (inputs must be canonical)");
  return PM_OK;
}

int validate_psi(const void* tw, int word_bytes, size_t N, size_t limbs, const uint64_t* q, const std::string& name,
                 hipStream_t s) {
  std::vector<uint64_t> psi(limbs, 0);
  std::vector<uint32_t> psi32(word_bytes == 4 ? limbs : 0, 0);
  void* dst = word_bytes == 4 ? (void*)psi32.data() : (void*)psi.data();
  hipError_t e = hipMemcpy2DAsync(dst, word_bytes, (const char*)tw + (N / 2) * word_bytes, N * word_bytes,
                                  word_bytes, limbs, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "table validation");
  for (size_t l = 0; l < limbs; ++l) {
    const uint64_t p = word_bytes == 4 ? psi32[l] : psi[l];
    if (p >= q[l] || powmod_h(p, N, q[l]) != q[l] - 1)
      return fail(PM_EINVAL, name + ": limb " + std::to_string(l) + ": entry N/2 (psi) fails psi^N = q - 1");
  }
  return PM_OK;
}

}  // namespace pm

namespace {

// Per-word-type pieces: modulus limits and constants, kernel-name tag.
template <typename W> struct Word;
template <> struct Word<uint64_t> {
  static constexpr const char* q_rule = "q must be odd with 3 <= q < 2^62";
  static bool make(uint64_t q, Mod* M) { return (q & 1) && q >= 3 && !(q >> 62) && make_mod(q, M); }
  static int kind(const Mod& M) { return mod_kind(M); }
};
template <> struct Word<uint32_t> {
  static constexpr const char* q_rule = "q must be odd with 3 <= q < 2^30";
  static bool make(uint32_t q, Mod32* M) { return make_mod32(q, M); }
  static int kind(const Mod32& M) { return mod_kind32(M); }
};

// A validated batch: sizes, the per-limb constants, the instantiation kind.
template <typename W>
struct BatchT {
  size_t N, limbs, polys;
  unsigned log2n;
  std::vector<typename ModOf<W>::type> mods;
  int kind;
};

template <typename W>
int check_batch(BatchT<W>* b, size_t N, size_t limbs, size_t polys, const W* q) {
  if (!is_pow2(N) || N < 2 || N > ((size_t)1 << PM_MAX_LOG2N))
    return fail(PM_EINVAL, "N must be a power of two in [2, 2^17], got " + std::to_string(N));
  if (limbs == 0 || polys == 0) return fail(PM_EINVAL, "limbs and polys_per_limb must be positive");
  if (polys > 65535) return fail(PM_EINVAL, "polys_per_limb above 65535 is not supported");
  if (!q) return fail(PM_EINVAL, "q (host array of limbs moduli) is null");
  b->N = N; b->limbs = limbs; b->polys = polys; b->log2n = log2u(N);
  b->mods.resize(limbs);
  b->kind = KIND_WIDE;
  for (size_t l = 0; l < limbs; ++l) {
    const W ql = q[l];
    if (!Word<W>::make(ql, &b->mods[l]))
      return fail(PM_EINVAL, "limb " + std::to_string(l) + ": " + Word<W>::q_rule);
    if ((ql - 1) % (2 * (uint64_t)N) != 0)
      return fail(PM_EINVAL, "limb " + std::to_string(l) + ": 2N must divide q - 1");
    if (Word<W>::kind(b->mods[l]) != KIND_WIDE) b->kind = KIND_ANY;
  }
  return PM_OK;
}

// Device pointers must be non-null and aligned to their word size.
template <typename W = uint64_t>
int check_ptr(const void* p, const char* name) {
  if (!p) return fail(PM_EINVAL, std::string(name) + " is null");
  if ((uintptr_t)p & (sizeof(W) - 1))
    return fail(PM_EINVAL, std::string(name) + " is not " + std::to_string(sizeof(W)) + "-byte aligned");
  return PM_OK;
}

// Launch wrappers that name each kernel for the event timer:
// row[32]_<mode>_c<logc>, with a trailing "s" for the small-batch geometry
// (4 words per thread), and col[32]_<fwd|inv>_r<logr>.
template <typename W>
const char* row_name(int mode, int logc, int ebx) {
  static const std::vector<std::string> names = [] {
    const std::string tag = sizeof(W) == 4 ? "row32_" : "row_";
    const char* m[5] = {"fwd_c", "inv_c", "mul_c", "sqr_c", "fmul_c"};
    std::vector<std::string> v;
    for (int g = 0; g < 2; ++g)
      for (int i = 0; i < 5; ++i)
        for (int c = 0; c <= 14; ++c) v.push_back(tag + m[i] + std::to_string(c) + (g ? "s" : ""));
    return v;
  }();
  return names[(ebx == 2 ? 75 : 0) + mode * 15 + logc].c_str();
}

// "col_fwd_r4" (one thread per column), "colq_fwd_r6" (four words per thread)
template <typename W>
const char* col_name(bool inv, int logr, bool quad) {
  static const std::vector<std::string> names = [] {
    const std::string w = sizeof(W) == 4 ? "32_" : "_";
    std::vector<std::string> v;
    for (int q = 0; q < 2; ++q)
      for (int i = 0; i < 2; ++i)
        for (int r = 0; r <= 7; ++r)
          v.push_back(std::string(q ? "colq" : "col") + w + (i ? "inv_r" : "fwd_r") + std::to_string(r));
    return v;
  }();
  return names[(quad ? 16 : 0) + (inv ? 8 : 0) + logr].c_str();
}

template <typename W>
hipError_t run_row(int logc, int kind, int mode, const RowArgsT<W>& a, hipStream_t s, int ebx = 4) {
  ProfScope ps(s, row_name<W>(mode, logc, ebx));
  return launch_row(logc, kind, mode, a, s, ebx);
}

// The column pass of a plan: four words per thread (k_colq) for the
// small-batch geometry, else one thread per column (k_col).
template <typename W>
hipError_t run_col(int logr, int kind, bool inv, const ColArgsT<W>& a, hipStream_t s, int ebx) {
  const bool quad = ebx == 2 && logr >= (int)PM_COLQ_MIN_LOGR;
  ProfScope ps(s, col_name<W>(inv, logr, quad));
  return quad ? launch_colq(logr, kind, inv, a, s) : launch_col(logr, kind, inv, a, s);
}

hipError_t run_stage(int kind, bool inv, const ColArgs& a, uint32_t log2m, hipStream_t s) {
  ProfScope ps(s, inv ? "stage_inv" : "stage_fwd");
  return launch_stage(kind, inv, a, log2m, s);
}

hipError_t run_pointwise(int kind, const uint64_t* A, const uint64_t* B, uint64_t* C, uint32_t log2n,
                         uint32_t polys, uint32_t limbs, const LimbSet& ls, hipStream_t s) {
  ProfScope ps(s, "pointwise");
  return launch_pointwise(kind, A, B, C, log2n, polys, limbs, ls, s);
}

// Calls f(limb0, nlimbs, LimbSetT<W>) for consecutive launch groups of at
// most ModOf<W>::maxl limbs.
template <typename W, class F>
int for_chunks(const BatchT<W>& b, F f) {
  LimbSetT<W> ls;
  constexpr size_t maxl = ModOf<W>::maxl;
  for (size_t l0 = 0; l0 < b.limbs; l0 += maxl) {
    const size_t nl = std::min(maxl, b.limbs - l0);
    std::memset(&ls, 0, sizeof(ls));
    for (size_t i = 0; i < nl; ++i) ls.mod[i] = b.mods[l0 + i];
    hipError_t e = f(l0, nl, ls);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
  }
  return PM_OK;
}

// PM_VALIDATE checks of a batch: input spans of polys * N words per limb,
// and twiddle tables.
template <typename W>
int validate_batch(const BatchT<W>& b, std::initializer_list<std::pair<const W*, const char*>> inputs,
                   std::initializer_list<std::pair<const W*, const char*>> tables, hipStream_t s) {
  std::vector<uint64_t> q(b.limbs);
  for (size_t l = 0; l < b.limbs; ++l) q[l] = b.mods[l].q;
  int rc;
  for (const auto& in : inputs)
    if ((rc = validate_canonical(in.first, sizeof(W), b.polys * b.N, b.limbs, q.data(), in.second, s))) return rc;
  for (const auto& t : tables)
    if ((rc = validate_psi(t.first, sizeof(W), b.N, b.limbs, q.data(), t.second, s))) return rc;
  return PM_OK;
}

// The merged transforms (Alg. 5 / Alg. 6 halved) over a batch, in place.
template <typename W>
int ntt_common(W* x, size_t N, size_t limbs, size_t polys, const W* q, const W* tw, pm_stream_t stream, bool inv) {
  BatchT<W> b;
  int rc;
  if ((rc = check_batch(&b, N, limbs, polys, q))) return rc;
  if ((rc = check_ptr<W>(x, "x")) || (rc = check_ptr<W>(tw, inv ? "psi_inv_br" : "psi_br"))) return rc;
  const PassPlan p = plan_for(inv ? OP_NTT_INV : OP_NTT_FWD, b.log2n, N * limbs * polys);
  hipStream_t s = (hipStream_t)stream;
  if (validate_enabled() &&
      (rc = validate_batch<W>(b, {{x, "x"}}, {{tw, inv ? "psi_inv_br" : "psi_br"}}, s)))
    return rc;
  rc = for_chunks(b, [&](size_t l0, size_t nl, const LimbSetT<W>& ls) -> hipError_t {
    W* xs = x + l0 * polys * N;
    const W* t = tw + l0 * N;
    RowArgsT<W> ra{xs, nullptr, xs, inv ? nullptr : t, inv ? t : nullptr, b.log2n, p.R, (uint32_t)polys,
                   (uint32_t)nl, &ls};
    ColArgsT<W> ca{xs, xs, nullptr, nullptr, t, b.log2n, (uint32_t)polys, (uint32_t)nl, 1, &ls};
    hipError_t e;
    if (!inv) {
      if (p.R > 1 && (e = run_col(p.logr, b.kind, false, ca, s, p.ebx)) != hipSuccess) return e;
      return run_row(p.logc, b.kind, ROW_FWD, ra, s, p.ebx);
    }
    if ((e = run_row(p.logc, b.kind, ROW_INV, ra, s, p.ebx)) != hipSuccess) return e;
    if (p.R > 1) return run_col(p.logr, b.kind, true, ca, s, p.ebx);
    return hipSuccess;
  });
  if (rc == PM_OK) g_err.clear();
  return rc;
}

template <typename W>
size_t polymul_workspace(size_t N, size_t limbs, size_t polys) {
  if (!is_pow2(N) || N < 2 || N > ((size_t)1 << PM_MAX_LOG2N)) return 0;
  const PassPlan p = plan_for(OP_POLYMUL, log2u(N), N * limbs * polys);
  return p.R > 1 ? N * limbs * polys * sizeof(W) : 0;
}

// Chunks of the software-pipelined product for a launch group of np
// products with a column radix of 2^logr, unless pm_tune_set_pipeline chose:
// 2 when the row pass has at least plan_pipe_rows(logr) rows (2048, never
// for radix 32, unless tuned), else 0 (the three-pass form). Each chunk's rows
// are one more phase on the critical path, and a row workgroup alone on its
// CU is bound by latency, so the overlap pays only once the rows fill the CUs
// several times over. At most PIPE_MAX_CHUNKS chunks and at most np.
constexpr size_t PIPE_MAX_CHUNKS = 64;
uint32_t pipe_chunks(size_t np, uint32_t logr) {
  const int set = plan_pipe();
  const size_t rows = np << logr;
  size_t g = set >= 0 ? (size_t)set : (rows >= plan_pipe_rows(logr) ? 2 : 0);
  if (g > PIPE_MAX_CHUNKS) g = PIPE_MAX_CHUNKS;
  if (g > np) g = np;
  return g > 1 ? (uint32_t)g : 0u;
}

// Eq. 2 over a batch (fused: Alg. 8's rows instead of the pointwise rows).
template <typename W>
int polymul_common(const W* a, const W* b_, W* c, size_t N, size_t limbs, size_t polys, const W* q,
                   const W* psi_br, const W* psi_inv_br, void* workspace, pm_stream_t stream, bool fused,
                   bool checks = true) {
  BatchT<W> b;
  int rc;
  if ((rc = check_batch(&b, N, limbs, polys, q))) return rc;
  if ((rc = check_ptr<W>(a, "a")) || (rc = check_ptr<W>(b_, "b")) || (rc = check_ptr<W>(c, "c")) ||
      (rc = check_ptr<W>(psi_br, "psi_br")) || (rc = check_ptr<W>(psi_inv_br, "psi_inv_br")))
    return rc;
  const PassPlan p = plan_for(OP_POLYMUL, b.log2n, N * limbs * polys);
  // the fused product needs N >= 4 (Alg. 8's squared-twiddle identity)
  fused = fused && b.log2n >= 2;
  const bool same = (a == b_);          // one operand: one column pass, no workspace
  // and, unfused, one row transform (the small-batch geometry has no squaring
  // mode: it runs the product with b = a)
  const bool square = same && !fused && p.ebx == 4;
  // the fused rows exist in the 16-word geometry only
  const int ebx = fused ? 4 : (int)p.ebx;
  const int mode = fused ? ROW_FMUL : (square ? ROW_SQR : ROW_MUL);
  // The product is commutative: when c aliases b, swap so that c aliases a.
  const W* A = a;
  const W* B = b_;
  if (c == B && c != A) std::swap(A, B);
  if (p.R > 1 && !same && (rc = check_ptr<W>(workspace, "workspace"))) return rc;
  W* ws = (W*)workspace;
  hipStream_t s = (hipStream_t)stream;
  if (checks && validate_enabled() &&
      (rc = validate_batch<W>(b, {{a, "a"}, {b_, "b"}}, {{psi_br, "psi_br"}, {psi_inv_br, "psi_inv_br"}}, s)))
    return rc;
  rc = for_chunks(b, [&](size_t l0, size_t nl, const LimbSetT<W>& ls) -> hipError_t {
    const size_t base = l0 * polys * N;
    const W* tf = psi_br + l0 * N;
    const W* ti = psi_inv_br + l0 * N;
    if (p.R == 1) {
      RowArgsT<W> ra{A + base, square ? nullptr : B + base, c + base, tf, ti, b.log2n, 1, (uint32_t)polys,
                     (uint32_t)nl, &ls};
      return run_row(p.logc, b.kind, mode, ra, s, ebx);
    }
    // software-pipelined form: G chunks of products, G + 2 launches (pipe_kernels.hip)
    {
      const size_t np = nl * polys;     // products of this launch group
      uint32_t G = pipe_chunks(np, p.logr);
      if (G > 1 && p.ebx == 4 && p.logc == 12 && p.logr >= 3 && p.logr <= 5) {
        const uint32_t nops = same ? 1u : 2u;
        const uint32_t R = 1u << p.logr;
        // a launch holds at most (R + 3 cbs) * ceil(np / G) workgroups (rows,
        // two forward operands, inverse); keep its grid under 2^32 threads
        const uint32_t cbs = pipe_col_blocks((int)p.logr);
        const size_t cap = (((size_t)1 << 24) - 1) / (R + 3 * cbs);
        G = std::max<uint32_t>(G, (uint32_t)((np + cap - 1) / cap));
        auto lo = [&](uint32_t k) { return (uint32_t)(k * np / G); };   // chunk k = products [lo(k), lo(k+1))
        for (uint32_t j = 0; j < G + 2; ++j) {
          PipeArgsT<W> pa{A + base, B + base, c + base, same ? c + base : ws + base, tf, ti, (uint32_t)polys,
                          0, 0, 0, 0, 0, 0, nops};
          if (j >= 1 && j <= G) pa.r0 = lo(j - 1), pa.nr = R * (lo(j) - lo(j - 1));
          if (j < G) pa.f0 = lo(j), pa.nf = cbs * nops * (lo(j + 1) - lo(j));
          if (j >= 2) pa.i0 = lo(j - 2), pa.ni = cbs * (lo(j - 1) - lo(j - 2));
          static const char* const names[2][3] = {{"pipe32_mul_c12", "pipe32_fmul_c12", "pipe32_sqr_c12"},
                                                  {"pipe_mul_c12", "pipe_fmul_c12", "pipe_sqr_c12"}};
          ProfScope ps(s, names[sizeof(W) == 8][mode == ROW_FMUL ? 1 : (mode == ROW_SQR ? 2 : 0)]);
          hipError_t e = launch_pipe((int)p.logr, mode, pa, ls, b.kind, s);
          if (e != hipSuccess) return e;
        }
        return hipSuccess;
      }
    }
    // column stages of a (-> c) and b (-> workspace), fused rows, inverse columns of c
    W* wb = same ? c + base : ws + base;
    ColArgsT<W> cf{A + base, c + base, B + base, wb, tf, b.log2n, (uint32_t)polys, (uint32_t)nl,
                   same ? 1u : 2u, &ls};
    hipError_t e = run_col(p.logr, b.kind, false, cf, s, p.ebx);
    if (e != hipSuccess) return e;
    RowArgsT<W> ra{c + base, square ? nullptr : wb, c + base, tf, ti, b.log2n, p.R, (uint32_t)polys,
                   (uint32_t)nl, &ls};
    if ((e = run_row(p.logc, b.kind, mode, ra, s, ebx)) != hipSuccess) return e;
    ColArgsT<W> ci{c + base, c + base, nullptr, nullptr, ti, b.log2n, (uint32_t)polys, (uint32_t)nl, 1, &ls};
    return run_col(p.logr, b.kind, true, ci, s, p.ebx);
  });
  if (rc == PM_OK) g_err.clear();
  return rc;
}

}  // namespace

namespace pm {

// pm_polymul with the workspace supplied by the library itself (pm_noalloc.hip):
// the PM_VALIDATE scans (which allocate) and the event timer are skipped.
int polymul_fixed_workspace(const uint64_t* a, const uint64_t* b, uint64_t* c, size_t N, size_t limbs,
                            size_t polys, const uint64_t* q, const uint64_t* psi_br, const uint64_t* psi_inv_br,
                            void* workspace, size_t workspace_cap, pm_stream_t stream) {
  const size_t need = polymul_workspace<uint64_t>(N, limbs, polys);
  if (need > workspace_cap)
    return fail(PM_EINVAL, "pm_polymul_noalloc: this batch needs " + std::to_string(need) +
                               " bytes of workspace, above the library's fixed " + std::to_string(workspace_cap) +
                               "-byte scratch buffer");
  ProfOff off;
  return polymul_common(a, b, c, N, limbs, polys, q, psi_br, psi_inv_br, need ? workspace : nullptr, stream, false,
                        false);
}

}  // namespace pm

// ====================================================================== ABI ==

extern "C" {

const char* pm_last_error(void) { return g_err.c_str(); }

int pm_barrett_mulmod(const uint64_t* a, const uint64_t* b, uint64_t* c, size_t n, uint64_t q,
                      pm_stream_t stream) {
  int rc;
  if (n == 0) return fail(PM_EINVAL, "n must be positive");
  if ((rc = check_ptr(a, "a")) || (rc = check_ptr(b, "b")) || (rc = check_ptr(c, "c"))) return rc;
  Mod M;
  if (!make_mod(q, &M)) return fail(PM_EINVAL, "q must satisfy 2 <= q < 2^62");
  if (validate_enabled() && ((rc = validate_canonical(a, 8, n, 1, &q, "a", (hipStream_t)stream)) ||
                             (rc = validate_canonical(b, 8, n, 1, &q, "b", (hipStream_t)stream))))
    return rc;
  hipError_t e;
  {
    ProfScope ps((hipStream_t)stream, "mulmod");
    e = launch_mulmod(a, b, c, n, M, mod_kind(M), (hipStream_t)stream);
  }
  if (e != hipSuccess) return hip_fail(e, "pm_barrett_mulmod launch");
  g_err.clear();
  return PM_OK;
}

int pm_ntt_fwd(uint64_t* x, size_t N, size_t limbs, size_t polys_per_limb, const uint64_t* q,
               const uint64_t* psi_br, pm_stream_t stream) {
  return ntt_common(x, N, limbs, polys_per_limb, q, psi_br, stream, false);
}

int pm_ntt_inv(uint64_t* x, size_t N, size_t limbs, size_t polys_per_limb, const uint64_t* q,
               const uint64_t* psi_inv_br, pm_stream_t stream) {
  return ntt_common(x, N, limbs, polys_per_limb, q, psi_inv_br, stream, true);
}

size_t pm_polymul_workspace_bytes(size_t N, size_t limbs, size_t polys_per_limb) {
  return polymul_workspace<uint64_t>(N, limbs, polys_per_limb);
}

int pm_polymul(const uint64_t* a, const uint64_t* b, uint64_t* c, size_t N, size_t limbs, size_t polys_per_limb,
               const uint64_t* q, const uint64_t* psi_br, const uint64_t* psi_inv_br, void* workspace,
               pm_stream_t stream) {
  return polymul_common(a, b, c, N, limbs, polys_per_limb, q, psi_br, psi_inv_br, workspace, stream, false);
}

int pm_polymul_fused(const uint64_t* a, const uint64_t* b, uint64_t* c, size_t N, size_t limbs,
                     size_t polys_per_limb, const uint64_t* q, const uint64_t* psi_br, const uint64_t* psi_inv_br,
                     void* workspace, pm_stream_t stream) {
  return polymul_common(a, b, c, N, limbs, polys_per_limb, q, psi_br, psi_inv_br, workspace, stream, true);
}

size_t pm_polymul_stagewise_workspace_bytes(size_t N, size_t limbs, size_t polys_per_limb) {
  return N * limbs * polys_per_limb * sizeof(uint64_t);
}

int pm_polymul_stagewise(const uint64_t* a, const uint64_t* b_, uint64_t* c, size_t N, size_t limbs,
                         size_t polys_per_limb, const uint64_t* q, const uint64_t* psi_br,
                         const uint64_t* psi_inv_br, void* workspace, pm_stream_t stream) {
  BatchT<uint64_t> b;
  int rc;
  const size_t polys = polys_per_limb;
  if ((rc = check_batch(&b, N, limbs, polys, q))) return rc;
  if ((rc = check_ptr(a, "a")) || (rc = check_ptr(b_, "b")) || (rc = check_ptr(c, "c")) ||
      (rc = check_ptr(psi_br, "psi_br")) || (rc = check_ptr(psi_inv_br, "psi_inv_br")))
    return rc;
  const bool square = (a == b_);
  const uint64_t* A = a;
  const uint64_t* B = b_;
  if (c == B && c != A) std::swap(A, B);
  if (!square && (rc = check_ptr(workspace, "workspace"))) return rc;
  uint64_t* ws = (uint64_t*)workspace;
  hipStream_t s = (hipStream_t)stream;
  if (validate_enabled() &&
      (rc = validate_batch<uint64_t>(b, {{a, "a"}, {b_, "b"}}, {{psi_br, "psi_br"}, {psi_inv_br, "psi_inv_br"}}, s)))
    return rc;
  rc = for_chunks(b, [&](size_t l0, size_t nl, const LimbSet& ls) -> hipError_t {
    const size_t base = l0 * polys * N;
    const uint64_t* tf = psi_br + l0 * N;
    const uint64_t* ti = psi_inv_br + l0 * N;
    uint64_t* wb = square ? c + base : ws + base;
    hipError_t e;
    for (unsigned lm = 0; lm < b.log2n; ++lm) {   // Alg. 5, stage m = 2^lm
      ColArgs ca{lm == 0 ? A + base : c + base, c + base, lm == 0 ? B + base : wb, wb, tf, b.log2n,
                 (uint32_t)polys, (uint32_t)nl, square ? 1u : 2u, &ls};
      if ((e = run_stage(b.kind, false, ca, lm, s)) != hipSuccess) return e;
    }
    if ((e = run_pointwise(b.kind, c + base, wb, c + base, b.log2n, (uint32_t)polys, (uint32_t)nl, ls, s)) !=
        hipSuccess)
      return e;
    for (int lm = (int)b.log2n - 1; lm >= 0; --lm) {   // Alg. 6, stage m = 2^lm, halved
      ColArgs ca{c + base, c + base, nullptr, nullptr, ti, b.log2n, (uint32_t)polys, (uint32_t)nl, 1, &ls};
      if ((e = run_stage(b.kind, true, ca, (uint32_t)lm, s)) != hipSuccess) return e;
    }
    return hipSuccess;
  });
  if (rc == PM_OK) g_err.clear();
  return rc;
}

// ---------------------------------------------------------- 32-bit words --
// The same merged transforms and Eq. 2 product on 32-bit words, for moduli of
// up to 30 bits (Alg. 4 with beta = 32), with the pass plan of the 64-bit path.

int pm_ntt_fwd_u32(uint32_t* x, size_t N, size_t limbs, size_t polys_per_limb, const uint32_t* q,
                   const uint32_t* psi_br, pm_stream_t stream) {
  return ntt_common(x, N, limbs, polys_per_limb, q, psi_br, stream, false);
}

int pm_ntt_inv_u32(uint32_t* x, size_t N, size_t limbs, size_t polys_per_limb, const uint32_t* q,
                   const uint32_t* psi_inv_br, pm_stream_t stream) {
  return ntt_common(x, N, limbs, polys_per_limb, q, psi_inv_br, stream, true);
}

size_t pm_polymul_u32_workspace_bytes(size_t N, size_t limbs, size_t polys_per_limb) {
  return polymul_workspace<uint32_t>(N, limbs, polys_per_limb);
}

int pm_polymul_u32(const uint32_t* a, const uint32_t* b, uint32_t* c, size_t N, size_t limbs,
                   size_t polys_per_limb, const uint32_t* q, const uint32_t* psi_br, const uint32_t* psi_inv_br,
                   void* workspace, pm_stream_t stream) {
  return polymul_common(a, b, c, N, limbs, polys_per_limb, q, psi_br, psi_inv_br, workspace, stream, false);
}

int pm_polymul_fused_u32(const uint32_t* a, const uint32_t* b, uint32_t* c, size_t N, size_t limbs,
                         size_t polys_per_limb, const uint32_t* q, const uint32_t* psi_br,
                         const uint32_t* psi_inv_br, void* workspace, pm_stream_t stream) {
  return polymul_common(a, b, c, N, limbs, polys_per_limb, q, psi_br, psi_inv_br, workspace, stream, true);
}

// ------------------------------------------------------ interleaved layout --
// Batch [limb][N][polys]: coefficient j of polynomial p at j * polys + p.
// A transform is a sequence of radix-2^r blocks of stages (il_kernels.hip),
// each one launch over the whole batch; n stages split into the fewest
// blocks of at most IL_MAXR stages, balanced, larger blocks first; the fused
// middle block of the product holds two operands and takes at most
// IL_MUL_MAXR stages.

static int il_plan(unsigned n, int maxlast, int* sizes) {
  int np = (int)((n + IL_MAXR - 1) / IL_MAXR);
  for (;; ++np) {
    const int base = (int)n / np, rem = (int)n % np;
    for (int i = 0; i < np; ++i) sizes[i] = base + (i < rem ? 1 : 0);
    if (sizes[np - 1] <= maxlast) return np;
  }
}

static const char* il_name(int mode, int logr) {
  static std::vector<std::string> names = [] {
    std::vector<std::string> v;
    const char* m[3] = {"il_fwd_r", "il_inv_r", "il_mul_r"};
    for (int i = 0; i < 3; ++i)
      for (int r = 0; r <= IL_MAXR; ++r) v.push_back(std::string(m[i]) + std::to_string(r));
    return v;
  }();
  return names[mode * (IL_MAXR + 1) + logr].c_str();
}

static hipError_t run_il(int logr, int kind, int mode, const IlArgs& a, hipStream_t s) {
  ProfScope ps(s, il_name(mode, logr));
  return launch_il(logr, kind, mode, a, s);
}

static int ntt_common_il(uint64_t* x, size_t N, size_t limbs, size_t polys, const uint64_t* q,
                         const uint64_t* tw, pm_stream_t stream, bool inv) {
  BatchT<uint64_t> b;
  int rc;
  if ((rc = check_batch(&b, N, limbs, polys, q))) return rc;
  if ((rc = check_ptr(x, "x")) || (rc = check_ptr(tw, inv ? "psi_inv_br" : "psi_br"))) return rc;
  int sz[32];
  const int np = il_plan(b.log2n, IL_MAXR, sz);
  hipStream_t s = (hipStream_t)stream;
  if (validate_enabled() &&
      (rc = validate_batch<uint64_t>(b, {{x, "x"}}, {{tw, inv ? "psi_inv_br" : "psi_br"}}, s)))
    return rc;
  rc = for_chunks(b, [&](size_t l0, size_t nl, const LimbSet& ls) -> hipError_t {
    uint64_t* xs = x + l0 * polys * N;
    const uint64_t* t = tw + l0 * N;
    IlArgs a{xs, nullptr, xs, nullptr, t, t, b.log2n, 0, (uint32_t)polys, (uint32_t)nl, 1, &ls};
    hipError_t e;
    if (!inv) {
      for (int k = 0; k < np; ++k) {
        if ((e = run_il(sz[k], b.kind, IL_FWD, a, s)) != hipSuccess) return e;
        a.s0 += (uint32_t)sz[k];
      }
    } else {
      a.s0 = b.log2n;
      for (int k = np - 1; k >= 0; --k) {
        a.s0 -= (uint32_t)sz[k];
        if ((e = run_il(sz[k], b.kind, IL_INV, a, s)) != hipSuccess) return e;
      }
    }
    return hipSuccess;
  });
  if (rc == PM_OK) g_err.clear();
  return rc;
}

int pm_ntt_fwd_il(uint64_t* x, size_t N, size_t limbs, size_t polys_per_limb, const uint64_t* q,
                  const uint64_t* psi_br, pm_stream_t stream) {
  return ntt_common_il(x, N, limbs, polys_per_limb, q, psi_br, stream, false);
}

int pm_ntt_inv_il(uint64_t* x, size_t N, size_t limbs, size_t polys_per_limb, const uint64_t* q,
                  const uint64_t* psi_inv_br, pm_stream_t stream) {
  return ntt_common_il(x, N, limbs, polys_per_limb, q, psi_inv_br, stream, true);
}

size_t pm_polymul_il_workspace_bytes(size_t N, size_t limbs, size_t polys_per_limb) {
  if (!is_pow2(N) || N < 2 || N > ((size_t)1 << PM_MAX_LOG2N)) return 0;
  int sz[32];
  return il_plan(log2u(N), IL_MUL_MAXR, sz) > 1 ? N * limbs * polys_per_limb * sizeof(uint64_t) : 0;
}

int pm_polymul_il(const uint64_t* a, const uint64_t* b_, uint64_t* c, size_t N, size_t limbs,
                  size_t polys_per_limb, const uint64_t* q, const uint64_t* psi_br, const uint64_t* psi_inv_br,
                  void* workspace, pm_stream_t stream) {
  BatchT<uint64_t> b;
  int rc;
  const size_t polys = polys_per_limb;
  if ((rc = check_batch(&b, N, limbs, polys, q))) return rc;
  if ((rc = check_ptr(a, "a")) || (rc = check_ptr(b_, "b")) || (rc = check_ptr(c, "c")) ||
      (rc = check_ptr(psi_br, "psi_br")) || (rc = check_ptr(psi_inv_br, "psi_inv_br")))
    return rc;
  int sz[32];
  const int np = il_plan(b.log2n, IL_MUL_MAXR, sz);
  const bool same = (a == b_);
  const uint64_t* A = a;
  const uint64_t* B = b_;
  if (c == B && c != A) std::swap(A, B);
  if (np > 1 && !same && (rc = check_ptr(workspace, "workspace"))) return rc;
  uint64_t* ws = (uint64_t*)workspace;
  hipStream_t s = (hipStream_t)stream;
  if (validate_enabled() &&
      (rc = validate_batch<uint64_t>(b, {{a, "a"}, {b_, "b"}}, {{psi_br, "psi_br"}, {psi_inv_br, "psi_inv_br"}}, s)))
    return rc;
  rc = for_chunks(b, [&](size_t l0, size_t nl, const LimbSet& ls) -> hipError_t {
    const size_t base = l0 * polys * N;
    const uint64_t* tf = psi_br + l0 * N;
    const uint64_t* ti = psi_inv_br + l0 * N;
    hipError_t e;
    if (np == 1) {
      IlArgs m{A + base, B + base, c + base, nullptr, tf, ti, b.log2n, 0, (uint32_t)polys, (uint32_t)nl, 1, &ls};
      return run_il(sz[0], b.kind, IL_MUL, m, s);
    }
    uint64_t* wb = same ? c + base : ws + base;
    // forward blocks of a (-> c) and b (-> workspace), then in place
    IlArgs f{A + base, B + base, c + base, wb, tf, ti, b.log2n, 0, (uint32_t)polys, (uint32_t)nl,
             same ? 1u : 2u, &ls};
    for (int k = 0; k < np - 1; ++k) {
      if ((e = run_il(sz[k], b.kind, IL_FWD, f, s)) != hipSuccess) return e;
      f.A = c + base;
      f.B = wb;
      f.s0 += (uint32_t)sz[k];
    }
    IlArgs m{c + base, wb, c + base, nullptr, tf, ti, b.log2n, f.s0, (uint32_t)polys, (uint32_t)nl, 1, &ls};
    if ((e = run_il(sz[np - 1], b.kind, IL_MUL, m, s)) != hipSuccess) return e;
    IlArgs iv{c + base, nullptr, c + base, nullptr, tf, ti, b.log2n, f.s0, (uint32_t)polys, (uint32_t)nl, 1, &ls};
    for (int k = np - 2; k >= 0; --k) {
      iv.s0 -= (uint32_t)sz[k];
      if ((e = run_il(sz[k], b.kind, IL_INV, iv, s)) != hipSuccess) return e;
    }
    return hipSuccess;
  });
  if (rc == PM_OK) g_err.clear();
  return rc;
}

// ------------------------------------------------------------ host helpers --


// Miller-Rabin with the seven Jaeschke/Sinclair bases, exact for 64-bit n.
static bool probable_prime(uint64_t n) {
  if (n < 4) return n >= 2;
  if (!(n & 1)) return false;
  uint64_t d = n - 1;
  int s = __builtin_ctzll(d);
  d >>= s;
  static const uint64_t W[7] = {2, 325, 9375, 28178, 450775, 9780504, 1795265022};
  for (uint64_t w : W) {
    uint64_t a = w % n;
    if (a == 0) continue;
    uint64_t x = powmod_h(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int r = 1; r < s && comp; ++r) {
      x = mulmod_h(x, x, n);
      if (x == n - 1) comp = false;
    }
    if (comp) return false;
  }
  return true;
}

size_t pm_ntt_primes(uint64_t two_n, unsigned bits, size_t count, uint64_t* out) {
  if (!two_n || bits < 2 || bits > 63 || !out) return 0;
  const uint64_t lim = ((uint64_t)1 << bits) - 1;
  size_t got = 0;
  for (uint64_t k = (lim - 1) / two_n; k > 0 && got < count; --k) {
    const uint64_t q = k * two_n + 1;
    if (probable_prime(q)) out[got++] = q;
  }
  return got;
}

uint64_t pm_find_psi(uint64_t q, size_t N) {
  if (N == 0 || q < 3 || (q - 1) % (2 * (uint64_t)N)) return 0;
  for (uint64_t g = 2; g < q; ++g)
    if (powmod_h(g, (q - 1) >> 1, q) == q - 1) return powmod_h(g, (q - 1) / (2 * (uint64_t)N), q);
  return 0;
}

int pm_make_tables(uint64_t q, size_t N, uint64_t psi, uint64_t* psi_br, uint64_t* psi_inv_br) {
  if (!is_pow2(N) || q < 3 || !psi_br || !psi_inv_br) return fail(PM_EINVAL, "bad arguments");
  if (powmod_h(psi, N, q) != q - 1) return fail(PM_EINVAL, "psi^N != q - 1");
  const unsigned bits = log2u(N);
  // powers psi^e, e = 0..N-1, by repeated multiplication, then permuted
  std::vector<uint64_t> pw(N), pwi(N);
  const uint64_t psi_inv = powmod_h(psi, 2 * (uint64_t)N - 1, q);
  pw[0] = pwi[0] = 1;
  for (size_t e = 1; e < N; ++e) {
    pw[e] = mulmod_h(pw[e - 1], psi, q);
    pwi[e] = mulmod_h(pwi[e - 1], psi_inv, q);
  }
  for (size_t i = 0; i < N; ++i) {
    size_t r = 0;
    for (unsigned k = 0; k < bits; ++k) r |= ((i >> k) & 1) << (bits - 1 - k);
    psi_br[i] = pw[r];
    psi_inv_br[i] = pwi[r];
  }
  g_err.clear();
  return PM_OK;
}

int pm_make_tables_u32(uint32_t q, size_t N, uint32_t psi, uint32_t* psi_br, uint32_t* psi_inv_br) {
  if ((q >> 30) != 0 || !psi_br || !psi_inv_br) return fail(PM_EINVAL, "bad arguments (q must be below 2^30)");
  if (!is_pow2(N)) return fail(PM_EINVAL, "bad arguments");
  std::vector<uint64_t> f(N), i(N);
  int rc = pm_make_tables(q, N, psi, f.data(), i.data());
  if (rc) return rc;
  for (size_t k = 0; k < N; ++k) {
    psi_br[k] = (uint32_t)f[k];
    psi_inv_br[k] = (uint32_t)i[k];
  }
  return PM_OK;
}

}  // extern "C"
