// Batched entry points over a job table (include/pm.h: pm_plan_*,
// pm_polymul_jobs). A job is `count` polynomial pairs sharing N and q; a
// batch mixes jobs of any N and modulus. Every job runs the three passes of
// Eq. 2 (forward columns, fused rows, inverse columns).
//
// Two forms:
//   * three-pass: each pass is one launch over the work items of all jobs
//     (three to six launches whatever the mix: rows up to 2^11, of 2^12 and tuned
//     long rows go to separate row kernels);
//   * software-pipelined (batches whose jobs of N >= 2^12 hold at least
//     JOBS_PIPE_MIN_ROWS rows of 2^12 words): those jobs take rows of 2^12
//     words, their products are split into G chunks of about equal work, and
//     G + 2 launches of k_jobs_pipe each run one chunk's rows beside the
//     column passes of its neighbours (so the memory-bound column work
//     overlaps the VALU-bound rows); jobs of N < 2^12 run their single row
//     pass in a three-pass launch before the pipeline.
//
// Device blob layout (built on the host, one copy to the device):
//   [JobDev x njobs][item->job maps, one per group]
//   [pad to 256 B][b's column outputs of the two-pass jobs]
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/pm.h"
#include "pm_host.hpp"
#include "pm_internal.hpp"
#include "pm_jobs.hpp"
#include "pm_plan.hpp"
#include "pm_prof.hpp"

using namespace pm;

namespace {

// maps: three-pass colf, row12, row13, row14, coli; pipelined rows, colf, coli;
// three-pass rows of up to 2^11 words
constexpr int NGROUP = 9;
enum { G_COLF = 0, G_ROW12 = 1, G_ROW13 = 2, G_ROW14 = 3, G_COLI = 4, G_PROW = 5, G_PCOLF = 6, G_PCOLI = 7,
       G_ROW11 = 8 };

struct Layout {
  std::vector<JobDev> jobs;            // device pointers patched once the base is known
  std::vector<uint32_t> map[NGROUP];   // item -> job
  size_t off_map[NGROUP];              // byte offsets in the blob
  size_t table_bytes;                  // jobs + maps
  size_t ws_off, ws_bytes;             // b's column outputs
  int kind;
  std::vector<JobsPipeLaunch> pipe;    // launches of the pipelined jobs (empty: three-pass form only)
};

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Pipelined form: used from this many rows of 2^12 words (jobs of N >= 2^12);
// chunks chosen by default as rows / JOBS_PIPE_ROWS_PER_CHUNK, within
// [2, JOBS_PIPE_MAX_AUTO]; at most JOBS_PIPE_MAX_CHUNKS when set.
constexpr uint64_t JOBS_PIPE_MIN_ROWS = 2048, JOBS_PIPE_ROWS_PER_CHUNK = 24576;
constexpr uint32_t JOBS_PIPE_MAX_AUTO = 16, JOBS_PIPE_MAX_CHUNKS = 256;
std::atomic<int> g_jobs_pipe{-1};

// Splits the pipelined jobs' products into G chunks of about equal work
// (rows x stages per product) and appends the G + 2 launches. A chunk
// boundary inside a job falls between two of its products; each phase's items
// of a product are contiguous, so a boundary is one item index per map.
bool plan_pipeline(Layout* L, const std::vector<uint32_t>& pjobs, uint32_t G) {
  struct Bound { uint64_t row, colf, coli; };
  auto per_product = [&](const JobDev& J, uint64_t* rows, uint64_t* colf, uint64_t* coli) {
    const uint64_t R = 1ull << J.logr;
    *rows = R;
    *colf = R > 1 ? (uint64_t)pipe_col_blocks(J.logr) * J.nops : 0;
    *coli = R > 1 ? pipe_col_blocks(J.logr) : 0;
  };
  long double W = 0;
  for (uint32_t j : pjobs) {
    const JobDev& J = L->jobs[j];
    W += (long double)J.count * (long double)((1ull << J.logr) * (12 + J.logr));
  }
  std::vector<Bound> B(G + 1);
  B[0] = {0, 0, 0};
  B[G] = {L->map[G_PROW].size(), L->map[G_PCOLF].size(), L->map[G_PCOLI].size()};
  size_t k = 0;                 // index into pjobs
  long double acc = 0;          // work of the jobs before pjobs[k]
  for (uint32_t c = 1; c < G; ++c) {
    const long double target = W * c / G;
    while (k < pjobs.size()) {
      const JobDev& J = L->jobs[pjobs[k]];
      const long double w = (long double)((1ull << J.logr) * (12 + J.logr));
      if (acc + w * J.count >= target) break;
      acc += w * J.count;
      ++k;
    }
    if (k == pjobs.size()) { B[c] = B[G]; continue; }
    const JobDev& J = L->jobs[pjobs[k]];
    const long double w = (long double)((1ull << J.logr) * (12 + J.logr));
    uint64_t poly = (uint64_t)((target - acc) / w + 0.5L);
    if (poly > J.count) poly = J.count;
    uint64_t r, f, i;
    per_product(J, &r, &f, &i);
    B[c] = {J.first[PH_ROW] + poly * r, J.first[PH_COLF] + poly * f, J.first[PH_COLI] + poly * i};
    for (int q = 0; q < 3; ++q) {         // keep boundaries monotone
      uint64_t* cur = q == 0 ? &B[c].row : (q == 1 ? &B[c].colf : &B[c].coli);
      const uint64_t prev = q == 0 ? B[c - 1].row : (q == 1 ? B[c - 1].colf : B[c - 1].coli);
      if (*cur < prev) *cur = prev;
    }
  }
  L->pipe.clear();
  for (uint32_t j = 0; j < G + 2; ++j) {
    JobsPipeLaunch pl{0, 0, 0, 0, 0, 0};
    if (j >= 1 && j <= G) pl.r0 = (uint32_t)B[j - 1].row, pl.nr = (uint32_t)(B[j].row - B[j - 1].row);
    if (j < G) pl.f0 = (uint32_t)B[j].colf, pl.nf = (uint32_t)(B[j + 1].colf - B[j].colf);
    if (j >= 2) pl.i0 = (uint32_t)B[j - 2].coli, pl.ni = (uint32_t)(B[j - 1].coli - B[j - 2].coli);
    const uint64_t blocks = (uint64_t)pl.nr + pl.nf + pl.ni;
    if (blocks >= (1ull << 24)) return false;       // keep each grid under 2^32 threads
    if (blocks) L->pipe.push_back(pl);
  }
  return true;
}

// The order in which jobs enter the work-item maps. Every transform of a row
// reads about as many twiddle words as it has coefficients, so jobs that
// share a table (same N and modulus: e.g. limb l of every request of size N)
// are placed next to each other, where the tables of neighbouring work items
// are still in cache. The groups of each size are interleaved (group k of
// every size before group k + 1 of any), so that every chunk of the
// pipelined form still mixes sizes. Ties keep the caller's order.
std::vector<uint32_t> table_order(const std::vector<JobDev>& jobs) {
  const size_t n = jobs.size();
  std::vector<uint32_t> rank(n, 0);
  std::vector<uint32_t> per_size(PM_MAX_LOG2N + 1, 0);   // tables seen so far, per size
  std::vector<std::unordered_map<const uint64_t*, uint32_t>> table_rank(PM_MAX_LOG2N + 1);
  for (size_t j = 0; j < n; ++j) {
    const uint32_t ln = jobs[j].log2n;
    auto it = table_rank[ln].find(jobs[j].tf);
    if (it == table_rank[ln].end()) it = table_rank[ln].emplace(jobs[j].tf, per_size[ln]++).first;
    rank[j] = it->second;
  }
  std::vector<uint32_t> order(n);
  for (size_t j = 0; j < n; ++j) order[j] = (uint32_t)j;
  std::stable_sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) {
    if (rank[x] != rank[y]) return rank[x] < rank[y];
    return jobs[x].log2n < jobs[y].log2n;
  });
  return order;
}

int build_layout(const pm_job* jobs, size_t njobs, Layout* L) {
  if (!jobs || njobs == 0) return set_error(PM_EINVAL, "empty job list");
  if (njobs > (1u << 24)) return set_error(PM_EINVAL, "too many jobs");
  L->jobs.assign(njobs, JobDev{});
  for (auto& m : L->map) m.clear();
  L->pipe.clear();
  L->kind = KIND_WIDE;
  uint64_t pipe_rows = 0;           // rows of 2^12 words of the jobs of N >= 2^12
  for (size_t j = 0; j < njobs; ++j) {
    const pm_job& in = jobs[j];
    const std::string tag = "job " + std::to_string(j) + ": ";
    if (in.log2n < 1 || in.log2n > PM_MAX_LOG2N) return set_error(PM_EINVAL, tag + "log2n must be in [1, 17]");
    if (in.count == 0) return set_error(PM_EINVAL, tag + "count must be positive");
    const uint64_t N = 1ull << in.log2n;
    if (!(in.q & 1) || in.q < 3 || (in.q >> 62)) return set_error(PM_EINVAL, tag + "q must be odd, 3 <= q < 2^62");
    if ((in.q - 1) % (2 * N)) return set_error(PM_EINVAL, tag + "2N must divide q - 1");
    const void* ptrs[5] = {in.psi_br, in.psi_inv_br, in.a, in.b, in.c};
    for (const void* p : ptrs)
      if (!p || ((uintptr_t)p & 7)) return set_error(PM_EINVAL, tag + "null or misaligned pointer");
    JobDev& J = L->jobs[j];
    make_mod(in.q, &J.mod);
    if (mod_kind(J.mod) != KIND_WIDE) L->kind = KIND_ANY;
    J.log2n = in.log2n;
    J.count = in.count;
    // The product is commutative: when c aliases b, swap so that c can only alias a.
    const bool swap = (in.c == in.b && in.c != in.a);
    J.a = swap ? in.b : in.a;
    J.b = swap ? in.a : in.b;
    J.c = in.c;
    J.tf = in.psi_br;
    J.ti = in.psi_inv_br;
    J.nops = (J.a == J.b) ? 1 : 2;
    if (in.log2n >= 12) pipe_rows += (uint64_t)in.count << (in.log2n - 12);
  }
  const int set = g_jobs_pipe.load();
  const bool pipelined = set != 0 && set != 1 && pipe_rows >= (set > 1 ? 1 : JOBS_PIPE_MIN_ROWS);
  const std::vector<uint32_t> order = table_order(L->jobs);
  size_t ws = 0;
  std::vector<size_t> ws_job(njobs, 0);
  std::vector<uint32_t> pjobs;
  for (const uint32_t j : order) {
    JobDev& J = L->jobs[j];
    const bool pj = pipelined && J.log2n >= 12;
    if (pj) {
      J.logc = 12;
      J.logr = J.log2n - 12;
      pjobs.push_back((uint32_t)j);
    } else {
      const PassPlan p = plan_for(OP_POLYMUL, J.log2n);
      J.logc = p.logc;
      J.logr = p.logr;
    }
    if (J.logr > 0 && J.nops == 2) {
      ws_job[j] = ws;
      ws += ((size_t)J.count << J.log2n) * sizeof(uint64_t);
    }
  }
  // work items, in the table order within each map; every phase's first
  // item is recorded (also when the job has none in that phase)
  for (const uint32_t j : order) {
    JobDev& J = L->jobs[j];
    const uint32_t R = 1u << J.logr;
    const bool pj = pipelined && J.log2n >= 12;
    auto add = [&](int g, int phase, uint64_t n) -> bool {
      if (L->map[g].size() + n > 0x7fffffffull) return false;
      J.first[phase] = (uint32_t)L->map[g].size();
      L->map[g].insert(L->map[g].end(), n, (uint32_t)j);
      return true;
    };
    bool ok = true;
    if (pj) {
      const uint64_t cols = R > 1 ? (uint64_t)pipe_col_blocks(J.logr) * J.count : 0;
      ok = add(G_PROW, PH_ROW, (uint64_t)J.count * R) && add(G_PCOLF, PH_COLF, cols * J.nops) &&
           add(G_PCOLI, PH_COLI, cols);
    } else {
      if (R > 1) {
        const uint64_t cbs = 1ull << (J.logc - 8);
        ok = add(G_COLF, PH_COLF, (uint64_t)J.nops * J.count * cbs) && add(G_COLI, PH_COLI, (uint64_t)J.count * cbs);
      }
      const int g = J.logc <= 11 ? G_ROW11 : (J.logc == 12 ? G_ROW12 : (J.logc == 13 ? G_ROW13 : G_ROW14));
      const uint64_t rows_per_item = J.logc <= 12 ? (4096u >> J.logc) : 1;   // RowGeom<logc>::ROWS
      const uint64_t tasks = (uint64_t)J.count * R;
      ok = ok && add(g, PH_ROW, (tasks + rows_per_item - 1) / rows_per_item);
    }
    if (!ok) return set_error(PM_EINVAL, "batch has more than 2^31 work items in one pass");
  }
  if (pipelined) {
    uint32_t G = set > 1 ? (uint32_t)std::min<int>(set, (int)JOBS_PIPE_MAX_CHUNKS)
                         : (uint32_t)std::min<uint64_t>(JOBS_PIPE_MAX_AUTO,
                                                        std::max<uint64_t>(2, pipe_rows / JOBS_PIPE_ROWS_PER_CHUNK));
    while (!plan_pipeline(L, pjobs, G)) {
      if (G >= (1u << 20)) return set_error(PM_EINVAL, "batch too large for the pipelined launches");
      G *= 2;
    }
  }
  size_t off = align_up(njobs * sizeof(JobDev), 256);
  for (int g = 0; g < NGROUP; ++g) {
    L->off_map[g] = off;
    off = align_up(off + L->map[g].size() * sizeof(uint32_t), 256);
  }
  L->table_bytes = off;
  L->ws_off = off;
  L->ws_bytes = ws;
  // remember where each job's b column output goes (relative offsets for now)
  for (size_t j = 0; j < njobs; ++j) L->jobs[j].wb = (uint64_t*)(uintptr_t)ws_job[j];
  return PM_OK;
}

// Writes the table part of the blob for a device base address.
void fill_blob(const Layout& L, char* host, char* dev_base) {
  std::vector<JobDev> jd = L.jobs;
  for (JobDev& J : jd) {
    if (J.logr > 0) J.wb = J.nops == 2 ? (uint64_t*)(dev_base + L.ws_off + (uintptr_t)J.wb) : J.c;
    else J.wb = nullptr;
  }
  std::memset(host, 0, L.table_bytes);
  std::memcpy(host, jd.data(), jd.size() * sizeof(JobDev));
  for (int g = 0; g < NGROUP; ++g)
    if (!L.map[g].empty()) std::memcpy(host + L.off_map[g], L.map[g].data(), L.map[g].size() * sizeof(uint32_t));
}

hipError_t launch_all(const Layout& L, char* dev_base, hipStream_t s, bool timed) {
  const JobDev* jobs = (const JobDev*)dev_base;
  auto map = [&](int g) { return (const uint32_t*)(dev_base + L.off_map[g]); };
  struct Step { int group, phase, maxlogc; const char* name; };
  static const Step steps[6] = {{G_COLF, PH_COLF, 0, "jobs_col_fwd"}, {G_ROW11, PH_ROW, 11, "jobs_row_mul_c11"},
                                {G_ROW12, PH_ROW, 12, "jobs_row_mul_c12"}, {G_ROW13, PH_ROW, 13, "jobs_row_mul_c13"},
                                {G_ROW14, PH_ROW, 14, "jobs_row_mul_c14"}, {G_COLI, PH_COLI, 0, "jobs_col_inv"}};
  for (const Step& st : steps) {
    const uint32_t n = (uint32_t)L.map[st.group].size();
    if (n == 0) continue;
    hipError_t e;
    if (timed) {
      ProfScope ps(s, st.name);
      e = launch_jobs(st.phase, st.maxlogc, L.kind, jobs, map(st.group), n, s);
    } else {
      e = launch_jobs(st.phase, st.maxlogc, L.kind, jobs, map(st.group), n, s);
    }
    if (e != hipSuccess) return e;
  }
  for (const JobsPipeLaunch& pl : L.pipe) {
    hipError_t e;
    if (timed) {
      ProfScope ps(s, "jobs_pipe_mul_c12");
      e = launch_jobs_pipe(L.kind, jobs, map(G_PROW), map(G_PCOLF), map(G_PCOLI), pl, s);
    } else {
      e = launch_jobs_pipe(L.kind, jobs, map(G_PROW), map(G_PCOLF), map(G_PCOLI), pl, s);
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Pinned staging buffers for pm_polymul_jobs: a small ring, each slot reused
// only after the copy that last read it has completed.
struct Stage {
  char* buf = nullptr;
  size_t cap = 0;
  hipEvent_t done = nullptr;
  bool used = false;
};
std::mutex g_stage_mu;
Stage g_stage[4];
unsigned g_stage_next = 0;

}  // namespace

struct pm_plan {
  int device;
  Layout L;
  char* dev = nullptr;
  size_t dev_bytes = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool use_graph = true;
};

// PM_VALIDATE checks of a job list: inputs canonical, and (tables) each
// job's twiddle tables hold a psi with psi^N = q - 1.
static int validate_jobs(const Layout& L, bool tables, hipStream_t s) {
  for (size_t j = 0; j < L.jobs.size(); ++j) {
    const JobDev& J = L.jobs[j];
    const uint64_t q = J.mod.q;
    const size_t N = (size_t)1 << J.log2n, words = (size_t)J.count * N;
    const std::string tag = "job " + std::to_string(j) + ": ";
    int rc;
    if ((rc = validate_canonical(J.a, 8, words, 1, &q, tag + "a", s))) return rc;
    if (J.b != J.a && (rc = validate_canonical(J.b, 8, words, 1, &q, tag + "b", s))) return rc;
    if (tables && ((rc = validate_psi(J.tf, 8, N, 1, &q, tag + "psi_br", s)) ||
                   (rc = validate_psi(J.ti, 8, N, 1, &q, tag + "psi_inv_br", s))))
      return rc;
  }
  return PM_OK;
}

extern "C" {

size_t pm_polymul_jobs_workspace_bytes(const pm_job* jobs, size_t njobs) {
  Layout L;
  if (build_layout(jobs, njobs, &L) != PM_OK) return 0;
  return L.ws_off + L.ws_bytes;
}

int pm_polymul_jobs(const pm_job* jobs, size_t njobs, void* workspace, size_t workspace_bytes, pm_stream_t stream) {
  Layout L;
  int rc = build_layout(jobs, njobs, &L);
  if (rc) return rc;
  const size_t need = L.ws_off + L.ws_bytes;
  if (!workspace || ((uintptr_t)workspace & 255))
    return set_error(PM_EINVAL, "workspace must be a 256-byte aligned device pointer");
  if (workspace_bytes < need)
    return set_error(PM_EINVAL, "workspace too small: need " + std::to_string(need) + " bytes");
  hipStream_t s = (hipStream_t)stream;
  if (validate_enabled() && (rc = validate_jobs(L, true, s))) return rc;
  char* base = (char*)workspace;
  {
    std::lock_guard<std::mutex> lk(g_stage_mu);
    Stage& st = g_stage[g_stage_next++ % 4];
    if (st.used && hipEventSynchronize(st.done) != hipSuccess) return set_error(PM_EHIP, "staging wait failed");
    if (st.cap < L.table_bytes) {
      // Freeing pinned memory can wait for the whole device, and pinning
      // takes time of its own: grow a slot in powers of two from 4 MiB (the
      // table of 4096 jobs of one product of N = 2^17 is under 3 MiB), so a
      // slot is reallocated rarely, if ever.
      size_t cap = (size_t)4 << 20;
      while (cap < L.table_bytes) cap <<= 1;
      if (st.buf) (void)hipHostFree(st.buf);
      st.buf = nullptr;
      st.cap = 0;
      if (hipHostMalloc((void**)&st.buf, cap, hipHostMallocDefault) != hipSuccess)
        return set_error(PM_ENOMEM, "pinned staging allocation failed");
      st.cap = cap;
    }
    if (!st.done && hipEventCreateWithFlags(&st.done, hipEventDisableTiming) != hipSuccess)
      return set_error(PM_EHIP, "event creation failed");
    fill_blob(L, st.buf, base);
    hipError_t e = hipMemcpyAsync(base, st.buf, L.table_bytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipEventRecord(st.done, s);
    if (e != hipSuccess) return set_error(PM_EHIP, std::string("job table upload: ") + hipGetErrorString(e));
    st.used = true;
  }
  hipError_t e = launch_all(L, base, s, true);
  if (e != hipSuccess) return set_error(PM_EHIP, std::string("job launch: ") + hipGetErrorString(e));
  return set_error(PM_OK, "");
}

int pm_plan_create(pm_plan** out, const pm_job* jobs, size_t njobs, unsigned flags) {
  if (!out) return set_error(PM_EINVAL, "plan pointer is null");
  *out = nullptr;
  pm_plan* p = new (std::nothrow) pm_plan();
  if (!p) return set_error(PM_ENOMEM, "host allocation failed");
  int rc = build_layout(jobs, njobs, &p->L);
  if (rc) { delete p; return rc; }
  if (validate_enabled() && (rc = validate_jobs(p->L, true, nullptr))) { delete p; return rc; }
  p->use_graph = !(flags & PM_PLAN_NO_GRAPH);
  (void)hipGetDevice(&p->device);
  p->dev_bytes = p->L.ws_off + p->L.ws_bytes;
  if (hipMalloc((void**)&p->dev, p->dev_bytes) != hipSuccess) {
    delete p;
    return set_error(PM_ENOMEM, "device allocation of " + std::to_string(p->dev_bytes) + " bytes failed");
  }
  std::vector<char> host(p->L.table_bytes);
  fill_blob(p->L, host.data(), p->dev);
  hipError_t e = hipMemcpy(p->dev, host.data(), p->L.table_bytes, hipMemcpyHostToDevice);
  if (e == hipSuccess && p->use_graph) {
    hipStream_t cs = nullptr;
    e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      hipError_t le = launch_all(p->L, p->dev, cs, false);
      e = hipStreamEndCapture(cs, &p->graph);
      if (le != hipSuccess) e = le;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    if (cs) (void)hipStreamDestroy(cs);
  }
  if (e != hipSuccess) {
    std::string msg = std::string("plan setup: ") + hipGetErrorString(e);
    pm_plan_destroy(p);
    return set_error(PM_EHIP, msg);
  }
  *out = p;
  return set_error(PM_OK, "");
}

int pm_plan_launch(pm_plan* p, pm_stream_t stream) {
  if (!p) return set_error(PM_EINVAL, "plan is null");
  int dev = -1;
  (void)hipGetDevice(&dev);
  if (dev != p->device) return set_error(PM_EINVAL, "plan belongs to another device");
  hipStream_t s = (hipStream_t)stream;
  if (validate_enabled()) {
    const int rc = validate_jobs(p->L, false, s);
    if (rc) return rc;
  }
  hipError_t e;
  if (p->use_graph) {
    ProfScope ps(s, "plan_graph");
    e = hipGraphLaunch(p->exec, s);
  } else {
    e = launch_all(p->L, p->dev, s, true);
  }
  if (e != hipSuccess) return set_error(PM_EHIP, std::string("plan launch: ") + hipGetErrorString(e));
  return set_error(PM_OK, "");
}

int pm_plan_destroy(pm_plan* p) {
  if (!p) return PM_OK;
  if (p->exec) (void)hipGraphExecDestroy(p->exec);
  if (p->graph) (void)hipGraphDestroy(p->graph);
  if (p->dev) {
    (void)hipDeviceSynchronize();
    (void)hipFree(p->dev);
  }
  delete p;
  return PM_OK;
}

size_t pm_plan_device_bytes(const pm_plan* p) { return p ? p->dev_bytes : 0; }

int pm_tune_set_jobs_pipeline(int chunks) {
  g_jobs_pipe.store(chunks < 0 ? -1 : chunks);
  return PM_OK;
}

int pm_tune_get_jobs_pipeline(void) { return g_jobs_pipe.load(); }

}  // extern "C"
