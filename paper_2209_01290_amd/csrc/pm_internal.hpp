// Declarations shared by the kernels file and the host runtime (not exported).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "modarith.hpp"
#include "modarith32.hpp"

namespace pm {

// The moduli of a launch group travel by value in the kernel arguments
// (at most 4 KiB per launch): up to 64 limbs of Mod (32 bytes) or 128 of Mod32
// (24 bytes); larger batches are launched in groups of that many limbs. Word
// types: uint64_t (q < 2^62, constants in Mod) and uint32_t (q < 2^30,
// constants in Mod32).
constexpr int MAXL = 64;

template <typename W> struct ModOf { using type = Mod; static constexpr int maxl = MAXL; };
template <> struct ModOf<uint32_t> { using type = Mod32; static constexpr int maxl = 128; };

template <typename W>
struct LimbSetT {
  typename ModOf<W>::type mod[ModOf<W>::maxl];
};
static_assert(sizeof(LimbSetT<uint64_t>) <= 2048 && sizeof(LimbSetT<uint32_t>) <= 3072, "kernel argument budget");
using LimbSet = LimbSetT<uint64_t>;
using LimbSet32 = LimbSetT<uint32_t>;

enum { ROW_FWD = 0, ROW_INV = 1, ROW_MUL = 2, ROW_SQR = 3, ROW_FMUL = 4 };

// Column workgroups (256 threads) per operand of one product in the
// software-pipelined kernels (rows of 2^12 words, column radix 2^logr): one
// thread per column, 256 columns each; for logr = 5 two lanes per column,
// 128 columns each.
constexpr uint32_t pipe_col_blocks(int logr) { return logr == 5 ? 32u : 16u; }

template <typename W>
struct RowArgsT {
  const W* A;             // input rows (FWD/INV: in place with C allowed)
  const W* B;             // second operand (MUL only)
  W* C;                   // output rows
  const W* twf;           // psi_br, [limbs][N]
  const W* twi;           // psi_inv_br, [limbs][N]
  uint32_t log2n, R, polys, limbs;
  const LimbSetT<W>* ls;
};
using RowArgs = RowArgsT<uint64_t>;

template <typename W>
struct ColArgsT {
  const W* src0;
  W* dst0;
  const W* src1;          // second operand (nops == 2)
  W* dst1;
  const W* tw;            // [limbs][N]
  uint32_t log2n, polys, limbs, nops;
  const LimbSetT<W>* ls;
};
using ColArgs = ColArgsT<uint64_t>;

hipError_t launch_mulmod(const uint64_t* a, const uint64_t* b, uint64_t* c, size_t n, const Mod& M, int kind,
                         hipStream_t s);
// ebx: log2 of the words per thread of the row pass: 4 (16 words, rounds of
// four stages) or 2 (4 words, rounds of two stages; rows of 2^5..2^12, modes
// FWD, INV and MUL only).
hipError_t launch_row(int logc, int kind, int mode, const RowArgs& a, hipStream_t s, int ebx = 4);
hipError_t launch_row(int logc, int kind, int mode, const RowArgsT<uint32_t>& a, hipStream_t s, int ebx = 4);
#define PM_DECL_ROW(L)                                                                               \
  hipError_t launch_row_##L(int kind, int mode, int ebx, const RowArgs& a, hipStream_t s);           \
  hipError_t launch_row_##L(int kind, int mode, int ebx, const RowArgsT<uint32_t>& a, hipStream_t s);
PM_DECL_ROW(1) PM_DECL_ROW(2) PM_DECL_ROW(3) PM_DECL_ROW(4) PM_DECL_ROW(5) PM_DECL_ROW(6) PM_DECL_ROW(7)
PM_DECL_ROW(8) PM_DECL_ROW(9) PM_DECL_ROW(10) PM_DECL_ROW(11) PM_DECL_ROW(12) PM_DECL_ROW(13) PM_DECL_ROW(14)
#undef PM_DECL_ROW
// The product rows (ROW_MUL, ROW_FMUL) of 2^12 words with the split's radix
// fixed at compile time (row_fixed.inc): 64-bit words with moduli of 34..61
// bits (row_12r.hip), 32-bit words (row_12r32.hip); false, launching
// nothing, for other modes, kinds or shapes.
bool launch_row12_fixed(int kind, int mode, const RowArgs& a, hipStream_t s);
bool launch_row12_fixed(int kind, int mode, const RowArgsT<uint32_t>& a, hipStream_t s);
hipError_t launch_col(int logr, int kind, bool inv, const ColArgs& a, hipStream_t s);
hipError_t launch_col(int logr, int kind, bool inv, const ColArgsT<uint32_t>& a, hipStream_t s);

// Interleaved (coefficient-major) layout: one radix-2^logr block of stages
// s0..s0+logr-1 per launch (il_kernels.hip).
enum { IL_FWD = 0, IL_INV = 1, IL_MUL = 2 };
constexpr int IL_MAXR = 6;       // words per thread: 2^6 (128 VGPRs of data)
constexpr int IL_MUL_MAXR = 5;   // the fused block holds both operands' words
struct IlArgs {
  const uint64_t* A;
  const uint64_t* B;             // second operand (IL_FWD with nops == 2, IL_MUL)
  uint64_t* C;
  uint64_t* D;                   // second output (IL_FWD with nops == 2)
  const uint64_t* twf;           // psi_br, [limbs][N]
  const uint64_t* twi;           // psi_inv_br, [limbs][N]
  uint32_t log2n, s0, polys, limbs, nops;
  const LimbSet* ls;
};
hipError_t launch_il(int logr, int kind, int mode, const IlArgs& a, hipStream_t s);

// PM_VALIDATE scan (pm_validate.hip): flags_dev[l] = 1 if some word of limb
// l's span of x (per_limb words of word_bytes each) is >= qs_dev[l].
hipError_t launch_canon(const void* x, int word_bytes, size_t per_limb, uint32_t limbs, const uint64_t* qs_dev,
                        uint32_t* flags_dev, hipStream_t s);
hipError_t launch_stage(int kind, bool inv, const ColArgs& a, uint32_t log2m, hipStream_t s);
hipError_t launch_pointwise(int kind, const uint64_t* A, const uint64_t* B, uint64_t* C, uint32_t log2n,
                            uint32_t polys, uint32_t limbs, const LimbSet& ls, hipStream_t s);

// Job-table passes (pm_jobs.hip): phase PH_COLF / PH_ROW / PH_COLI, the row
// phase split by maximal row length (12, 13 or 14).
struct JobDev;
hipError_t launch_jobs(int phase, int maxlogc, int kind, const JobDev* jobs, const uint32_t* item_job,
                       uint32_t nitems, hipStream_t s);

// Barrett variant study (barrett_study.hip, barrett_study_host.cpp).
struct RedParams {
  uint64_t q;
  uint64_t mu;      // floor(2^(2m + e) / q) with e = 0, 3, 1 for Alg. 2, 3, 4
  uint32_t m;       // len(q)
  uint32_t pad;
};
hipError_t launch_reduce_apply(int variant, int word_bits, const uint64_t* a, const uint64_t* b, uint64_t* c,
                               uint32_t* hist, size_t n, const RedParams& P, hipStream_t s);
hipError_t launch_reduce_chain(int variant, int word_bits, uint64_t* out, size_t threads, uint64_t y, int iters,
                               const RedParams& P, hipStream_t s);

// Eq. 2 over a batch with a caller-fixed workspace of workspace_cap bytes
// (PM_EINVAL when the batch needs more); no device allocation, no PM_VALIDATE
// scan, no event timer. stream is a hipStream_t (pm_capi.cpp).
int polymul_fixed_workspace(const uint64_t* a, const uint64_t* b, uint64_t* c, size_t N, size_t limbs,
                            size_t polys, const uint64_t* q, const uint64_t* psi_br, const uint64_t* psi_inv_br,
                            void* workspace, size_t workspace_cap, void* stream);

}  // namespace pm
