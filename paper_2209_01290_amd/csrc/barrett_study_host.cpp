// Host side of the Barrett variant study (include/pm.h: pm_reduce_apply,
// pm_reduce_chain): validation and the constants of Alg. 2, 3 and 4.
#include <hip/hip_runtime.h>

#include <string>

#include "../../include/pm.h"
#include "pm_host.hpp"
#include "pm_internal.hpp"

namespace pm {

// mu of each variant: floor(2^(2m)/q) (Alg. 2), floor(2^(2m+3)/q) (Alg. 3),
// floor(2^(2m+1)/q) (Alg. 4); word-size limits as the paper states them:
// len(q) <= beta-2 for Alg. 2 and 4, len(q) <= beta-4 for Alg. 3.
static int red_params(int variant, unsigned word_bits, uint64_t q, RedParams* P) {
  if (word_bits != 32 && word_bits != 64) return set_error(PM_EINVAL, "word_bits must be 32 or 64");
  if (q < 2) return set_error(PM_EINVAL, "q must be at least 2");
  const int m = 64 - __builtin_clzll(q);
  const int beta = (int)word_bits;
  int e;
  switch (variant) {
    case 0:
      if (word_bits == 32 && (q >> 32)) return set_error(PM_EINVAL, "q must fit 32 bits");
      if (word_bits == 64 && (q >> 62)) return set_error(PM_EINVAL, "q must be below 2^62");
      P->q = q; P->mu = 0; P->m = (uint32_t)m; P->pad = 0;
      return PM_OK;
    case 2: e = 0; if (m > beta - 2 || m < 1) return set_error(PM_EINVAL, "Alg. 2 needs len(q) <= word size - 2"); break;
    case 3: e = 3; if (m > beta - 4 || m < 2) return set_error(PM_EINVAL, "Alg. 3 needs len(q) <= word size - 4"); break;
    case 4: e = 1; if (m > beta - 2 || m < 2) return set_error(PM_EINVAL, "Alg. 4 needs len(q) <= word size - 2"); break;
    default: return set_error(PM_EINVAL, "variant must be 0 (%), 2, 3 or 4 (algorithm number)");
  }
  P->q = q;
  P->mu = (uint64_t)((((unsigned __int128)1) << (2 * m + e)) / q);
  P->m = (uint32_t)m;
  P->pad = 0;
  return PM_OK;
}

}  // namespace pm

using namespace pm;

extern "C" int pm_reduce_apply(int variant, unsigned word_bits, const uint64_t* a, const uint64_t* b, uint64_t* c,
                               uint32_t* hist, size_t n, uint64_t q, pm_stream_t stream) {
  RedParams P;
  int rc = red_params(variant, word_bits, q, &P);
  if (rc) return rc;
  if (n == 0 || !a || !b || !c || !hist) return set_error(PM_EINVAL, "empty input or null pointer");
  hipError_t e = launch_reduce_apply(variant, (int)word_bits, a, b, c, hist, n, P, (hipStream_t)stream);
  if (e != hipSuccess) return set_error(PM_EHIP, std::string("reduce launch: ") + hipGetErrorString(e));
  return set_error(PM_OK, "");
}

extern "C" int pm_reduce_chain(int variant, unsigned word_bits, uint64_t* out, size_t threads, uint64_t y, int iters,
                               uint64_t q, pm_stream_t stream) {
  RedParams P;
  int rc = red_params(variant, word_bits, q, &P);
  if (rc) return rc;
  if (!out || threads == 0 || threads % 256 || iters < 0 || y >= q)
    return set_error(PM_EINVAL, "out null, threads not a positive multiple of 256, or y >= q");
  hipError_t e = launch_reduce_chain(variant, (int)word_bits, out, threads, y, iters, P, (hipStream_t)stream);
  if (e != hipSuccess) return set_error(PM_EHIP, std::string("reduce launch: ") + hipGetErrorString(e));
  return set_error(PM_OK, "");
}
