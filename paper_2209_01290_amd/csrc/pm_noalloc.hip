// pm_polymul_noalloc (include/pm.h): the Eq. 2 product of pm_polymul with its
// workspace (b's column-pass output) in a fixed device array of this library
// instead of a caller buffer, for callers that cannot allocate device memory.
//
// `scratch` exists once per GPU: the array is created when the library's code
// object is loaded on that GPU and is held until the process ends. In host
// code its name is a host-side stand-in, never a device address, so host code
// never hands it to a kernel or a copy. Its device address is looked up once
// per device with hipGetSymbolAddress, with that device current, and kept in
// g_ptr[device]; every launch takes that pointer.
//
// Every call on one GPU shares that GPU's array. The workspace is written in
// full by the forward column pass before the row pass reads it, so nothing
// needs clearing between calls; calls that overlap on one GPU (two streams,
// or two threads) race on the array.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/pm.h"
#include "pm_host.hpp"
#include "pm_internal.hpp"

namespace {

constexpr size_t SCRATCH_BYTES = (size_t)PM_NOALLOC_SCRATCH_BYTES;
static_assert(SCRATCH_BYTES % 256 == 0, "scratch is a whole number of 256-byte blocks");

static __device__ __align__(256) uint64_t scratch[SCRATCH_BYTES / sizeof(uint64_t)];

constexpr int MAXDEV = 64;
std::mutex g_mu;
void* g_ptr[MAXDEV];   // device address of `scratch` on each device, once looked up

// The device address of `scratch` on device dev, looked up (with dev current)
// on the first call for that device.
int scratch_ptr(int dev, void** out) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ptr[dev]) {
    *out = g_ptr[dev];
    return PM_OK;
  }
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e == hipSuccess && cur != dev) e = hipSetDevice(dev);
  void* p = nullptr;
  if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (cur >= 0 && cur != dev) {
    const hipError_t e2 = hipSetDevice(cur);
    if (e == hipSuccess) e = e2;
  }
  if (e != hipSuccess || !p)
    return pm::set_error(PM_EHIP, std::string("pm_polymul_noalloc: scratch address lookup: ") +
                                      (e != hipSuccess ? hipGetErrorString(e) : "null address"));
  g_ptr[dev] = p;
  *out = p;
  return PM_OK;
}

}  // namespace

extern "C" int pm_polymul_noalloc(const uint64_t* a, const uint64_t* b, uint64_t* c, size_t N, size_t limbs,
                                  size_t polys_per_limb, const uint64_t* q, const uint64_t* psi_br,
                                  const uint64_t* psi_inv_br, pm_stream_t stream) {
  int dev = -1;
  const hipError_t e = hipStreamGetDevice((hipStream_t)stream, &dev);
  if (e != hipSuccess) return pm::set_error(PM_EHIP, std::string("pm_polymul_noalloc: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= MAXDEV) return pm::set_error(PM_EUNSUPPORTED, "pm_polymul_noalloc: device index above 63");
  void* ws = nullptr;
  const int rc = scratch_ptr(dev, &ws);
  if (rc != PM_OK) return rc;
  return pm::polymul_fixed_workspace(a, b, c, N, limbs, polys_per_limb, q, psi_br, psi_inv_br, ws, SCRATCH_BYTES,
                                     stream);
}
