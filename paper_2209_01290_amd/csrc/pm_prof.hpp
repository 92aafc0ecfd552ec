// Kernel timing with HIP events (see pm_prof_* in include/pm.h).
#pragma once
#include <hip/hip_runtime.h>

namespace pm {

// Brackets one kernel launch on stream s when timing is enabled:
//   ProfScope ps(s, "row_mul_c12"); launch...; ps.done();
class ProfScope {
 public:
  ProfScope(hipStream_t s, const char* name);
  void done();
  ~ProfScope() { done(); }

 private:
  hipStream_t s_;
  const char* name_;
  int slot_;
};

// While one is alive on a thread, ProfScope records nothing on that thread
// (entry points that must not create events or touch host-side pools).
class ProfOff {
 public:
  ProfOff();
  ~ProfOff();
  ProfOff(const ProfOff&) = delete;
  ProfOff& operator=(const ProfOff&) = delete;
};

}  // namespace pm
