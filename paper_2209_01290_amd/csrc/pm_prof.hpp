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

}  // namespace pm
