// Opt-in per-phase timing (profile.hip).
#pragma once
#include <hip/hip_runtime.h>

namespace phdc {

enum Phase {
  PH_LEAF = 0, PH_DEFLATE, PH_ROTATE, PH_SECULAR, PH_LOWNER, PH_UNORM, PH_UWRITE, PH_RANK, PH_GEMM, PH_COPY,
  PH_CANON, PH_SPLIT_SLICE, PH_SPLIT_GEMM, PH_HSS_SAMPLE, PH_HSS_COMPRESS, PH_HSS_APPLY, PH_ADJ_GEMM, PH_ADJ_BAND,
  PH_SMALL_MERGE, PH_FILL, PH_COUNT
};

// Records an event pair around the kernels launched in its lifetime when
// profiling is enabled; otherwise does nothing.
class ProfScope {
 public:
  ProfScope(int phase, hipStream_t s);
  ~ProfScope();

 private:
  int phase_;
  hipStream_t s_;
  void* a_;
};

}  // namespace phdc
