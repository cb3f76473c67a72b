#include "nufft.h"
namespace pfmm {
size_t nufft_workspace_bytes(const pfmm_plan_s*, int64_t, int64_t) { return 0; }
int nufft_far(const pfmm_plan_s*, int64_t, int64_t, const double*, const double*, const double*,
              const double*, const double*, char*, hipStream_t, const double**) {
  return PFMM_EINVAL;
}
}  // namespace pfmm
