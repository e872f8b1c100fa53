// Emulation build only: the FP32 and split-BF16 projection kernels run on
// matrix-core instructions that the host emulation does not model, so their
// launchers report "unsupported" here (the device tests cover them).
#include <hip/hip_runtime.h>

#include "../../paper_2211_12487_amd/csrc/kernels.h"

namespace ttice {
template <typename TIn>
hipError_t proj_columns_lp(hipStream_t, int, int, int32_t, int32_t, int32_t, const TIn*, View, const double*, int64_t,
                           double*, View, double*, double*, hipEvent_t, hipEvent_t) {
  return hipErrorInvalidValue;
}
template hipError_t proj_columns_lp<float>(hipStream_t, int, int, int32_t, int32_t, int32_t, const float*, View,
                                           const double*, int64_t, double*, View, double*, double*, hipEvent_t,
                                           hipEvent_t);
template hipError_t proj_columns_lp<double>(hipStream_t, int, int, int32_t, int32_t, int32_t, const double*, View,
                                            const double*, int64_t, double*, View, double*, double*, hipEvent_t,
                                            hipEvent_t);
template <typename TIn>
hipError_t proj_group_lp(hipStream_t, int, const ProjGroup&) {
  return hipErrorInvalidValue;
}
template hipError_t proj_group_lp<float>(hipStream_t, int, const ProjGroup&);
template hipError_t proj_group_lp<double>(hipStream_t, int, const ProjGroup&);
}  // namespace ttice
