// Emulation build only: the split-BF16 and FP32 products run on matrix-core
// instructions the host emulation does not model, so its launcher reports
// "unsupported" here (the device tests cover it).
#include <hip/hip_runtime.h>

#include "../../paper_2211_12487_amd/csrc/kernels.h"

namespace ttice {
template <typename TB, typename TE, typename TD>
hipError_t gemm_mx_bf3(hipStream_t, int32_t, int32_t, int32_t, double, const double*, View, const TB*, View, double,
                       const TE*, View, TD*, View, double*) {
  return hipErrorInvalidValue;
}
template <typename TB, typename TE, typename TD>
hipError_t gemm_mx_f32(hipStream_t, int32_t, int32_t, int32_t, double, const double*, View, const TB*, View, double,
                       const TE*, View, TD*, View, double*) {
  return hipErrorInvalidValue;
}
#define STUB(TB, TE, TD)                                                                                          \
  template hipError_t gemm_mx_bf3<TB, TE, TD>(hipStream_t, int32_t, int32_t, int32_t, double, const double*, View, \
                                              const TB*, View, double, const TE*, View, TD*, View, double*);    \
  template hipError_t gemm_mx_f32<TB, TE, TD>(hipStream_t, int32_t, int32_t, int32_t, double, const double*, View, \
                                              const TB*, View, double, const TE*, View, TD*, View, double*);
STUB(double, double, double)
STUB(float, double, double)
STUB(double, float, double)
STUB(float, float, double)
STUB(double, double, float)
STUB(float, float, float)
STUB(double, float, float)
STUB(float, double, float)
}  // namespace ttice
