// Matrix-core tiled products (gemm_mx.h): the FP64 instantiations and the
// launcher behind gemm()'s route for large level contractions.
#include "gemm_mx.h"

#include <algorithm>

namespace ttice {

template <int P, typename TB, typename TE, typename TD>
hipError_t launch_gemm_mx(hipStream_t st, int32_t M, int32_t N, int32_t K, double alpha, const double* A, View va,
                          const TB* B, View vb, double beta, const TE* E, View ve, TD* D, View vd,
                          double* colpart) {
  static_assert(P == mx::kMxF64, "the FP64 launcher");
  constexpr size_t lds = mx::lds_bytes<P>();
  static const hipError_t attr = hipFuncSetAttribute((const void*)mx::k_gemm_mx64<TB, TE, TD>,
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (attr != hipSuccess) return attr;
  const dim3 grid((unsigned)((N + mx::BN - 1) / mx::BN), (unsigned)((M + mx::BM - 1) / mx::BM));
  hipLaunchKernelGGL((mx::k_gemm_mx64<TB, TE, TD>), grid, dim3(mx::kThreads), lds, st, M, N, K, alpha, A, va, B,
                     vb, beta, E, ve, D, vd, colpart);
  return hipGetLastError();
}

bool gemm_mx_fits(int32_t M, int32_t N, int32_t K, const View& va, const View& vb, const View& ve, const View& vd,
                  bool has_e, bool has_d, bool bnorm) {
  if (bnorm || M <= 0 || N <= 0 || K <= 0) return false;
  if (va.rpf != kUnframed || va.cpf != kUnframed || vb.rpf != kUnframed) return false;
  if ((has_e && ve.rpf != kUnframed) || (has_d && vd.rpf != kUnframed)) return false;
  // enough output tiles to fill the device without splitting K
  const int64_t tiles = (int64_t)((N + mx::BN - 1) / mx::BN) * ((M + mx::BM - 1) / mx::BM);
  return tiles >= 96 && (int64_t)M * N * (int64_t)K >= ((int64_t)1 << 24);
}

int32_t gemm_mx_split_slices(int32_t M, int32_t N, int32_t K, const View& va, const View& vb, int64_t ws_len) {
  if (M <= 0 || N <= 0 || K < 2048) return 0;
  if (va.rpf != kUnframed || va.cpf != kUnframed || vb.rpf != kUnframed) return 0;
  const int64_t tiles = (int64_t)((N + mx::BN - 1) / mx::BN) * ((M + mx::BM - 1) / mx::BM);
  // (96 tiles and more: the unsplit product fills the device)
  if (tiles >= 96 || tiles < 8 || (int64_t)M * N * (int64_t)K < ((int64_t)1 << 27)) return 0;
  int64_t S = (256 + tiles - 1) / tiles;  // about one block per CU
  S = std::min<int64_t>({S, (int64_t)K / 1024, 8, ws_len / ((int64_t)M * N)});
  return S >= 2 ? (int32_t)S : 0;
}

template <typename TB>
hipError_t gemm_mx64_part(hipStream_t st, int32_t M, int32_t N, int32_t K, int32_t S, int32_t kchunk,
                          const double* A, View va, const TB* B, View vb, double* part) {
  constexpr size_t lds = mx::lds_bytes<mx::kMxF64>();
  static const hipError_t attr = hipFuncSetAttribute((const void*)mx::k_gemm_mx64_part<TB>,
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (attr != hipSuccess) return attr;
  const dim3 grid((unsigned)((N + mx::BN - 1) / mx::BN), (unsigned)((M + mx::BM - 1) / mx::BM), (unsigned)S);
  hipLaunchKernelGGL((mx::k_gemm_mx64_part<TB>), grid, dim3(mx::kThreads), lds, st, M, N, K, kchunk, A, va, B, vb,
                     part);
  return hipGetLastError();
}
template hipError_t gemm_mx64_part<double>(hipStream_t, int32_t, int32_t, int32_t, int32_t, int32_t, const double*,
                                           View, const double*, View, double*);
template hipError_t gemm_mx64_part<float>(hipStream_t, int32_t, int32_t, int32_t, int32_t, int32_t, const double*,
                                          View, const float*, View, double*);

template <typename TB, typename TE, typename TD>
hipError_t gemm_mx(hipStream_t st, int prec, int32_t M, int32_t N, int32_t K, double alpha, const double* A,
                   View va, const TB* B, View vb, double beta, const TE* E, View ve, TD* D, View vd,
                   double* colpart) {
  if (prec == kProjBF16x3)
    return gemm_mx_bf3<TB, TE, TD>(st, M, N, K, alpha, A, va, B, vb, beta, E, ve, D, vd, colpart);
  if (prec == kProjFP32)
    return gemm_mx_f32<TB, TE, TD>(st, M, N, K, alpha, A, va, B, vb, beta, E, ve, D, vd, colpart);
  return launch_gemm_mx<mx::kMxF64, TB, TE, TD>(st, M, N, K, alpha, A, va, B, vb, beta, E, ve, D, vd, colpart);
}

#define TTICE_GEMM_MX_INST(TB, TE, TD)                                                                          \
  template hipError_t gemm_mx<TB, TE, TD>(hipStream_t, int, int32_t, int32_t, int32_t, double, const double*,   \
                                          View, const TB*, View, double, const TE*, View, TD*, View, double*); \
  template hipError_t launch_gemm_mx<mx::kMxF64, TB, TE, TD>(hipStream_t, int32_t, int32_t, int32_t, double,   \
                                                             const double*, View, const TB*, View, double,      \
                                                             const TE*, View, TD*, View, double*);
TTICE_GEMM_MX_INST(double, double, double)
TTICE_GEMM_MX_INST(float, double, double)
TTICE_GEMM_MX_INST(double, float, double)
TTICE_GEMM_MX_INST(float, float, double)
TTICE_GEMM_MX_INST(double, double, float)
TTICE_GEMM_MX_INST(float, float, float)
TTICE_GEMM_MX_INST(double, float, float)
TTICE_GEMM_MX_INST(float, double, float)

}  // namespace ttice
