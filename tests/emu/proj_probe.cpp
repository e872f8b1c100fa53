// Test-only entry point of the emulation build: run the library's fused
// column-projection kernel on host buffers (tests/test_emu.py compares it
// with NumPy in FP64).  Z is N frame-major (rows x cols) matrices with frame
// stride fs (dtype 0: float, 1: double); C receives N frames (r x cols) with
// frame stride fs_c; prec is the products' arithmetic (kProj*).  U must carry the kernel's kProjTail over-read.
#include <hip/hip_runtime.h>

#include "../../paper_2211_12487_amd/csrc/kernels.h"

extern "C" int hipemu_proj(int rows, int r, int N, int cols, long long fs, int dtype, const void* Z,
                           const double* U, long long ldu, double* C, long long fs_c, double* zn, double* rh,
                           int prec) {
  const ttice::View vz = ttice::unfolding(cols, fs);
  const ttice::View vc = ttice::unfolding(cols, fs_c);
  const int Ncol = N * cols;
  hipError_t e;
  if (dtype == 0)
    e = ttice::proj_columns<float>(nullptr, rows, r, Ncol, (const float*)Z, vz, U, ldu, C, vc, zn, rh, prec);
  else
    e = ttice::proj_columns<double>(nullptr, rows, r, Ncol, (const double*)Z, vz, U, ldu, C, vc, zn, rh, prec);
  return e == hipSuccess ? 0 : -1;
}
