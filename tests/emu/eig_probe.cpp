// Test-only entry point of the emulation build: run the library's
// eigensolver kernels on a host matrix (tests/test_emu.py compares them with
// LAPACK through NumPy).
#include <hip/hip_runtime.h>

#include <vector>

#include "../../paper_2211_12487_amd/csrc/kernels.h"

extern "C" int hipemu_sym_eig(int m, const double* A_in, double* w, int r, double* X) {
  std::vector<double> A(A_in, A_in + (size_t)m * m);
  std::vector<double> d(m), e(m), tau(m), ws((size_t)ttice::sym_eigvecs_ws(m, r > 0 ? r : 1));
  std::vector<double> ews(ttice::sym_eig_ws(m));
  if (ttice::sym_eigvals(nullptr, m, A.data(), d.data(), e.data(), tau.data(), w, ews.data()) != hipSuccess)
    return -1;
  if (r > 0 && ttice::sym_eigvecs(nullptr, m, r, d.data(), e.data(), w, A.data(), tau.data(), ws.data(), X) !=
                   hipSuccess)
    return -2;
  return 0;
}

// Tridiagonal form only (d, e) of a host matrix.
extern "C" int hipemu_tridiag(int m, const double* A_in, double* d, double* e) {
  std::vector<double> A(A_in, A_in + (size_t)m * m);
  std::vector<double> tau(m), w(m);
  std::vector<double> ews(ttice::sym_eig_ws(m));
  return ttice::sym_eigvals(nullptr, m, A.data(), d, e, tau.data(), w.data(), ews.data()) == hipSuccess ? 0 : -1;
}
