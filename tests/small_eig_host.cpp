// Host build of the per-atom LNO eigen-routines (the same header the GPU kernel compiles),
// exported with C linkage for the CPU tests.  Matrices are row-major with row stride 16.
#include "small_eig.h"

extern "C" {

int host_hess_schur(double *a, double *z, double *wr, double *wi, int n) {
  ldc::small::hessenberg(a, z, n);
  return ldc::small::schur(a, z, wr, wi, n);
}

int host_lno_atom(const double *lam, const double *sjj, int m, double lambda_th, int k_min, int k_max, int fixed,
                  double *u) {
  double work[6 * ldc::small::LD * ldc::small::LD];
  return ldc::small::lno_atom(lam, sjj, m, lambda_th, k_min, k_max, fixed, u, work);
}

}
