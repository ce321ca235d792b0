// LNO kernels (Sec. II.B, steps (i)-(iii)).
//
// lambda_kernel: Lambda_j = sum_k rho_jk S_kj (Eq. 17), one wavefront per atom.  With S
//   symmetric, S_kj = S_jk^T, so only row j of the block pattern is read:
//   Lambda_j[a][b] = sum_k sum_g rho_jk[a][g] S_jk[b][g].
// lno_eig_kernel: one thread per atom: Hessenberg + Francis QR to real Schur form,
//   ranking by real part and the rank rule, eigenvectors of the kept eigenvalues by
//   back-substitution, S_jj-Loewdin orthonormalisation (small_eig.h).
#include "dev_common.h"
#include "small_eig.h"

namespace ldc {

__global__ void __launch_bounds__(256) lambda_kernel(int n_atoms, const int *__restrict__ n_orb,
                                                     const int *__restrict__ row_ptr, const int *__restrict__ col,
                                                     const long long *__restrict__ blk_off,
                                                     const double *__restrict__ S, const double *__restrict__ D,
                                                     double *__restrict__ lam) {
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (j >= n_atoms) return;
  const int m = n_orb[j];
  for (int e = lane; e < m * m; e += 64) {
    const int a = e / m, b = e % m;
    double acc = 0.0;
    for (int bb = row_ptr[j]; bb < row_ptr[j + 1]; ++bb) {
      const int k = col[bb];
      const int mk = n_orb[k];
      const double *dj = D + blk_off[bb] + a * mk;
      const double *sj = S + blk_off[bb] + b * mk;
      for (int g = 0; g < mk; ++g) acc += dj[g] * sj[g];
    }
    lam[(long long)j * kMaxOrb * kMaxOrb + a * kMaxOrb + b] = acc;
  }
}

__global__ void __launch_bounds__(64) lno_eig_kernel(int n_atoms, const int *__restrict__ n_orb,
                                                    const int *__restrict__ row_ptr, const int *__restrict__ col,
                                                    const long long *__restrict__ blk_off,
                                                    const double *__restrict__ S, const double *__restrict__ lam,
                                                    const int *__restrict__ fixed, double lambda_th, int k_min,
                                                    int k_max, int *__restrict__ rank, double *__restrict__ U,
                                                    DevStatus *st) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_atoms) return;
  const int m = n_orb[j];
  double lj[kMaxOrb * kMaxOrb], sjj[kMaxOrb * kMaxOrb], work[6 * kMaxOrb * kMaxOrb], u[kMaxOrb * kMaxOrb];
  for (int i = 0; i < m * m; ++i) {
    const int a = i / m, b = i % m;
    lj[a * kMaxOrb + b] = lam[(long long)j * kMaxOrb * kMaxOrb + a * kMaxOrb + b];
  }
  // diagonal block of S (row j)
  int bd = -1;
  for (int bb = row_ptr[j]; bb < row_ptr[j + 1]; ++bb)
    if (col[bb] == j) bd = bb;
  if (bd < 0) {
    report(st, LDC_ERR_ARG, j);
    rank[j] = 0;
    return;
  }
  for (int i = 0; i < m * m; ++i) {
    const int a = i / m, b = i % m;
    sjj[a * kMaxOrb + b] = S[blk_off[bd] + i];
  }
  const int k = small::lno_atom(lj, sjj, m, lambda_th, k_min, k_max, fixed ? fixed[j] : -1, u, work);
  if (k < 0) {
    report(st, k == -1 ? LDC_ERR_EIG_NOCONV : LDC_ERR_RANK, j);
    rank[j] = 0;
    return;
  }
  rank[j] = k;
  double *uj = U + (long long)j * kMaxOrb * kMaxOrb;
  for (int i = 0; i < m * k; ++i) uj[i] = u[i];
}

void launch_lambda(Plan &p, const double *d_S, const double *d_D) {
  const int waves_per_block = 4;
  const int blocks = (p.n_atoms + waves_per_block - 1) / waves_per_block;
  hipLaunchKernelGGL(lambda_kernel, dim3(blocks), dim3(64 * waves_per_block), 0, p.stream, p.n_atoms, p.d_n_orb,
                     p.d_row_ptr, p.d_col, p.d_blk_off, d_S, d_D, p.d_lambda);
}

void launch_lno_eig(Plan &p, const double *d_S, double lambda_th, int k_min, int k_max) {
  const int blocks = (p.n_atoms + 63) / 64;
  hipLaunchKernelGGL(lno_eig_kernel, dim3(blocks), dim3(64), 0, p.stream, p.n_atoms, p.d_n_orb, p.d_row_ptr,
                     p.d_col, p.d_blk_off, d_S, p.d_lambda, p.d_fixed, lambda_th, k_min, k_max, p.d_rank, p.d_U,
                     p.d_status);
}

}  // namespace ldc
