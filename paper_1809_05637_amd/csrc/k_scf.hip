// Toy self-consistent loop around the density build: Sec. II.C step (i) recomputes the LNOs
// from the density of the previous SCF step, so that they become self-consistent.  The model
// Hamiltonian of the loop is H0 plus a Hubbard-like potential on the Mulliken populations:
//   q_i  = g sum_{j in the pattern row of i} sum_ab D_ij[a, b] S_ij[a, b]   (row i of D from
//          cluster i; with the full density this is g sum_{a in i} (D S)_aa),
//   v_i  = U (q_i^in - q0_i),   H_ij = H0_ij + (v_i + v_j) / 2 S_ij,
// with linear mixing of the input populations.  Every kernel is deterministic (fixed
// reduction order).
#include <algorithm>

#include "dev_common.h"
#include "ldc_internal.h"

namespace ldc {

// q_i for every atom: one wave per atom row, the row's elements in four interleaved partial
// sums per lane, then the wave sum.
__global__ void __launch_bounds__(256) mulliken_kernel(int n_atoms, const long long *__restrict__ row_elem,
                                                       const double *__restrict__ D, const double *__restrict__ S,
                                                       double g, double *__restrict__ q) {
  const int lane = threadIdx.x & 63;
  const int nwave = gridDim.x * (blockDim.x >> 6);
  for (int i = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); i < n_atoms; i += nwave) {
    const long long lo = row_elem[i], hi = row_elem[i + 1];
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    long long e = lo + lane;
    for (; e + 192 < hi; e += 256) {
      a0 += D[e] * S[e];
      a1 += D[e + 64] * S[e + 64];
      a2 += D[e + 128] * S[e + 128];
      a3 += D[e + 192] * S[e + 192];
    }
    for (; e < hi; e += 64) a0 += D[e] * S[e];
    const double t = wave_sum((a0 + a1) + (a2 + a3));
    if (lane == 0) q[i] = g * t;
  }
}

// H = H0 + (v_i + v_j) / 2 S on every pattern block (H may be H0 itself: each element is read
// before it is written by the same lane): one wave per atom row, lanes over a block's elements.
__global__ void __launch_bounds__(256) potential_kernel(int n_atoms, const int *__restrict__ row_ptr,
                                                        const int *__restrict__ col, const int *__restrict__ n_orb,
                                                        const long long *__restrict__ blk_off,
                                                        const double *H0, const double *__restrict__ S,
                                                        const double *__restrict__ v, double *H) {
  const int lane = threadIdx.x & 63;
  const int nwave = gridDim.x * (blockDim.x >> 6);
  for (int i = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); i < n_atoms; i += nwave) {
    const double vi = v[i];
    const int mi = n_orb[i];
    for (int b = row_ptr[i]; b < row_ptr[i + 1]; ++b) {
      const int j = col[b];
      const double f = 0.5 * (vi + v[j]);
      const long long o = blk_off[b];
      const int ne = mi * n_orb[j];
      for (int e = lane; e < ne; e += 64) H[o + e] = H0[o + e] + f * S[o + e];
    }
  }
}

// Linear mixing, one workgroup: q_in <- q_in + alpha (q_out - q_in), v = U (q_in - q0), and
// res[0] = max_i |q_out - q_in| (before the mixing).
__global__ void __launch_bounds__(256) scf_mix_kernel(int n_atoms, const double *__restrict__ q_out,
                                                      double *__restrict__ q_in, const double *__restrict__ q0,
                                                      double U, double alpha, double *__restrict__ v,
                                                      double *__restrict__ res) {
  __shared__ double wmax[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double m = 0.0;
  for (int i = tid; i < n_atoms; i += blockDim.x) {
    const double qi = q_in[i], d = q_out[i] - qi;
    m = fmax(m, fabs(d));
    const double qn = qi + alpha * d;
    q_in[i] = qn;
    v[i] = U * (qn - q0[i]);
  }
  m = wave_max(m);
  if (lane == 0) wmax[wave] = m;
  __syncthreads();
  if (tid == 0) {
    double r = wmax[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) r = fmax(r, wmax[w]);
    res[0] = r;
  }
}

// Neutral reference populations of the toy loop: q0_i = N_e M_i / sum_j M_j.
__global__ void reference_populations_kernel(int n_atoms, const int *__restrict__ n_orb, double n_e, double n_basis,
                                             double *__restrict__ q0) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_atoms; i += gridDim.x * blockDim.x)
    q0[i] = n_e * (double)n_orb[i] / n_basis;
}

void launch_reference_populations(Plan &p, double n_electrons, double *d_q0) {
  const int blocks = std::max(1, std::min(256, (p.n_atoms + 255) / 256));
  hipLaunchKernelGGL(reference_populations_kernel, dim3(blocks), dim3(256), 0, p.stream, p.n_atoms, p.d_n_orb,
                     n_electrons, (double)p.n_basis, d_q0);
}

void launch_mulliken(Plan &p, const double *d_D, const double *d_S, double *d_q, double g) {
  const int wgs = std::max(1, std::min(p.workgroups * 4, (p.n_atoms + 3) / 4));
  hipLaunchKernelGGL(mulliken_kernel, dim3(wgs), dim3(kWG), 0, p.stream, p.n_atoms, p.d_row_elem, d_D, d_S, g, d_q);
}

void launch_potential(Plan &p, const double *d_H0, const double *d_S, const double *d_v, double *d_H) {
  const int wgs = std::max(1, std::min(p.workgroups * 4, (p.n_atoms + 3) / 4));
  hipLaunchKernelGGL(potential_kernel, dim3(wgs), dim3(kWG), 0, p.stream, p.n_atoms, p.d_row_ptr, p.d_col, p.d_n_orb,
                     p.d_blk_off, d_H0, d_S, d_v, d_H);
}

void launch_scf_mix(Plan &p, const double *d_q_out, double *d_q_in, const double *d_q0, double U, double alpha,
                    double *d_v, double *d_res) {
  hipLaunchKernelGGL(scf_mix_kernel, dim3(1), dim3(kWG), 0, p.stream, p.n_atoms, d_q_out, d_q_in, d_q0, U, alpha, d_v,
                     d_res);
}

}  // namespace ldc
