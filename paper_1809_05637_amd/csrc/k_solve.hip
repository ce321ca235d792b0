// Cluster problem kernels (Sec. II.C (ii)-(iii)): gather of H^(i), S^(i) with PAO/LNO
// blocks (Eq. 26), Cholesky of S^(i), reduction to the standard problem and Householder
// tridiagonalization.  One 256-thread workgroup per cluster; workgroups walk the clusters
// largest-first with a fixed stride (persistent launch, deterministic assignment).
#include "wg_blas.h"

namespace ldc {

constexpr int NB = 32;  // panel width of the blocked factorizations

// ---------------------------------------------------------------------------------------
// (a)+(c) gather: dense column-major H^(i), S^(i) (leading dimension = cluster dimension).
// Long members enter through their LNOs: blocks U_a^T X, X U_b or U_a^T X U_b.
__global__ void __launch_bounds__(256) gather_kernel(int n_clusters, const int *__restrict__ order,
                                                     const int *__restrict__ mem_ptr, const int *__restrict__ mem_atom,
                                                     const int *__restrict__ mem_long, const int *__restrict__ pair_ptr,
                                                     const int *__restrict__ pair_ab, const int *__restrict__ pair_blk,
                                                     const int *__restrict__ n_orb, const long long *__restrict__ blk_off,
                                                     const double *__restrict__ H, const double *__restrict__ S,
                                                     int lno_mode, const int *__restrict__ rank,
                                                     const double *__restrict__ U, double *__restrict__ mat,
                                                     const long long *__restrict__ mat_off, const int *__restrict__ dmax,
                                                     int *__restrict__ dim) {
  __shared__ int off[kMaxMembers + 1];
  __shared__ int dm[kMaxMembers];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int s = blockIdx.x; s < n_clusters; s += gridDim.x) {
    const int c = order[s];
    const int mb = mem_ptr[c], nm = mem_ptr[c + 1] - mb;
    __syncthreads();
    for (int a = tid; a < nm; a += blockDim.x) {
      const int atom = mem_atom[mb + a];
      dm[a] = (lno_mode && mem_long[mb + a]) ? rank[atom] : n_orb[atom];
    }
    __syncthreads();
    if (tid == 0) {
      off[0] = 0;
      for (int a = 0; a < nm; ++a) off[a + 1] = off[a] + dm[a];
      dim[c] = off[nm];
    }
    __syncthreads();
    const int n = off[nm];
    double *Hc = mat + mat_off[c];
    double *Sc = Hc + (long long)dmax[c] * dmax[c];
    for (long long e = tid; e < (long long)n * n; e += blockDim.x) {
      Hc[e] = 0.0;
      Sc[e] = 0.0;
    }
    __syncthreads();
    for (int pp = pair_ptr[c] + wave; pp < pair_ptr[c + 1]; pp += (blockDim.x >> 6)) {
      const int ab = pair_ab[pp];
      const int a = ab & 0xffff, b = ab >> 16;
      const int blk = pair_blk[pp];
      const int ja = mem_atom[mb + a], jb = mem_atom[mb + b];
      const int ma = n_orb[ja], mbb = n_orb[jb];
      const bool la = lno_mode && mem_long[mb + a];
      const bool lb = lno_mode && mem_long[mb + b];
      const int da = dm[a], db = dm[b];
      const double *hb = H + blk_off[blk];
      const double *sb = S + blk_off[blk];
      const double *Ua = U + (long long)ja * kMaxOrb * kMaxOrb;
      const double *Ub = U + (long long)jb * kMaxOrb * kMaxOrb;
      for (int e = lane; e < da * db; e += 64) {
        const int r = e % da, q = e / da;
        double h = 0.0, sv = 0.0;
        if (!la && !lb) {
          h = hb[r * mbb + q];
          sv = sb[r * mbb + q];
        } else if (la && !lb) {
          for (int al = 0; al < ma; ++al) {
            const double u = Ua[al + r * ma];
            h += u * hb[al * mbb + q];
            sv += u * sb[al * mbb + q];
          }
        } else if (!la && lb) {
          for (int be = 0; be < mbb; ++be) {
            const double u = Ub[be + q * mbb];
            h += hb[r * mbb + be] * u;
            sv += sb[r * mbb + be] * u;
          }
        } else {
          for (int al = 0; al < ma; ++al) {
            double th = 0.0, ts = 0.0;
            for (int be = 0; be < mbb; ++be) {
              const double u = Ub[be + q * mbb];
              th += hb[al * mbb + be] * u;
              ts += sb[al * mbb + be] * u;
            }
            const double u = Ua[al + r * ma];
            h += u * th;
            sv += u * ts;
          }
        }
        const long long o = (long long)(off[b] + q) * n + off[a] + r;
        Hc[o] = h;
        Sc[o] = sv;
      }
    }
  }
}

// ---------------------------------------------------------------------------------------
// Blocked right-looking Cholesky S^(i) = L L^T (lower; the strictly-upper part is left as
// it was).  A non-positive pivot reports LDC_ERR_NOT_SPD for the cluster.
__global__ void __launch_bounds__(256) potrf_kernel(int n_clusters, const int *__restrict__ order,
                                                    double *__restrict__ mat, const long long *__restrict__ mat_off,
                                                    const int *__restrict__ dmax, const int *__restrict__ dim,
                                                    DevStatus *st) {
  __shared__ double L11[NB][NB + 1];
  __shared__ double gl[kGemmLds];
  __shared__ int bad;
  const int tid = threadIdx.x;
  for (int s = blockIdx.x; s < n_clusters; s += gridDim.x) {
    const int c = order[s];
    const int n = dim[c], ld = n;
    double *S = mat + mat_off[c] + (long long)dmax[c] * dmax[c];
    __syncthreads();
    if (tid == 0) bad = 0;
    for (int j0 = 0; j0 < n; j0 += NB) {
      const int jb = min(NB, n - j0);
      __syncthreads();
      for (int e = tid; e < NB * NB; e += blockDim.x) {
        const int r = e % NB, q = e / NB;
        L11[r][q] = (r < jb && q < jb && r >= q) ? S[(long long)(j0 + q) * ld + j0 + r] : 0.0;
      }
      __syncthreads();
      for (int q = 0; q < jb; ++q) {
        if (tid == 0) {
          double piv = L11[q][q];
          if (!(piv > 0.0)) {
            bad = 1;
            piv = 1.0;
          }
          L11[q][q] = sqrt(piv);
        }
        __syncthreads();
        if (tid > q && tid < jb) L11[tid][q] /= L11[q][q];
        __syncthreads();
        for (int e = tid; e < NB * NB; e += blockDim.x) {
          const int r = e % NB, t = e / NB;
          if (t > q && r >= t && r < jb) L11[r][t] -= L11[r][q] * L11[t][q];
        }
        __syncthreads();
      }
      for (int e = tid; e < NB * NB; e += blockDim.x) {
        const int r = e % NB, q = e / NB;
        if (r < jb && q < jb && r >= q) S[(long long)(j0 + q) * ld + j0 + r] = L11[r][q];
      }
      __syncthreads();
      if (bad) break;
      for (int r = j0 + jb + tid; r < n; r += blockDim.x) {
        double x[NB];
#pragma unroll
        for (int q = 0; q < NB; ++q) x[q] = (q < jb) ? S[(long long)(j0 + q) * ld + r] : 0.0;
#pragma unroll
        for (int q = 0; q < NB; ++q) {
          double v = x[q];
#pragma unroll
          for (int t = 0; t < q; ++t) v -= x[t] * L11[q][t];
          x[q] = (q < jb) ? v / L11[q][q] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < NB; ++q)
          if (q < jb) S[(long long)(j0 + q) * ld + r] = x[q];
      }
      __syncthreads();
      if (j0 + jb < n) {
        double *L21 = S + (long long)j0 * ld + j0 + jb;
        wg_gemm_sub<true, true>(S + (long long)(j0 + jb) * ld + j0 + jb, ld, L21, ld, L21, ld, n - j0 - jb, n - j0 - jb,
                                jb, gl);
      }
    }
    __syncthreads();
    if (bad && tid == 0) report(st, LDC_ERR_NOT_SPD, c);
  }
}

// X <- L^{-1} X for lower-triangular L (n x n) and X (n x n), both column-major, ld = n.
__device__ void trsm_lower_left(double *X, const double *L, int n, double (*L11)[NB + 1], double *gl) {
  const int tid = threadIdx.x;
  const int ld = n;
  for (int j0 = 0; j0 < n; j0 += NB) {
    const int jb = min(NB, n - j0);
    __syncthreads();
    for (int e = tid; e < NB * NB; e += blockDim.x) {
      const int r = e % NB, q = e / NB;
      L11[r][q] = (r < jb && q < jb && r >= q) ? L[(long long)(j0 + q) * ld + j0 + r] : 0.0;
    }
    __syncthreads();
    for (int col = tid; col < n; col += blockDim.x) {
      double *xc = X + (long long)col * ld + j0;
      double x[NB];
#pragma unroll
      for (int q = 0; q < NB; ++q) x[q] = (q < jb) ? xc[q] : 0.0;
#pragma unroll
      for (int q = 0; q < NB; ++q) {
        double v = x[q];
#pragma unroll
        for (int t = 0; t < q; ++t) v -= L11[q][t] * x[t];
        x[q] = (q < jb) ? v / L11[q][q] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < NB; ++q)
        if (q < jb) xc[q] = x[q];
    }
    __syncthreads();
    if (j0 + jb < n)
      wg_gemm_sub<false, false>(X + j0 + jb, ld, L + (long long)j0 * ld + j0 + jb, ld, X + j0, ld, n - j0 - jb, n, jb,
                                gl);
  }
  __syncthreads();
}

// Standard form A = L^{-1} H L^{-T}: X = L^{-1} H, transpose, A = L^{-1} X^T (H slot).
__global__ void __launch_bounds__(256) sygst_kernel(int n_clusters, const int *__restrict__ order,
                                                    double *__restrict__ mat, const long long *__restrict__ mat_off,
                                                    const int *__restrict__ dmax, const int *__restrict__ dim) {
  __shared__ double L11[NB][NB + 1];
  __shared__ double gl[kGemmLds];
  const int tid = threadIdx.x;
  for (int s = blockIdx.x; s < n_clusters; s += gridDim.x) {
    const int c = order[s];
    const int n = dim[c];
    double *H = mat + mat_off[c];
    const double *L = H + (long long)dmax[c] * dmax[c];
    trsm_lower_left(H, L, n, L11, gl);
    for (long long e = tid; e < (long long)n * n; e += blockDim.x) {
      const int i = (int)(e % n), j = (int)(e / n);
      if (i > j) {
        const double t = H[(long long)j * n + i];
        H[(long long)j * n + i] = H[(long long)i * n + j];
        H[(long long)i * n + j] = t;
      }
    }
    __syncthreads();
    trsm_lower_left(H, L, n, L11, gl);
  }
}

// ---------------------------------------------------------------------------------------
// Householder tridiagonalization of A (lower triangle, column-major, ld = n):
// Q^T A Q = T with Q = H_0 H_1 ... H_{n-2}, H_k = I - tau_k v_k v_k^T, v_k(k+1) = 1 and
// v_k(k+2:) stored in A(k+2:, k).  One pass per column: the trailing lower triangle gets the
// previous rank-2 update and feeds the product with the new reflector in the same sweep.
// The tracked columns X = [L^{-1} E_i | L^T E_i] (E_i: the centre atom's unit columns)
// are initialised here and replaced by Q^T X, row-major with stride kTrack.
__global__ void __launch_bounds__(256) sytrd_kernel(int n_clusters, const int *__restrict__ order,
                                                    double *__restrict__ mat, const long long *__restrict__ mat_off,
                                                    double *__restrict__ vec, const long long *__restrict__ vec_off,
                                                    const int *__restrict__ dmax, const int *__restrict__ dim,
                                                    const int *__restrict__ n_orb, int nmax) {
  extern __shared__ double sh[];
  double *vprev = sh, *wprev = sh + nmax, *v = sh + 2 * nmax, *prow = sh + 3 * nmax, *pacc = sh + 4 * nmax;
  __shared__ double red[2 * kTrack * 4 + 8];
  __shared__ double scal[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
  for (int s = blockIdx.x; s < n_clusters; s += gridDim.x) {
    const int c = order[s];
    const int n = dim[c], ld = n;
    const int M = n_orb[c];
    const int nt = 2 * M;
    double *A = mat + mat_off[c];
    const double *L = A + (long long)dmax[c] * dmax[c];
    const VecLayout vl = VecLayout::make(dmax[c]);
    double *cv = vec + vec_off[c];
    double *dd = cv + vl.d, *ee = cv + vl.e, *tt = cv + vl.tau, *X = cv + vl.G0;
    __syncthreads();
    // tracked columns: X_u = L^{-1} E_i (nonzero in the last M rows), X_v = L^T E_i
    for (long long e = tid; e < (long long)n * kTrack; e += blockDim.x) X[e] = 0.0;
    for (int i = tid; i < nmax; i += blockDim.x) {
      vprev[i] = 0.0;
      wprev[i] = 0.0;
      v[i] = 0.0;
      prow[i] = 0.0;
    }
    for (int i = tid; i < nw * nmax; i += blockDim.x) pacc[i] = 0.0;
    __syncthreads();
    const int b0 = n - M;
    if (tid < M) {
      const int al = tid;
      // column al of the inverse of the trailing M x M block of L
      double col[kMaxOrb];
      for (int r = 0; r < M; ++r) col[r] = 0.0;
      col[al] = 1.0 / L[(long long)(b0 + al) * ld + b0 + al];
      for (int r = al + 1; r < M; ++r) {
        double acc = 0.0;
        for (int t = al; t < r; ++t) acc += L[(long long)(b0 + t) * ld + b0 + r] * col[t];
        col[r] = -acc / L[(long long)(b0 + r) * ld + b0 + r];
      }
      for (int r = 0; r < M; ++r) X[(long long)(b0 + r) * kTrack + al] = col[r];
    }
    for (long long e = tid; e < (long long)n * M; e += blockDim.x) {
      const int r = (int)(e % n), al = (int)(e / n);
      if (r <= b0 + al) X[(long long)r * kTrack + M + al] = L[(long long)r * ld + b0 + al];
    }
    __syncthreads();
    for (int k = 0; k + 1 < n; ++k) {
      // (1) previous rank-2 update on column k
      for (int i = k + tid; i < n; i += blockDim.x)
        A[(long long)k * ld + i] -= vprev[i] * wprev[k] + wprev[i] * vprev[k];
      __syncthreads();
      // (2) reflector from A(k+1:, k)
      double part = 0.0;
      for (int i = k + 2 + tid; i < n; i += blockDim.x) {
        const double a = A[(long long)k * ld + i];
        part += a * a;
      }
      const double sigma = block_sum(part, red);
      const double alpha = A[(long long)k * ld + k + 1];
      double beta, tau, sc;
      if (sigma == 0.0) {
        tau = 0.0;
        beta = alpha;
        sc = 0.0;
      } else {
        beta = -copysign(sqrt(alpha * alpha + sigma), alpha);
        tau = (beta - alpha) / beta;
        sc = 1.0 / (alpha - beta);
      }
      for (int i = tid; i < n; i += blockDim.x) {
        double vi = 0.0;
        if (i == k + 1) vi = 1.0;
        else if (i > k + 1) {
          vi = A[(long long)k * ld + i] * sc;
          A[(long long)k * ld + i] = vi;
        }
        v[i] = vi;
      }
      if (tid == 0) {
        dd[k] = A[(long long)k * ld + k];
        ee[k] = beta;
        tt[k] = tau;
      }
      __syncthreads();
      // (3) trailing lower triangle: apply the previous update and accumulate A22 v
      for (int i0 = k + 1 + wave * 64; i0 < n; i0 += blockDim.x) {
        const int i = i0 + lane;
        const bool rowok = i < n;
        const double vpi = rowok ? vprev[i] : 0.0, wpi = rowok ? wprev[i] : 0.0, vi = rowok ? v[i] : 0.0;
        double racc = 0.0;
        const int jend = min(i0 + 63, n - 1);
        for (int j = k + 1; j <= jend; ++j) {
          double cp = 0.0;
          if (rowok && i >= j) {
            double *pa = A + (long long)j * ld + i;
            const double a = *pa - (vpi * wprev[j] + wpi * vprev[j]);
            *pa = a;
            racc += a * v[j];
            if (i > j) cp = a * vi;
          }
          cp = wave_sum(cp);
          if (lane == 0) pacc[wave * nmax + j] += cp;
        }
        if (rowok) prow[i] = racc;
      }
      __syncthreads();
      // (4) p = tau A22 v, w = p - (tau/2)(p.v) v
      double pv = 0.0;
      for (int i = k + 1 + tid; i < n; i += blockDim.x) {
        double p = prow[i];
        for (int w = 0; w < nw; ++w) p += pacc[w * nmax + i];
        p *= tau;
        prow[i] = p;
        pv += p * v[i];
      }
      pv = block_sum(pv, red);
      for (int i = tid; i < n; i += blockDim.x) {
        if (i > k) {
          wprev[i] = prow[i] - 0.5 * tau * pv * v[i];
          vprev[i] = v[i];
        } else {
          wprev[i] = 0.0;
          vprev[i] = 0.0;
        }
        for (int w = 0; w < nw; ++w) pacc[w * nmax + i] = 0.0;
      }
      // (5) tracked columns: X(k+1:, :) -= tau v (v^T X(k+1:, :))
      if (tau != 0.0) {
        double pc[kTrack];
#pragma unroll
        for (int q = 0; q < kTrack; ++q) pc[q] = 0.0;
        for (int i = k + 1 + tid; i < n; i += blockDim.x) {
          const double vi = v[i];
          for (int q = 0; q < nt; ++q) pc[q] += vi * X[(long long)i * kTrack + q];
        }
        __syncthreads();
        for (int q = 0; q < nt; ++q) {
          const double t = wave_sum(pc[q]);
          if (lane == 0) red[wave * kTrack + q] = t;
        }
        __syncthreads();
        for (int e = tid; e < (n - k - 1) * nt; e += blockDim.x) {
          const int i = k + 1 + e / nt, q = e % nt;
          double sq = 0.0;
          for (int w = 0; w < nw; ++w) sq += red[w * kTrack + q];
          X[(long long)i * kTrack + q] -= tau * sq * v[i];
        }
      }
      __syncthreads();
    }
    if (tid == 0) {
      dd[n - 1] = A[(long long)(n - 1) * ld + n - 1];
      if (n >= 1) ee[n - 1] = 0.0;
    }
  }
}

// ---------------------------------------------------------------------------------------
void launch_gather(Plan &p, const double *d_H, const double *d_S) {
  hipLaunchKernelGGL(gather_kernel, dim3(p.workgroups), dim3(kWG), 0, p.stream, p.n_atoms, p.d_order, p.d_mem_ptr,
                     p.d_mem_atom, p.d_mem_long, p.d_pair_ptr, p.d_pair_ab, p.d_pair_blk, p.d_n_orb, p.d_blk_off, d_H,
                     d_S, p.lno_mode, p.d_rank, p.d_U, p.d_mat, p.d_mat_off, p.d_dmax, p.d_dim);
}

void launch_potrf(Plan &p) {
  hipLaunchKernelGGL(potrf_kernel, dim3(p.workgroups), dim3(kWG), 0, p.stream, p.n_atoms, p.d_order, p.d_mat,
                     p.d_mat_off, p.d_dmax, p.d_dim, p.d_status);
}

void launch_sygst(Plan &p) {
  hipLaunchKernelGGL(sygst_kernel, dim3(p.workgroups), dim3(kWG), 0, p.stream, p.n_atoms, p.d_order, p.d_mat,
                     p.d_mat_off, p.d_dmax, p.d_dim);
}

void launch_sytrd(Plan &p) {
  const int nmax = p.max_dim;
  const size_t lds = sizeof(double) * (size_t)nmax * (4 + kWG / 64);
  hipLaunchKernelGGL(sytrd_kernel, dim3(p.workgroups), dim3(kWG), lds, p.stream, p.n_atoms, p.d_order, p.d_mat,
                     p.d_mat_off, p.d_vec, p.d_vec_off, p.d_dmax, p.d_dim, p.d_n_orb, nmax);
}

}  // namespace ldc
