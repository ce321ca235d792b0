// Cluster problem kernels (Sec. II.C (ii)-(iii)): gather of H^(i), S^(i) with PAO/LNO
// blocks (Eq. 26), Cholesky of S^(i), reduction to the standard problem and Householder
// tridiagonalization.  One 256-thread workgroup per cluster; workgroups walk the clusters
// largest-first with a fixed stride (persistent launch, deterministic assignment).
#include "wg_blas.h"
#include "wg_qapply.h"

#include <algorithm>

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
// Rows times a small triangular factor held in LDS:
//   dst(r, q) = sum_t src(r, t) F(q, t)   (F_T: F(t, q)),  r < m, q < jb,
// with F = Li (NB x NB, padded with zeros).  src and dst are column-major (leading
// dimensions lds_, ldd) and may be the same memory: rows are staged through LDS (64 per
// step, buffer of 64 (NB + 1) doubles) before they are overwritten.  Thread (rr, q0) forms
// the outputs (rr, q0 + 4 j).
template <bool F_T>
__device__ void wg_rows_times_small(const double *src, int lds_, double *dst, int ldd, int m, int jb,
                                    const double (*Li)[NB + 1], double *stage) {
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int rr = tid & 63, q0 = tid >> 6;
  for (int r0 = 0; r0 < m; r0 += 64) {
    const int rows = min(64, m - r0);
    __syncthreads();
    for (int e = tid; e < 64 * NB; e += nthr) {
      const int r = e & 63, t = e >> 6;
      stage[r * (NB + 1) + t] = (r < rows && t < jb) ? src[t * lds_ + r0 + r] : 0.0;
    }
    __syncthreads();
    double acc[NB / 4];
#pragma unroll
    for (int j = 0; j < NB / 4; ++j) acc[j] = 0.0;
#pragma unroll 2
    for (int t = 0; t < NB; ++t) {
      const double a = stage[rr * (NB + 1) + t];
#pragma unroll
      for (int j = 0; j < NB / 4; ++j) {
        const int q = q0 + 4 * j;
        acc[j] += a * (F_T ? Li[q][t] : Li[t][q]);
      }
    }
    if (rr < rows) {
#pragma unroll
      for (int j = 0; j < NB / 4; ++j) {
        const int q = q0 + 4 * j;
        if (q < jb) dst[q * ldd + r0 + rr] = acc[j];
      }
    }
  }
  __syncthreads();
}

// 32 x 32 lower-triangular inverse in LDS: Li = L11^{-1} (column c by thread c, forward
// substitution).  Entries above the diagonal of Li are set to zero.
__device__ inline void lds_tri_inverse(double (*L11)[NB + 1], double (*Li)[NB + 1], int jb) {
  const int tid = threadIdx.x;
  if (tid < NB) {
    const int c = tid;
    for (int r = 0; r < NB; ++r) {
      double val = 0.0;
      if (c < jb && r < jb && r >= c) {
        double acc = (r == c) ? 1.0 : 0.0;
        for (int t = c; t < r; ++t) acc -= L11[r][t] * Li[t][c];
        val = acc / L11[r][r];
      }
      Li[r][c] = val;
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------------------
// Blocked right-looking Cholesky S^(i) = L L^T (lower; the strictly-upper part is left as
// it was).  Per panel: unblocked factor of the diagonal block in LDS, its inverse, the
// panel below as L21 = A21 L11^{-T}, and the trailing update A22 -= L21 L21^T (MFMA GEMM).
// A non-positive pivot reports LDC_ERR_NOT_SPD for the cluster.
__global__ void __launch_bounds__(256, 2) potrf_kernel(int n_clusters, const int *__restrict__ order,
                                                       double *__restrict__ mat, const long long *__restrict__ mat_off,
                                                       const int *__restrict__ dmax, const int *__restrict__ dim,
                                                       DevStatus *st) {
  __shared__ double L11[NB][NB + 1];
  __shared__ double Li[NB][NB + 1];
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
      const int m = n - j0 - jb;
      if (m > 0) {
        lds_tri_inverse(L11, Li, jb);
        double *P = S + (long long)j0 * ld + j0 + jb;
        wg_rows_times_small<true>(P, ld, P, ld, m, jb, Li, gl);
        wg_gemm_sub<true, true>(S + (long long)(j0 + jb) * ld + j0 + jb, ld, P, ld, P, ld, m, m, jb, gl);
      }
    }
    __syncthreads();
    if (bad && tid == 0) report(st, LDC_ERR_NOT_SPD, c);
  }
}

// Standard form (Sec. II.C (iii) via Cholesky): with S = L L^T,
//   A = L^{-1} H L^{-T}.
// 1. L^{-1} in place of L (block columns from the last: B21 <- -L22^{-1} L21 L11^{-1},
//    L11 <- L11^{-1}); the strictly-upper part of the S slot is cleared first.
// 2. W = L^{-1} H in place of H, block rows from the last (each block row only needs rows
//    of H above it, which are still intact).
// 3. A = L^{-1} W^T (lower part) in place of W, block rows from the last.
// All products are MFMA GEMMs that skip the structurally zero part of L^{-1}.  The tracked
// columns of the tridiagonal solver are set up here: X_u = L^{-1} E_i (the last M columns of
// L^{-1}) and X_v = L^T E_i (the last M rows of L, taken before the inversion).
__global__ void __launch_bounds__(256, 2) sygst_kernel(int n_clusters, const int *__restrict__ order,
                                                    double *__restrict__ mat, const long long *__restrict__ mat_off,
                                                    double *__restrict__ vec, const long long *__restrict__ vec_off,
                                                    const int *__restrict__ dmax, const int *__restrict__ dim,
                                                    const int *__restrict__ n_orb) {
  __shared__ double L11[NB][NB + 1];
  __shared__ double Li[NB][NB + 1];
  __shared__ double gl[kGemmLds];
  const int tid = threadIdx.x, nthr = blockDim.x;
  for (int s = blockIdx.x; s < n_clusters; s += gridDim.x) {
    const int c = order[s];
    const int n = dim[c], ld = n;
    const int M = n_orb[c];
    double *H = mat + mat_off[c];
    double *L = H + (long long)dmax[c] * dmax[c];
    const VecLayout vl = VecLayout::make(dmax[c]);
    double *cv = vec + vec_off[c];
    double *X = cv + vl.G0;
    double *tmp = cv + vl.G1;  // n x NB scratch (column-major, ld n)
    const int b0 = n - M;
    __syncthreads();
    // tracked columns: X_v = L^T E_i (rows of L of the centre atom); X_u filled below
    for (long long e = tid; e < (long long)n * kTrack; e += nthr) X[e] = 0.0;
    __syncthreads();
    for (long long e = tid; e < (long long)n * M; e += nthr) {
      const int r = (int)(e % n), al = (int)(e / n);
      if (r <= b0 + al) X[(long long)r * kTrack + M + al] = L[(long long)r * ld + b0 + al];
    }
    // clear the strictly-upper triangle of the S slot
    for (long long e = tid; e < (long long)n * n; e += nthr) {
      const int r = (int)(e % n), q = (int)(e / n);
      if (r < q) L[e] = 0.0;
    }
    __syncthreads();
    // 1. L <- L^{-1}
    const int nblk = (n + NB - 1) / NB;
    for (int bj = nblk - 1; bj >= 0; --bj) {
      const int j = bj * NB, jb = min(NB, n - j);
      for (int e = tid; e < NB * NB; e += nthr) {
        const int r = e % NB, q = e / NB;
        L11[r][q] = (r < jb && q < jb && r >= q) ? L[(long long)(j + q) * ld + j + r] : 0.0;
      }
      __syncthreads();
      lds_tri_inverse(L11, Li, jb);
      const int m = n - j - jb;
      if (m > 0) {
        // tmp = -L22^{-1} L21
        wg_gemm_sub<false, false, false, false, true>(tmp, n, L + (long long)(j + jb) * ld + j + jb, ld,
                                                       L + (long long)j * ld + j + jb, ld, m, jb, m, gl, 0);
        // L21 <- tmp L11^{-1}
        wg_rows_times_small<false>(tmp, n, L + (long long)j * ld + j + jb, ld, m, jb, Li, gl);
      }
      for (int e = tid; e < NB * NB; e += nthr) {
        const int r = e % NB, q = e / NB;
        if (r < jb && q < jb && r >= q) L[(long long)(j + q) * ld + j + r] = Li[r][q];
      }
      __syncthreads();
    }
    // X_u = L^{-1} E_i: rows b0.. of the last M columns of L^{-1}
    for (int e = tid; e < M * M; e += nthr) {
      const int r = e % M, al = e / M;
      X[(long long)(b0 + r) * kTrack + al] = (r >= al) ? L[(long long)(b0 + al) * ld + b0 + r] : 0.0;
    }
    // 2. W = L^{-1} H, block rows from the last (tmp holds -W_b, NB x n, ld NB)
    for (int bj = nblk - 1; bj >= 0; --bj) {
      const int r0 = bj * NB, jb = min(NB, n - r0), r1 = r0 + jb;
      wg_gemm_sub<false, false, false, false, true>(tmp, NB, L + r0, ld, H, ld, jb, n, r1, gl, r0);
      for (long long e = tid; e < (long long)jb * n; e += nthr) {
        const int rr = (int)(e % jb), q = (int)(e / jb);
        H[(long long)q * ld + r0 + rr] = -tmp[(long long)q * NB + rr];
      }
      __syncthreads();
    }
    // 3. A = L^{-1} W^T, lower part: block row b of A = L^{-1}(rows b, cols 0:r1) W(0:r1, 0:r1)^T
    for (int bj = nblk - 1; bj >= 0; --bj) {
      const int r0 = bj * NB, jb = min(NB, n - r0), r1 = r0 + jb;
      wg_gemm_sub<true, false, false, false, true>(tmp, NB, L + r0, ld, H, ld, jb, r1, r1, gl, r0);
      for (long long e = tid; e < (long long)jb * r1; e += nthr) {
        const int rr = (int)(e % jb), q = (int)(e / jb);
        H[(long long)q * ld + r0 + rr] = -tmp[(long long)q * NB + rr];
      }
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------------------
// Partial products of y = A v for the symmetric m x m matrix held in the lower triangle of
// A (column-major, leading dimension lda), streamed by whole columns.  The columns form
// strips of SC; wave w takes the strips w, w + nw, ... and walks each from its diagonal
// down in chunks of 64 SU rows (lane = row).  The loads of the next chunk are issued before
// the current one is used (two chunks in flight per wave).  For every row the strip's
// contribution to y(r) goes to the wave's private partial row my (LDS, no workgroup
// barrier needed); each column's stored part feeds y(c) through one wave reduction per
// strip.  The caller sums the nw partial rows.
constexpr int SU = 2;
constexpr int SC = 8;
__device__ void wg_symv_lower_partial(const double *__restrict__ A, int lda, int m, const double *v, double *my) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int r = lane; r < m; r += 64) my[r] = 0.0;
  int s = wave, r0 = s * SC;
  if (r0 >= m) return;
  // Rows and columns past the end are clamped, so the loads are unconditional (all in
  // flight together); entries outside the lower triangle are masked where they are used.
  auto fetch = [&](int st, int rs, double (*a)[SC]) {
    const int c0 = st * SC;
#pragma unroll
    for (int u = 0; u < SU; ++u) {
      const int r = rs + u * 64 + lane, rc = r < m ? r : m - 1;
#pragma unroll
      for (int j = 0; j < SC; ++j) {
        const int cc = c0 + j < m ? c0 + j : m - 1;
        a[u][j] = A[cc * lda + rc];
      }
    }
  };
  double cur[SU][SC], nxt[SU][SC], acc[SC], vc[SC];
  fetch(s, r0, cur);
#pragma unroll
  for (int j = 0; j < SC; ++j) {
    acc[j] = 0.0;
    vc[j] = (r0 + j < m) ? v[r0 + j] : 0.0;
  }
  while (true) {
    int ns = s, nr0 = r0 + 64 * SU;
    if (nr0 >= m) {
      ns = s + nw;
      nr0 = ns * SC;
    }
    const bool more = nr0 < m;
    if (more) fetch(ns, nr0, nxt);
    const int c0 = s * SC;
#pragma unroll
    for (int u = 0; u < SU; ++u) {
      const int r = r0 + u * 64 + lane;
      if (r < m) {
        const double vr = v[r];
        double t = 0.0;
#pragma unroll
        for (int j = 0; j < SC; ++j) {
          const double x = (r >= c0 + j) ? cur[u][j] : 0.0;
          t += x * vc[j];
          if (r > c0 + j) acc[j] += x * vr;
        }
        my[r] += t;
      }
    }
    if (ns != s) {
#pragma unroll
      for (int j = 0; j < SC; ++j) {
        const double t = wave_sum(acc[j]);
        if (lane == 0 && c0 + j < m) my[c0 + j] += t;
        acc[j] = 0.0;
        vc[j] = (more && nr0 + j < m) ? v[nr0 + j] : 0.0;
      }
    }
    if (!more) break;
    s = ns;
    r0 = nr0;
#pragma unroll
    for (int u = 0; u < SU; ++u)
#pragma unroll
      for (int j = 0; j < SC; ++j) cur[u][j] = nxt[u][j];
  }
}

constexpr int NBT = 32;        // panel width of the tridiagonalization
constexpr int VWS = 2 * NBT;  // row stride of [V | W]

// out(r) = [V | W](r, :) . cf for rows r in [r_begin, r_end) of the row-major n x 2 NBT block
// [V | W] (cf: 2 NBT coefficients in LDS).  Eight lanes share a row (each reads 8 contiguous
// doubles, whole cache lines per wave) and combine their parts with three shuffles; a
// workgroup step covers 4 x 32 rows (loads of all four in flight together; rows past the end
// are clamped).  f(r, value) is called by the first lane of each group.
template <class F>
__device__ void wg_rows_dot_vw(const double *__restrict__ VW, int r_begin, int r_end, const double *cf, F f) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int g = lane >> 3, sub = lane & 7;
  static_assert(VWS == 64, "eight lanes of eight coefficients per row");
  double c[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) c[q] = cf[sub * 8 + q];
  constexpr int RU = 4;
  for (int r0 = r_begin; r0 < r_end; r0 += RU * 8 * nw) {
    double x[RU][8];
#pragma unroll
    for (int u = 0; u < RU; ++u) {
      const int r = r0 + (u * nw + wave) * 8 + g, rc = r < r_end ? r : r_end - 1;
      const double *row = VW + (long long)rc * VWS + sub * 8;
#pragma unroll
      for (int q = 0; q < 8; ++q) x[u][q] = row[q];
    }
#pragma unroll
    for (int u = 0; u < RU; ++u) {
      const int r = r0 + (u * nw + wave) * 8 + g;
      double part = 0.0;
#pragma unroll
      for (int q = 0; q < 8; ++q) part += x[u][q] * c[q];
      part += __shfl_xor(part, 1, 64);
      part += __shfl_xor(part, 2, 64);
      part += __shfl_xor(part, 4, 64);
      if (sub == 0 && r < r_end) f(r, part);
    }
  }
}

// Householder tridiagonalization of A (lower triangle, column-major, ld = n), blocked:
// Q^T A Q = T with Q = H_0 H_1 ... H_{n-2}, H_k = I - tau_k v_k v_k^T, v_k(k+1) = 1 and
// v_k(k+2:) stored in A(k+2:, k).  Panels of NBT columns: inside a panel each column takes
// the updates of the panel's earlier reflectors from the n x 2 NBT block [V | W] (row-major,
// so a row's coefficients are one contiguous load), its reflector is generated, and
// w = tau (A v - V (W^T v) - W (V^T v)) - (tau/2)(w^T v) v uses the trailing matrix as left
// by the previous panel; after the panel the trailing matrix gets A -= V W^T + W V^T (one
// tiled MFMA GEMM over its lower triangle, [V | W] times [W | V]^T).
// The tracked columns X = [L^{-1} E_i | L^T E_i] (E_i: the centre atom's unit columns) are
// replaced by Q^T X (row-major, stride kTrack).
__global__ void __launch_bounds__(256, 2) sytrd_kernel(int n_clusters, const int *__restrict__ order,
                                                       double *__restrict__ mat, const long long *__restrict__ mat_off,
                                                       double *__restrict__ vec, const long long *__restrict__ vec_off,
                                                       const int *__restrict__ dmax, const int *__restrict__ dim,
                                                       const int *__restrict__ n_orb, int nmax) {
  extern __shared__ double sh[];
  double *v = sh, *y = sh + nmax, *yw = sh + 2 * nmax;
  __shared__ double red[8];
  __shared__ double coef[2 * NBT];
  __shared__ double dpart[4 * 64];
  __shared__ double rowk[2 * NBT];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6, nthr = blockDim.x;
  for (int s = blockIdx.x; s < n_clusters; s += gridDim.x) {
    const int c = order[s];
    const int n = dim[c], ld = n;
    const int M = n_orb[c];
    const int nt = 2 * M;
    double *A = mat + mat_off[c];
    const VecLayout vl = VecLayout::make(dmax[c]);
    double *cv = vec + vec_off[c];
    double *dd = cv + vl.d, *ee = cv + vl.e, *tt = cv + vl.tau, *X = cv + vl.G0;
    double *VW = cv + vl.G1;  // n x 2 NBT, row-major (spans G1 and u; u takes the T factors at the end)
    __syncthreads();
    for (long long e = tid; e < (long long)n * VWS; e += nthr) VW[e] = 0.0;
    __syncthreads();
    for (int j0 = 0; j0 + 1 < n; j0 += NBT) {
      const int j1 = min(j0 + NBT, n - 1);
      const int nbp = j1 - j0;
      for (int i = 0; i < nbp; ++i) {
        const int k = j0 + i;
        // (1) column k takes the panel's earlier updates: A(:,k) -= V W(k,:)^T + W V(k,:)^T
        //     (the products run over all NBT columns: the columns >= i of V and W are zero)
        if (i > 0) {
          if (tid < VWS) rowk[tid] = VW[(long long)k * VWS + ((tid + NBT) & (VWS - 1))];
          __syncthreads();
          double *ak = A + (long long)k * ld;
          wg_rows_dot_vw(VW, k, n, rowk, [&](int r, double x) { ak[r] -= x; });
        }
        __syncthreads();
        // (2) reflector from A(k+1:, k)
        double part = 0.0;
        for (int r = k + 2 + tid; r < n; r += nthr) {
          const double a = A[(long long)k * ld + r];
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
        for (int r = tid; r < n; r += nthr) {
          double vr = 0.0;
          if (r == k + 1) vr = 1.0;
          else if (r > k + 1) {
            vr = A[(long long)k * ld + r] * sc;
            A[(long long)k * ld + r] = vr;
          }
          v[r] = vr;
          VW[(long long)r * VWS + i] = vr;
        }
        if (tid == 0) {
          dd[k] = A[(long long)k * ld + k];
          ee[k] = beta;
          tt[k] = tau;
        }
        __syncthreads();
        if (tau == 0.0) {
          for (int r = tid; r < n; r += nthr) VW[(long long)r * VWS + NBT + i] = 0.0;
          __syncthreads();
          continue;
        }
        const int m = n - k - 1;
        // (3) per-wave partial rows of A(k+1:, k+1:) v(k+1:); before that every wave forms
        //     partial sums of W(:,t)^T v (lanes 0..31) and V(:,t)^T v (lanes 32..63) over
        //     its share of the rows
        {
          const double *base = VW + ((lane + NBT) & (VWS - 1));
          double acc = 0.0;
          if ((lane & (NBT - 1)) < i) {
            // 16 rows per step; rows past the end are clamped and masked, so the loads are
            // unconditional and issue back to back
            for (int r0 = k + 1 + wave; r0 < n; r0 += 16 * nw) {
              double a[16], b[16];
#pragma unroll
              for (int u = 0; u < 16; ++u) {
                const int r = r0 + u * nw, rc = r < n ? r : n - 1;
                a[u] = base[(long long)rc * VWS];
                b[u] = r < n ? v[rc] : 0.0;
              }
#pragma unroll
              for (int u = 0; u < 16; ++u) acc += a[u] * b[u];
            }
          }
          dpart[wave * 64 + lane] = acc;
        }
        wg_symv_lower_partial(A + (long long)(k + 1) * ld + k + 1, ld, m, v + k + 1, yw + wave * nmax);
        __syncthreads();
        if (tid < 64) {
          double a = 0.0;
          for (int w = 0; w < nw; ++w) a += dpart[w * 64 + tid];
          coef[tid] = a;
        }
        __syncthreads();
        // (4) w = tau (A v - V (W^T v) - W (V^T v)); w -= (tau/2)(w^T v) v
        double wvp = 0.0;
        wg_rows_dot_vw(VW, k + 1, n, coef, [&](int r, double x) {
          double acc = 0.0;
          for (int w = 0; w < nw; ++w) acc += yw[w * nmax + r - k - 1];
          acc = (acc - x) * tau;
          y[r] = acc;
          wvp += acc * v[r];
        });
        const double wv = block_sum(wvp, red);
        const double al = -0.5 * tau * wv;
        for (int r = k + 1 + tid; r < n; r += nthr) VW[(long long)r * VWS + NBT + i] = y[r] + al * v[r];
        __syncthreads();
      }
      // trailing update A(j1:, j1:) -= V2 W2^T + W2 V2^T (lower triangle); the GEMM stages
      // its tiles in the LDS that held v, y and the partial rows
      const int m2 = n - j1;
      if (m2 > 0) {
        const double *P = VW + (long long)j1 * VWS;
        wg_gemm_sub<true, true, true, true>(A + (long long)j1 * ld + j1, ld, P, VWS, P, VWS, m2, m2, VWS, sh, -1, NBT);
      }
      // the next panel starts from zero V, W
      for (long long e = tid; e < (long long)n * VWS; e += nthr) VW[e] = 0.0;
      __syncthreads();
    }
    if (tid == 0) {
      dd[n - 1] = A[(long long)(n - 1) * ld + n - 1];
      ee[n - 1] = 0.0;
    }
    // tracked columns: X <- Q^T X, panel by panel in compact WY form (T factors kept for
    // the density step)
    __syncthreads();
    wg_apply_q(A, ld, n, tt, cv + vl.u, true, X, kTrack, nt, true, sh);
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
                     p.d_mat_off, p.d_vec, p.d_vec_off, p.d_dmax, p.d_dim, p.d_n_orb);
}

void launch_sytrd(Plan &p) {
  const int nmax = p.max_dim;
  const size_t lds =
      sizeof(double) * std::max({(size_t)nmax * (2 + kWG / 64), (size_t)kQapplyLds, (size_t)kGemmLds});
  hipLaunchKernelGGL(sytrd_kernel, dim3(p.workgroups), dim3(kWG), lds, p.stream, p.n_atoms, p.d_order, p.d_mat,
                     p.d_mat_off, p.d_vec, p.d_vec_off, p.d_dmax, p.d_dim, p.d_n_orb, nmax);
}

}  // namespace ldc
