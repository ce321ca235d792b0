// Cluster problem kernels (Sec. II.C (ii)-(iii)): gather of H^(i), S^(i) with PAO/LNO
// blocks (Eq. 26), Cholesky of S^(i) and reduction to the standard problem (the
// tridiagonalization is in k_tridiag.hip).  One 256-thread workgroup per cluster;
// workgroups walk the clusters largest-first with a fixed stride (persistent launch,
// deterministic assignment).
#include "wg_blas.h"
#include "wg_qapply.h"

#include <algorithm>

namespace ldc {

constexpr int NB = 32;  // panel width of the blocked factorizations

// ---------------------------------------------------------------------------------------
// LNO blocks of Eq. 26 for every pattern block (i, j), formed once per call and shared by all
// clusters in which i or j is a long member: out[(2 v + x) total + blk_off[b] + ...] holds,
// row-major, v = 0: U_i^T X_ij (k_i x M_j), v = 1: X_ij U_j (M_i x k_j), v = 2: U_i^T X_ij U_j
// (k_i x k_j), for x = 0: X = H, x = 1: X = S.  U_j is column-major M_j x k_j (ld M_j).
// One workgroup per atom row i; each wave takes one block of the row at a time.
// TH: arithmetic of the H contractions (double, or float in the precision form: the entries are
// rounded to FP32 and accumulated in FP32; the results are stored as FP64 values).  The S
// contractions are always FP64 (the cluster overlap stays exact, so that C^T S C = I and the
// electron count g Tr(D S) keep FP64 accuracy).
template <typename TH>
__global__ void __launch_bounds__(256) lno_blocks_kernel(int n_atoms, const int *__restrict__ row_ptr,
                                                         const int *__restrict__ col, const int *__restrict__ n_orb,
                                                         const long long *__restrict__ blk_off,
                                                         const int *__restrict__ rank, const double *__restrict__ U,
                                                         const double *__restrict__ H, const double *__restrict__ S,
                                                         double *__restrict__ out, long long total) {
  constexpr int Q = kMaxOrb * kMaxOrb;
  __shared__ double ui[Q];
  __shared__ double uj[4][Q], xs[4][Q], xu[4][Q];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int i = blockIdx.x; i < n_atoms; i += gridDim.x) {
    const int Mi = n_orb[i], ki = rank[i];
    const int b0 = row_ptr[i], nb = row_ptr[i + 1] - b0;
    __syncthreads();
    for (int e = tid; e < Mi * ki; e += blockDim.x) ui[e] = U[(long long)i * Q + e];
    // every wave runs the same number of rounds so that the barriers match
    for (int t0 = 0; t0 < nb; t0 += 4) {
      const int bl = t0 + wave;
      const bool act = bl < nb;
      const int b = b0 + (act ? bl : 0), j = col[b];
      const int Mj = n_orb[j], kj = rank[j];
      const long long bo = blk_off[b];
      if (act)
        for (int e = lane; e < Mj * kj; e += 64) uj[wave][e] = U[(long long)j * Q + e];
      for (int x = 0; x < 2; ++x) {
        const double *X = (x ? S : H) + bo;
        __syncthreads();
        if (act)
          for (int e = lane; e < Mi * Mj; e += 64) xs[wave][e] = X[e];
        __syncthreads();
        // the three products in the arithmetic of this matrix (type of the tag)
        auto contract = [&](auto tag) {
          using TC = decltype(tag);
          if (act) {
            double *o0 = out + (long long)x * total + bo;            // U_i^T X
            double *o1 = out + (long long)(2 + x) * total + bo;      // X U_j
            for (int e = lane; e < Mi * kj; e += 64) {
              const int r = e / kj, q = e % kj;
              TC a = 0;
              for (int be = 0; be < Mj; ++be) a += (TC)xs[wave][r * Mj + be] * (TC)uj[wave][be + q * Mj];
              xu[wave][e] = (double)a;
              o1[e] = (double)a;
            }
            for (int e = lane; e < ki * Mj; e += 64) {
              const int r = e / Mj, q = e % Mj;
              TC a = 0;
              for (int al = 0; al < Mi; ++al) a += (TC)ui[al + r * Mi] * (TC)xs[wave][al * Mj + q];
              o0[e] = (double)a;
            }
          }
          __syncthreads();
          if (act) {
            double *o2 = out + (long long)(4 + x) * total + bo;      // U_i^T X U_j
            for (int e = lane; e < ki * kj; e += 64) {
              const int r = e / kj, q = e % kj;
              TC a = 0;
              for (int al = 0; al < Mi; ++al) a += (TC)ui[al + r * Mi] * (TC)xu[wave][al * kj + q];
              o2[e] = (double)a;
            }
          }
        };
        if (x == 0) contract(TH{});
        else contract(double{});
      }
    }
  }
}

// ---------------------------------------------------------------------------------------
// (a)+(c) gather: dense column-major H^(i), S^(i) (leading dimension = cluster dimension n),
// written column block by column block, every element once (zeros included).  The H slot
// receives H_L, the lower triangle of H^(i) with half its diagonal and zeros above
// (H^(i) = H_L + H_L^T; the standard form works from H_L), each column in full; the S slot
// each column of S^(i) from its diagonal block down.  The (a, b) block of the cluster matrix is C_a X_ab C_b with C the LNO contraction of a
// long member (identity otherwise); by the symmetry of H and S it is read as the transpose of
// the row-b pattern block X_ba or its contraction from lno_blocks_kernel (U_b^T X_ba, X_ba U_a
// or U_b^T X_ba U_a), whose rows have length d_a either way, so that a column of the cluster
// matrix reads contiguous runs of each block row.
// Dynamic LDS: n 16-bit member indices (row -> member).
__global__ void __launch_bounds__(256) gather_kernel(int n_clusters, const int *__restrict__ order,
                                                     const int *__restrict__ mem_ptr, const int *__restrict__ mem_atom,
                                                     const int *__restrict__ mem_long, const int *__restrict__ pair_ptr,
                                                     const int *__restrict__ pair_ab, const int *__restrict__ pair_blk,
                                                     const int *__restrict__ n_orb, const long long *__restrict__ blk_off,
                                                     const double *__restrict__ H, const double *__restrict__ S,
                                                     int lno_mode, const int *__restrict__ rank,
                                                     const double *__restrict__ lno_blk, long long total,
                                                     double *__restrict__ mat,
                                                     const long long *__restrict__ mat_off, const int *__restrict__ dmax,
                                                     int *__restrict__ dim, int round32, int *__restrict__ queue) {
  extern __shared__ __attribute__((aligned(16))) unsigned short rowmem[];
  __shared__ int off[kMaxMembers + 1];
  __shared__ int dm[kMaxMembers];
  __shared__ unsigned char lng[kMaxMembers];
  __shared__ int rs[kMaxMembers], re[kMaxMembers];  // pairs of member row a: [rs[a], re[a])
  __shared__ long long pbo[kMaxMembers];            // block offset of (b, a) for the current b, or -1
  const int tid = threadIdx.x;
  for (int s = queue_next(queue); s < n_clusters; s = queue_next(queue)) {
    const int c = order[s];
    const int mb = mem_ptr[c], nm = mem_ptr[c + 1] - mb;
    const int p0 = pair_ptr[c], p1 = pair_ptr[c + 1];
    __syncthreads();
    for (int a = tid; a < nm; a += blockDim.x) {
      const int atom = mem_atom[mb + a];
      const bool lg = lno_mode && mem_long[mb + a];
      dm[a] = lg ? rank[atom] : n_orb[atom];
      lng[a] = lg;
      rs[a] = 0;
      re[a] = 0;
    }
    __syncthreads();
    if (tid == 0) {
      off[0] = 0;
      for (int a = 0; a < nm; ++a) off[a + 1] = off[a] + dm[a];
      dim[c] = off[nm];
    }
    // the pairs are grouped by row member: mark where each group starts and ends
    for (int q = p0 + tid; q < p1; q += blockDim.x) {
      const int a = pair_ab[q] & 0xffff;
      if (q == p0 || (pair_ab[q - 1] & 0xffff) != a) rs[a] = q;
      if (q == p1 - 1 || (pair_ab[q + 1] & 0xffff) != a) re[a] = q + 1;
    }
    __syncthreads();
    const int n = off[nm];
    for (int a = 0; a < nm; ++a)
      for (int r = off[a] + tid; r < off[a + 1]; r += blockDim.x) rowmem[r] = (unsigned short)a;
    double *Hc = mat + mat_off[c];
    double *Sc = Hc + (long long)dmax[c] * dmax[c];
    for (int b = 0; b < nm; ++b) {
      __syncthreads();
      for (int a = tid; a < nm; a += blockDim.x) pbo[a] = -1;
      __syncthreads();
      for (int q = rs[b] + tid; q < re[b]; q += blockDim.x) pbo[pair_ab[q] >> 16] = blk_off[pair_blk[q]];
      __syncthreads();
      const int db = dm[b], cb = off[b];
      const bool lb = lng[b];
      for (int r = tid; r < n; r += blockDim.x) {
        const int a = rowmem[r], da = dm[a], rr = r - off[a];
        const long long bo = pbo[a];
        const bool la = lng[a];
        // variant of the (b, a) block: rows contracted when b is long, columns when a is
        const int v = lb ? (la ? 2 : 0) : 1;
        const double *hb = (la || lb) ? lno_blk + (long long)(2 * v) * total : H;
        const double *sb = (la || lb) ? lno_blk + (long long)(2 * v + 1) * total : S;
        const long long src = bo + rr;
        // S above the diagonal block is never read (the Cholesky reads the lower triangle and
        // the standard form clears the strict upper one first): not loaded, not written
        const bool s_rows = r >= cb;
        double *hc = Hc + (long long)cb * n + r, *sc = Sc + (long long)cb * n + r;
        for (int q0 = 0; q0 < db; q0 += 4) {
          double hv[4], sv[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int q = min(q0 + u, db - 1);
            hv[u] = bo >= 0 ? hb[src + (long long)q * da] : 0.0;
            sv[u] = (bo >= 0 && s_rows) ? sb[src + (long long)q * da] : 0.0;
          }
          if (round32) {  // precision form: the cluster Hamiltonian holds FP32 values (S stays FP64)
#pragma unroll
            for (int u = 0; u < 4; ++u) hv[u] = (double)(float)hv[u];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (q0 + u < db) {
              const int c = cb + q0 + u;
              hc[(long long)(q0 + u) * n] = r > c ? hv[u] : (r == c ? 0.5 * hv[u] : 0.0);
              if (s_rows) sc[(long long)(q0 + u) * n] = sv[u];
            }
        }
      }
    }
  }
  queue_leave(queue);
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
    // lane c keeps column c in registers; the rows of L11 are read by every lane in step
    // (broadcast), and x(t) = 0 for t < c makes the full sums equal to the sums from t = c
    const int c = tid;
    double x[NB];
#pragma unroll
    for (int r = 0; r < NB; ++r) {
      double acc = (r == c) ? 1.0 : 0.0;
#pragma unroll
      for (int t = 0; t < r; ++t) acc -= L11[r][t] * x[t];
      const bool on = c < jb && r < jb && r >= c;
      const double q = acc / L11[r][r];
      x[r] = on ? q : 0.0;
    }
#pragma unroll
    for (int r = 0; r < NB; ++r) Li[r][c] = x[r];
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------------------
// Blocked right-looking Cholesky S^(i) = L L^T (lower; parts of the strictly-upper triangle
// of the diagonal blocks are overwritten -- the standard-form step clears it).  Per panel:
// unblocked factor of the diagonal block, its inverse, the panel below as
// L21 = A21 L11^{-T}; panels go in pairs: the first updates only the second's columns, the
// second updates the rest of the trailing matrix with both (A22 -= L21 L21^T with K = 2 NB on
// MFMA), so the trailing matrix is streamed once per pair.
// A non-positive pivot reports LDC_ERR_NOT_SPD for the cluster.
__global__ void __launch_bounds__(256, 2) potrf_kernel(int n_clusters, const int *__restrict__ order,
                                                       double *__restrict__ mat, const long long *__restrict__ mat_off,
                                                       const int *__restrict__ dmax, const int *__restrict__ dim,
                                                       DevStatus *st, int *__restrict__ queue) {
  __shared__ double L11[NB][NB + 1];
  __shared__ double Li[NB][NB + 1];
  __shared__ double gl[kGemmLds];
  __shared__ int bad;
  const int tid = threadIdx.x;
  for (int s = queue_next(queue); s < n_clusters; s = queue_next(queue)) {
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
      // unblocked factor of the diagonal block by wave 0 alone: lane r keeps row r in
      // registers, the pivot comes by a lane read and column q through LDS (no workgroup
      // barriers inside the block)
      if (tid < 64) {
        const int r = tid;
        double row[NB];
#pragma unroll
        for (int t = 0; t < NB; ++t) row[t] = (r < jb) ? L11[min(r, NB - 1)][t] : 0.0;
        int badl = 0;
#pragma unroll
        for (int q = 0; q < NB; ++q) {
          if (q < jb) {
            const double pv = lane_value(row[q], q);
            const bool ok = pv > 0.0;
            badl |= ok ? 0 : 1;
            const double sp = sqrt(ok ? pv : 1.0);
            row[q] = (r == q) ? sp : ((r > q) ? row[q] / sp : row[q]);
            if (r < NB) Li[r][0] = row[q];  // column q of L, staged for the update
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int t = q + 1; t < NB; ++t) {
              const double ltq = Li[t][0];
              if (r >= t) row[t] -= row[q] * ltq;
            }
            __builtin_amdgcn_wave_barrier();
          }
        }
        if (r < jb) {
#pragma unroll
          for (int t = 0; t < NB; ++t) L11[r][t] = (t <= r) ? row[t] : 0.0;
        }
        if (r == 0 && badl) bad = 1;
      }
      __syncthreads();
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
        double *C = S + (long long)(j0 + jb) * ld + j0 + jb;
        if (((j0 / NB) & 1) == 0) {
          // first panel of a pair: update only the next panel's columns now; the rest of the
          // trailing matrix takes both panels at once (K = 2 NB) after the next panel
          wg_gemm<G_TRANS_B>(C, ld, P, ld, P, ld, m, min(NB, m), jb, gl);
        } else {
          // second panel: A22 -= [L21 of both panels] [L21 of both panels]^T (the first
          // panel's L21 rows below this panel sit in the NB columns to the left)
          const double *P2 = S + (long long)(j0 - NB) * ld + j0 + jb;
          wg_gemm<G_TRANS_B | G_LOWER | G_EARLY_C>(C, ld, P2, ld, P2, ld, m, m, NB + jb, gl);
        }
      }
    }
    __syncthreads();
    if (bad && tid == 0) report(st, LDC_ERR_NOT_SPD, c);
  }
  queue_leave(queue);
}

// Standard form (Sec. II.C (iii) via Cholesky): with S = L L^T and H = H_L + H_L^T (H_L the lower
// triangle with half the diagonal, as the gather stores it),
//   A = L^{-1} H L^{-T} = P L^{-T} + L^{-1} P^T,  P = L^{-1} H_L,
// with P lower triangular (a product of two lower triangles), so both steps run only over
// their nonzero K ranges: n^3 / 3 + 2 n^3 / 3 flops instead of n^3 + 2 n^3 / 3 with a full
// L^{-1} H.
// 1. L^{-1} in place of L (block columns of 2 NB from the last: B21 <- -L22^{-1} L21 L11^{-1},
//    L11 <- L11^{-1}); the strictly-upper part of the S slot is cleared first.
// 2. P = L^{-1} H_L in place of H_L, block rows from the last (a block row needs rows of H_L
//    above it and its own, still intact), each tile's K range from its first column (H_L is
//    lower) to the end of its block row (L^{-1} is lower).
// 3. A = P L^{-T} + L^{-1} P^T (lower part) in place of P, block rows from the last and tiles
//    right to left: tile (I, J) reads P of block row I only in columns up to its own, and
//    rows of P above block row I; both products run over K up to the tile's last column.
// All products are MFMA GEMMs.  The tracked
// columns of the tridiagonal solver are set up here: X_u = L^{-1} E_i (the last M columns of
// L^{-1}) and X_v = L^T E_i (the last M rows of L, taken before the inversion).
// TP: compute type of the two products (double, or float in the precision form: FP32 matrix
// cores with FP32 accumulation; the inverse of L stays FP64).
template <typename TP>
__global__ void __launch_bounds__(256, 2) sygst_kernel(int n_clusters, const int *__restrict__ order,
                                                    double *__restrict__ mat, const long long *__restrict__ mat_off,
                                                    double *__restrict__ vec, const long long *__restrict__ vec_off,
                                                    const int *__restrict__ dmax, const int *__restrict__ dim,
                                                    const int *__restrict__ n_orb, int *__restrict__ queue) {
  // GEMM staging; the four NB x NB blocks of the inversion share it (they are dead whenever
  // a product runs)
  constexpr int kInvLds = 4 * NB * (NB + 1);
  __shared__ double gl[kGemmLdsWide > kInvLds ? kGemmLdsWide : kInvLds];
  double(*L11)[NB + 1] = reinterpret_cast<double(*)[NB + 1]>(gl);
  double(*Li)[NB + 1] = L11 + NB;
  double(*Pi)[NB + 1] = Li + NB;
  double(*Bq)[NB + 1] = Pi + NB;
  const int tid = threadIdx.x, nthr = blockDim.x;
  for (int s = queue_next(queue); s < n_clusters; s = queue_next(queue)) {
    const int c = order[s];
    const int n = dim[c], ld = n;
    const int M = n_orb[c];
    double *H = mat + mat_off[c];
    double *L = H + (long long)dmax[c] * dmax[c];
    const VecLayout vl = VecLayout::make(dmax[c]);
    double *cv = vec + vec_off[c];
    double *X = cv + vl.G0;
    double *tmp = cv + vl.G1;  // n x 2 NB scratch of the inversion (the tracked-column partner and the T-factor area)
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
    // 1. L <- L^{-1}, block columns of 2 NB from the last.  The inverse of a diagonal block
    //    [P 0; B Q] (P, Q of NB) is [P^{-1} 0; -Q^{-1} B P^{-1} Q^{-1}], from the two NB x NB
    //    inverses; then L21 <- -L22^{-1} L21 L11^{-1} with two MFMA products of full 64-wide tiles.
    constexpr int BW = 2 * NB;
    const int nblk = (n + BW - 1) / BW;
    for (int bj = nblk - 1; bj >= 0; --bj) {
      const int j = bj * BW, jbt = min(BW, n - j);
      const int ja = min(NB, jbt), jc = jbt - ja;
      __syncthreads();
      for (int e = tid; e < NB * NB; e += nthr) {
        const int r = e % NB, q = e / NB;
        L11[r][q] = (r < ja && q < ja && r >= q) ? L[(long long)(j + q) * ld + j + r] : 0.0;
      }
      __syncthreads();
      lds_tri_inverse(L11, Li, ja);
      for (int e = tid; e < NB * NB; e += nthr) Pi[e % NB][e / NB] = Li[e % NB][e / NB];
      __syncthreads();
      if (jc > 0) {
        for (int e = tid; e < NB * NB; e += nthr) {
          const int r = e % NB, q = e / NB;
          L11[r][q] = (r < jc && q < jc && r >= q) ? L[(long long)(j + NB + q) * ld + j + NB + r] : 0.0;
          Bq[r][q] = (r < jc && q < ja) ? L[(long long)(j + q) * ld + j + NB + r] : 0.0;
        }
        __syncthreads();
        lds_tri_inverse(L11, Li, jc);  // Li = Q^{-1}
        // L11 <- B P^{-1}, then Bq <- -Q^{-1} (B P^{-1})
        for (int e = tid; e < NB * NB; e += nthr) {
          const int r = e % NB, q = e / NB;
          double acc = 0.0;
          for (int t = q; t < NB; ++t) acc += Bq[r][t] * Pi[t][q];
          L11[r][q] = acc;
        }
        __syncthreads();
        for (int e = tid; e < NB * NB; e += nthr) {
          const int r = e % NB, q = e / NB;
          double acc = 0.0;
          for (int t = 0; t <= r; ++t) acc += Li[r][t] * L11[t][q];
          Bq[r][q] = -acc;
        }
        __syncthreads();
      }
      // the inverse of the diagonal block into place (lower part)
      for (int e = tid; e < NB * NB; e += nthr) {
        const int r = e % NB, q = e / NB;
        if (r < ja && q < ja && r >= q) L[(long long)(j + q) * ld + j + r] = Pi[r][q];
        if (r < jc && q < jc && r >= q) L[(long long)(j + NB + q) * ld + j + NB + r] = Li[r][q];
        if (r < jc && q < ja) L[(long long)(j + q) * ld + j + NB + r] = Bq[r][q];
      }
      __syncthreads();
      const int m = n - j - jbt;
      if (m > 0) {
        double *L21 = L + (long long)j * ld + j + jbt;
        // tmp = -L22^{-1} L21 (L22^{-1} lower triangular: K limited per tile row)
        wg_gemm<G_OVERWRITE>(tmp, n, L + (long long)(j + jbt) * ld + j + jbt, ld, L21, ld, m, jbt, m, gl, 0);
        // L21 <- tmp L11^{-1}
        wg_gemm<G_OVERWRITE | G_PLUS>(L21, ld, tmp, n, L + (long long)j * ld + j, ld, m, jbt, jbt, gl);
      }
    }
    // X_u = L^{-1} E_i: rows b0.. of the last M columns of L^{-1}
    for (int e = tid; e < M * M; e += nthr) {
      const int r = e % M, al = e / M;
      X[(long long)(b0 + r) * kTrack + al] = (r >= al) ? L[(long long)(b0 + al) * ld + b0 + r] : 0.0;
    }
    // 2. P = L^{-1} H_L in place, block rows of GT from the last; a tile of block row b reads
    //    only its own columns of H_L (rows 0..r1, its own rows included) and is written after its
    //    last read.  P is lower triangular (its diagonal tile's upper part comes out zero).
    const int nblk2 = (n + GT - 1) / GT;
    for (int bj = nblk2 - 1; bj >= 0; --bj) {
      const int r0 = bj * GT, jb = min(GT, n - r0), r1 = r0 + jb;
      wg_gemm<G_OVERWRITE | G_PLUS | G_B_LOWER, 64, 128, TP>(H + r0, ld, L + r0, ld, H, ld, jb, r1, r1, gl, r0);
    }
    // 3. A = P L^{-T} + L^{-1} P^T in place, lower part: block row b of A from L^{-1} and P of
    //    rows b and of rows 0:r1, in one pass of both products per tile.
    for (int bj = nblk2 - 1; bj >= 0; --bj) {
      const int r0 = bj * GT, jb = min(GT, n - r0), r1 = r0 + jb;
      wg_gemm<G_TRANS_B | G_OVERWRITE | G_PLUS | G_REV | G_DUAL, 64, 128, TP>(H + r0, ld, L + r0, ld, H, ld, jb, r1,
                                                                               r1, gl, -1, 0, H + r0, L);
    }
  }
  queue_leave(queue);
}

// ---------------------------------------------------------------------------------------
void launch_lno_blocks(Plan &p, const double *d_H, const double *d_S) {
  if (p.opt.prec == LDC_MIXED_FP32)
    hipLaunchKernelGGL(lno_blocks_kernel<float>, dim3(std::min(p.n_atoms, 8 * p.n_cu)), dim3(kWG), 0, p.stream,
                       p.n_atoms, p.d_row_ptr, p.d_col, p.d_n_orb, p.d_blk_off, p.d_rank, p.d_U, d_H, d_S, p.d_lno_blk,
                       p.blk_total);
  else
    hipLaunchKernelGGL(lno_blocks_kernel<double>, dim3(std::min(p.n_atoms, 8 * p.n_cu)), dim3(kWG), 0, p.stream,
                       p.n_atoms, p.d_row_ptr, p.d_col, p.d_n_orb, p.d_blk_off, p.d_rank, p.d_U, d_H, d_S, p.d_lno_blk,
                       p.blk_total);
}

void launch_gather(Plan &p, const double *d_H, const double *d_S) {
  // default four workgroups per CU: the dense pass is bound by memory traffic, not by
  // registers or LDS
  const int n = cur_count(p);
  const int grid = std::max(1, std::min(stage_grid(p, kTGather, 4 * p.n_cu), n));
  hipLaunchKernelGGL(gather_kernel, dim3(grid), dim3(kWG), sizeof(unsigned short) * cur_dim(p), p.stream, n,
                     cur_order(p), p.d_mem_ptr, p.d_mem_atom, p.d_mem_long, p.d_pair_ptr, p.d_pair_ab, p.d_pair_blk,
                     p.d_n_orb, p.d_blk_off, d_H, d_S, p.lno_mode, p.d_rank, p.d_lno_blk, p.blk_total, p.d_mat,
                     p.d_mat_off, p.d_dmax, p.d_dim, p.opt.prec == LDC_MIXED_FP32 ? 1 : 0, p.d_queue);
}

void launch_potrf(Plan &p) {
  const int n = cur_count(p);
  const int grid = std::max(1, std::min(stage_grid(p, kTPotrf, p.workgroups), n));
  hipLaunchKernelGGL(potrf_kernel, dim3(grid), dim3(kWG), 0, p.stream, n, cur_order(p), p.d_mat, p.d_mat_off, p.d_dmax,
                     p.d_dim, p.d_status, p.d_queue);
}

void launch_sygst(Plan &p) {
  const int n = cur_count(p);
  const int grid = std::max(1, std::min(stage_grid(p, kTSygst, p.workgroups), n));
  if (p.opt.prec == LDC_MIXED_FP32)
    hipLaunchKernelGGL(sygst_kernel<float>, dim3(grid), dim3(kWG), 0, p.stream, n, cur_order(p), p.d_mat,
                       p.d_mat_off, p.d_vec, p.d_vec_off, p.d_dmax, p.d_dim, p.d_n_orb, p.d_queue);
  else
    hipLaunchKernelGGL(sygst_kernel<double>, dim3(grid), dim3(kWG), 0, p.stream, n, cur_order(p), p.d_mat,
                       p.d_mat_off, p.d_vec, p.d_vec_off, p.d_dmax, p.d_dim, p.d_n_orb, p.d_queue);
}

}  // namespace ldc
