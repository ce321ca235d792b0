// Workgroup-level FP64 building blocks on column-major matrices in global memory.
// One 256-thread workgroup cooperates on one call; LDS staging tiles are passed in.
#pragma once

#include "dev_common.h"

namespace ldc {

constexpr int GT = 64;    // output tile edge
constexpr int GK = 16;    // K chunk
constexpr int GPAD = 1;   // LDS padding (doubles)

// LDS needed by wg_gemm_sub: 2 * GK * (GT + GPAD) doubles.
constexpr int kGemmLds = 2 * GK * (GT + GPAD);

// C[m x n] -= A[m x k] * op(B), op(B) = B^T (B: n x k) if TRANS_B else B (B: k x n).
// LOWER: only output tiles that touch the lower triangle (tile row >= tile column) are
// computed (the strictly-upper part of diagonal tiles is computed too and must be unused).
template <bool TRANS_B, bool LOWER>
__device__ void wg_gemm_sub(double *C, int ldc, const double *A, int lda, const double *B, int ldb, int m, int n,
                            int k, double *lds) {
  double *As = lds;                  // [GK][GT+GPAD]
  double *Bs = lds + GK * (GT + GPAD);
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  const int mt = (m + GT - 1) / GT, nt = (n + GT - 1) / GT;
  for (int tile = 0; tile < mt * nt; ++tile) {
    const int ti = tile / nt, tj = tile % nt;
    if (LOWER && tj > ti) continue;
    const int r0 = ti * GT, c0 = tj * GT;
    double acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
    for (int k0 = 0; k0 < k; k0 += GK) {
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e = tid + 256 * q;
        const int row = e & 63, kk = e >> 6;
        const int gr = r0 + row, gk = k0 + kk;
        As[kk * (GT + GPAD) + row] = (gr < m && gk < k) ? A[(long long)gk * lda + gr] : 0.0;
      }
      if (TRANS_B) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int e = tid + 256 * q;
          const int col = e & 63, kk = e >> 6;
          const int gc = c0 + col, gk = k0 + kk;
          Bs[kk * (GT + GPAD) + col] = (gc < n && gk < k) ? B[(long long)gk * ldb + gc] : 0.0;
        }
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int e = tid + 256 * q;
          const int kk = e & 15, col = e >> 4;
          const int gc = c0 + col, gk = k0 + kk;
          Bs[kk * (GT + GPAD) + col] = (gc < n && gk < k) ? B[(long long)gc * ldb + gk] : 0.0;
        }
      }
      __syncthreads();
#pragma unroll 4
      for (int kk = 0; kk < GK; ++kk) {
        double av[4], bv[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) av[a] = As[kk * (GT + GPAD) + tx + 16 * a];
#pragma unroll
        for (int b = 0; b < 4; ++b) bv[b] = Bs[kk * (GT + GPAD) + ty + 16 * b];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[a][b] = fma(av[a], bv[b], acc[a][b]);
      }
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int gc = c0 + ty + 16 * b;
      if (gc >= n) continue;
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int gr = r0 + tx + 16 * a;
        if (gr < m) C[(long long)gc * ldc + gr] -= acc[a][b];
      }
    }
  }
  __syncthreads();
}

}  // namespace ldc
