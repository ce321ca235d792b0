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

typedef double ldc_double4 __attribute__((ext_vector_type(4)));

// C[m x n] -= A[m x k] * op(B), op(B) = B^T (B: n x k) if TRANS_B else B (B: k x n).
// LOWER: only output tiles that touch the lower triangle (tile row >= tile column) are
// computed (the strictly-upper part of diagonal tiles is computed too and must be unused).
// 64 x 64 output tiles; each of the 4 waves owns a 32 x 32 quarter as 2 x 2 blocks of
// v_mfma_f64_16x16x4 (FP64 matrix cores).  Operands are swapped so that each output
// register covers 16 consecutive rows of one column (coalesced column-major stores):
// the instruction's A operand takes op(B) (lane l: op(B)[k0 + l/16][c0 + l%16]) and its B
// operand takes A (lane l: A[r0 + l%16][k0 + l/16]); register r of lane l then holds
// C[r0 + l%16][c0 + 4 r + l/16].
// A_RM / B_RM: A (resp. B) stored row-major with row stride lda (ldb) instead of
// column-major with leading dimension lda (ldb).  OVERWRITE: C = -A op(B) (C is not read).
// a_diag >= 0: A is zero above its a_diag-th superdiagonal (A[r][kk] = 0 for kk > r + a_diag),
// so each tile row only runs over the K range that can be nonzero.
template <bool TRANS_B, bool LOWER, bool A_RM = false, bool B_RM = false, bool OVERWRITE = false>
__device__ void wg_gemm_sub(double *C, int ldc, const double *A, int lda, const double *B, int ldb, int m, int n,
                            int k, double *lds, int a_diag = -1) {
  double *As = lds;                  // [GK][GT+GPAD]
  double *Bs = lds + GK * (GT + GPAD);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int li = lane & 15, lk = lane >> 4;
  const int mt = (m + GT - 1) / GT, nt = (n + GT - 1) / GT;
  for (int tile = 0; tile < mt * nt; ++tile) {
    const int ti = tile / nt, tj = tile % nt;
    if (LOWER && tj > ti) continue;
    const int r0 = ti * GT, c0 = tj * GT;
    ldc_double4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) acc[a][b] = ldc_double4{0.0, 0.0, 0.0, 0.0};
    const int kend = (a_diag >= 0) ? min(k, r0 + GT + a_diag) : k;
    for (int k0 = 0; k0 < kend; k0 += GK) {
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int e = tid + 256 * q;
        const int row = e & 63, kk = e >> 6;
        const int gr = r0 + row, gk = k0 + kk;
        As[kk * (GT + GPAD) + row] =
            (gr < m && gk < k) ? (A_RM ? A[(long long)gr * lda + gk] : A[(long long)gk * lda + gr]) : 0.0;
      }
      if (TRANS_B) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int e = tid + 256 * q;
          const int col = e & 63, kk = e >> 6;
          const int gc = c0 + col, gk = k0 + kk;
          Bs[kk * (GT + GPAD) + col] =
              (gc < n && gk < k) ? (B_RM ? B[(long long)gc * ldb + gk] : B[(long long)gk * ldb + gc]) : 0.0;
        }
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int e = tid + 256 * q;
          const int kk = e & 15, col = e >> 4;
          const int gc = c0 + col, gk = k0 + kk;
          Bs[kk * (GT + GPAD) + col] =
              (gc < n && gk < k) ? (B_RM ? B[(long long)gk * ldb + gc] : B[(long long)gc * ldb + gk]) : 0.0;
        }
      }
      __syncthreads();
#pragma unroll
      for (int s4 = 0; s4 < GK / 4; ++s4) {
        const int kr = (4 * s4 + lk) * (GT + GPAD);
        double af[2], bf[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) af[a] = As[kr + wr * 32 + a * 16 + li];
#pragma unroll
        for (int b = 0; b < 2; ++b) bf[b] = Bs[kr + wc * 32 + b * 16 + li];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(bf[b], af[a], acc[a][b], 0, 0, 0);
      }
    }
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const int gr = r0 + wr * 32 + a * 16 + li;
#pragma unroll
      for (int b = 0; b < 2; ++b) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int gc = c0 + wc * 32 + b * 16 + 4 * r + lk;
          if (gr < m && gc < n) {
            if (OVERWRITE) C[(long long)gc * ldc + gr] = -acc[a][b][r];
            else C[(long long)gc * ldc + gr] -= acc[a][b][r];
          }
        }
      }
    }
  }
  __syncthreads();
}

}  // namespace ldc
