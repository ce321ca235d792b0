// Workgroup-level FP64 building blocks on matrices in global memory.
// One 256-thread workgroup cooperates on one call; LDS staging tiles are passed in.
#pragma once

#include "dev_common.h"

namespace ldc {

constexpr int GT = 64;    // output tile edge
constexpr int GK = 32;    // K chunk
constexpr int GPAD = 1;   // LDS padding (doubles)

// LDS needed by wg_gemm_sub: 2 * GK * (GT + GPAD) doubles.
constexpr int kGemmLds = 2 * GK * (GT + GPAD);

typedef double ldc_double4 __attribute__((ext_vector_type(4)));

// C[m x n] -= A[m x k] * op(B), op(B) = B^T (B: n x k) if TRANS_B else B (B: k x n).
// LOWER: only output tiles that touch the lower triangle (tile row >= tile column) are
// computed (the strictly-upper part of diagonal tiles is computed too and must be unused).
// A_RM / B_RM: A (resp. B) stored row-major with row stride lda (ldb) instead of
// column-major with leading dimension lda (ldb).  OVERWRITE: C = -A op(B) (C is not read).
// a_diag >= 0: A is zero above its a_diag-th superdiagonal (A[r][kk] = 0 for kk > r + a_diag),
// so each tile row only runs over the K range that can be nonzero.
// 0 < b_rot < k: the K index of op(B) is rotated, op(B)[kk][c] = op(B')[(kk + b_rot) mod k][c];
// with A = [V | W] row-major and B = A this forms V W^T + W V^T in one pass.
//
// 64 x 64 output tiles; each of the 4 waves owns a 32 x 32 quarter as 2 x 2 blocks of
// v_mfma_f64_16x16x4 (FP64 matrix cores).  Operands are swapped so that each output
// register covers 16 consecutive rows of one column (coalesced column-major stores):
// the instruction's A operand takes op(B) (lane l: op(B)[k0 + l/16][c0 + l%16]) and its B
// operand takes A (lane l: A[r0 + l%16][k0 + l/16]); register r of lane l then holds
// C[r0 + l%16][c0 + 4 r + l/16].  The next K chunk of A and op(B) is fetched into registers
// while the current one is multiplied; after the last chunk the same registers fetch C.
template <bool TRANS_B, bool LOWER, bool A_RM = false, bool B_RM = false, bool OVERWRITE = false>
__device__ void wg_gemm_sub(double *C, int ldc, const double *A, int lda, const double *B, int ldb, int m, int n,
                            int k, double *lds, int a_diag = -1, int b_rot = 0) {
  constexpr int LS = GT + GPAD;
  constexpr int PER = GT * GK / 256;  // staged elements per thread and operand (8)
  double *As = lds;                   // [GK][LS]
  double *Bs = lds + GK * LS;         // [GK][LS]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int li = lane & 15, lk = lane >> 4;
  const int mt = (m + GT - 1) / GT, nt = (n + GT - 1) / GT;
  // Staging: element q of this thread's share of a 64 x GK tile sits at (e0 + q STEP) along
  // the 64 edge and ek along K, or at e0 along the edge and (ek + q STEP) along K; the
  // faster-running index follows the operand's memory layout (coalesced loads).  Offsets
  // are 32-bit (a cluster matrix has far fewer than 2^31 elements).
  constexpr bool A_KFAST = A_RM;
  constexpr bool B_KFAST = !((TRANS_B && !B_RM) || (!TRANS_B && B_RM));
  const int a_e = A_KFAST ? tid / GK : tid % GT, a_k = A_KFAST ? tid % GK : tid / GT;
  const int b_e = B_KFAST ? tid / GK : tid % GT, b_k = B_KFAST ? tid % GK : tid / GT;
  constexpr int A_STEP = A_KFAST ? 256 / GK : 256 / GT;
  constexpr int B_STEP = B_KFAST ? 256 / GK : 256 / GT;
  // element (row, kk) of A and (col, kk) of op(B) in memory
  const int a_rs = A_RM ? lda : 1, a_ks = A_RM ? 1 : lda;
  const int b_cs = (TRANS_B != B_RM) ? 1 : ldb, b_ks = (TRANS_B != B_RM) ? ldb : 1;
  auto fetch = [&](int r0, int c0, int k0, double *ra, double *rb) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int gr = r0 + a_e + (A_KFAST ? q * A_STEP : 0), gk = k0 + a_k + (A_KFAST ? 0 : q * A_STEP);
      ra[q] = (gr < m && gk < k) ? A[gr * a_rs + gk * a_ks] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int gc = c0 + b_e + (B_KFAST ? q * B_STEP : 0);
      int gk = k0 + b_k + (B_KFAST ? 0 : q * B_STEP);
      const bool in = gc < n && gk < k;
      if (b_rot > 0) {
        gk += b_rot;
        if (gk >= k) gk -= k;
      }
      rb[q] = in ? B[gc * b_cs + gk * b_ks] : 0.0;
    }
  };
  auto stage = [&](const double *ra, const double *rb) {
#pragma unroll
    for (int q = 0; q < PER; ++q)
      As[(a_k + (A_KFAST ? 0 : q * A_STEP)) * LS + a_e + (A_KFAST ? q * A_STEP : 0)] = ra[q];
#pragma unroll
    for (int q = 0; q < PER; ++q)
      Bs[(b_k + (B_KFAST ? 0 : q * B_STEP)) * LS + b_e + (B_KFAST ? q * B_STEP : 0)] = rb[q];
  };

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
    double ra[PER], rb[PER];
    if (kend > 0) fetch(r0, c0, 0, ra, rb);
    double cold[2][2][4];
    for (int k0 = 0; k0 < kend; k0 += GK) {
      __syncthreads();
      stage(ra, rb);
      __syncthreads();
      if (k0 + GK < kend) {
        fetch(r0, c0, k0 + GK, ra, rb);
      } else if (!OVERWRITE) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int gr = r0 + wr * 32 + a * 16 + li, gc = c0 + wc * 32 + b * 16 + 4 * r + lk;
              cold[a][b][r] = (gr < m && gc < n) ? C[gc * ldc + gr] : 0.0;
            }
      }
#pragma unroll
      for (int s4 = 0; s4 < GK / 4; ++s4) {
        const int kr = (4 * s4 + lk) * LS;
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
    if (kend <= 0 && !OVERWRITE) continue;  // nothing to subtract
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const int gr = r0 + wr * 32 + a * 16 + li;
#pragma unroll
      for (int b = 0; b < 2; ++b) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int gc = c0 + wc * 32 + b * 16 + 4 * r + lk;
          if (gr < m && gc < n) {
            if (OVERWRITE) C[gc * ldc + gr] = -acc[a][b][r];
            else C[gc * ldc + gr] = cold[a][b][r] - acc[a][b][r];
          }
        }
      }
    }
  }
  __syncthreads();
}

}  // namespace ldc
