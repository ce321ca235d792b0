// Workgroup-level FP64 building blocks on matrices in global memory.
// One 256-thread workgroup cooperates on one call; LDS staging tiles are passed in.
#pragma once

#include "dev_common.h"

namespace ldc {

constexpr int GT = 64;    // output tile edge
constexpr int GK = 32;    // K chunk
constexpr int GPAD = 1;   // LDS padding (doubles)

// LDS needed by wg_gemm: 2 * GK * (GT + GPAD) doubles; by the tall 128 x 32 tiles
// (wg_gemm<F, 128, 32>): GK * (128 + 32 + 2 GPAD); by the wide 64 x 128 tiles
// (wg_gemm<F, 64, 128>, K chunks of GK / 2): GK / 2 * (64 + 128 + 2 GPAD).
constexpr int kGemmLds = 2 * GK * (GT + GPAD);
constexpr int kGemmLdsTall = GK * (128 + 32 + 2 * GPAD);
constexpr int kGemmLdsWide = GK / 2 * (64 + 128 + 2 * GPAD);

typedef double ldc_double4 __attribute__((ext_vector_type(4)));
typedef float ldc_float4 __attribute__((ext_vector_type(4)));

// One 16 x 16 x 4 matrix-core product for the compute type of wg_gemm: FP64 (v_mfma_f64_16x16x4)
// or FP32 with FP32 accumulation (v_mfma_f32_16x16x4).  The two lay out their 16 x 16 result
// differently: output register r of lane l holds row l / 16 + 4 r (FP64) or 4 (l / 16) + r (FP32)
// of the instruction's result, column l % 16.
template <typename TC>
struct Mfma;
template <>
struct Mfma<double> {
  typedef ldc_double4 acc_t;
  __device__ static acc_t step(double a, double b, acc_t c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __device__ static int row_of(int r, int lk) { return 4 * r + lk; }
};
template <>
struct Mfma<float> {
  typedef ldc_float4 acc_t;
  __device__ static acc_t step(float a, float b, acc_t c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int row_of(int r, int lk) { return 4 * lk + r; }
};

// Operand layouts and options of wg_gemm (bit flags).
enum : unsigned {
  G_TRANS_B = 1u,     // op(B) = B^T (B: n x k); otherwise op(B) = B (B: k x n)
  G_LOWER = 2u,       // only output tiles touching the lower triangle (tile row >= tile column)
  G_A_RM = 4u,        // A row-major (row stride lda); otherwise column-major (leading dimension lda)
  G_B_RM = 8u,        // B row-major (row stride ldb)
  G_OVERWRITE = 16u,  // C = -A op(B) (C is not read)
  G_LATE_C = 32u,     // read C at the store instead of prefetching it (fewer registers)
  G_C_RM = 64u,       // C row-major (row stride ldc)
  G_A_SYM = 128u,     // A is symmetric, held in the lower triangle of a column-major array
  G_PLUS = 256u,      // add instead of subtract: C += A op(B) (G_OVERWRITE: C = A op(B))
  G_REV = 512u,       // tiles from the last to the first
  G_EARLY_C = 1024u,  // fetch C with the tile's first K chunk (short K: more time to arrive)
  G_B_LOWER = 2048u,  // op(B) is lower triangular (op(B)[kk][c] = 0 for kk < c): a tile's K loop
                      // starts at its first column
  G_DUAL = 4096u,     // two products in one pass: A op(B) + A2 op(B2), A2 and B2 laid out like A
                      // and B; op(B) and op(B2) vanish for kk beyond the tile's last column, so each
                      // product runs over K < (tile's column end)
};

// C[m x n] -= A[m x k] * op(B)   (G_OVERWRITE: C = -A op(B); G_PLUS: + instead of -).
// G_LOWER: the strictly-upper part of diagonal tiles is computed too and must be unused.
// a_diag >= 0: A is zero above its a_diag-th superdiagonal (A[r][kk] = 0 for kk > r + a_diag),
// so each tile row only runs over the K range that can be nonzero.
// G_DUAL: the K loop runs over both products, the second's chunks after the first's.
// 0 < b_rot < k: the K index of op(B) is rotated, op(B)[kk][c] = op(B')[(kk + b_rot) mod k][c];
// with A = [V | W] row-major and B = A this forms V W^T + W V^T in one pass.
// G_A_SYM: A[r][kk] = A_lo[max(r,kk)][min(r,kk)]; a K chunk wholly right of the tile's rows
// is read along rows of the stored lower triangle, the others down its columns (coalesced
// except in the chunks that cross the diagonal).
//
// TM x TN output tiles: 64 x 64, 128 x 32 (outputs 32 columns wide) or 64 x 128 (fewer
// re-reads of A); each of the 4 waves owns a 32 x 32 part (32 x 64 for 64 x 128 tiles) as
// 2 x BN blocks of v_mfma_f64_16x16x4 (FP64 matrix cores).  Operands are swapped so that each output
// register covers 16 consecutive rows of one column (coalesced column-major stores):
// the instruction's A operand takes op(B) (lane l: op(B)[k0 + l/16][c0 + l%16]) and its B
// operand takes A (lane l: A[r0 + l%16][k0 + l/16]); register r of lane l then holds
// C[r0 + l%16][c0 + 4 r + l/16].  The next K chunk of A and op(B) (after a tile's last
// chunk: the next tile's first) is fetched into registers while the current one is multiplied;
// with the last chunk C is fetched too (with the first under G_EARLY_C; not under G_LATE_C).
//
// TC: compute type.  double: FP64 products (the default).  float: the operands are rounded to
// FP32 when staged and multiplied on the FP32 matrix cores with FP32 accumulation; C stays FP64
// in memory (the FP32 product is added to it in FP64).
template <unsigned F, int TM = GT, int TN = GT, typename TC = double>
__device__ void wg_gemm(double *C, int ldc, const double *A, int lda, const double *B, int ldb, int m, int n, int k,
                        double *lds, int a_diag = -1, int b_rot = 0, const double *A2 = nullptr,
                        const double *B2 = nullptr) {
  typedef typename Mfma<TC>::acc_t acc_t;
  constexpr bool TRANS_B = F & G_TRANS_B, LOWER = F & G_LOWER, A_RM = F & G_A_RM, B_RM = F & G_B_RM;
  constexpr bool OVERWRITE = F & G_OVERWRITE, PREFETCH_C = !(F & G_LATE_C), C_RM = F & G_C_RM;
  constexpr bool A_SYM = F & G_A_SYM, PLUS = F & G_PLUS, REV = F & G_REV, EARLY_C = F & G_EARLY_C;
  constexpr bool B_LOWER = F & G_B_LOWER, DUAL = F & G_DUAL;
  static_assert(!(DUAL && (A_SYM || B_LOWER)), "the two-product pass takes plain operands");
  static_assert(!(A_SYM && A_RM), "a symmetric A is stored column-major");
  constexpr int KC = (TN == 128) ? GK / 2 : GK;  // K chunk (halved for the wide tiles: fewer registers)
  // wave grid GR x GC (GR = TM / 32 rows of waves), each wave 32 x (16 BN)
  constexpr int GR = TM / 32, GC = 4 / GR, BN = TN / (16 * GC), WN = 16 * BN;
  static_assert(TM % 32 == 0 && GR * GC == 4 && (BN == 2 || BN == 4) && WN * GC == TN, "tile shape");
  static_assert(!LOWER || TM == TN, "lower-triangle tiling needs square tiles");
  // LDS row padding: one double, or 16 floats for FP32 staging (a 16-wide read of four
  // consecutive K rows then falls into four disjoint quarters of the 64 banks)
  constexpr int PAD = sizeof(TC) == 4 ? 16 : GPAD;
  constexpr int LSA = TM + PAD, LSB = TN + PAD;
  static_assert(sizeof(TC) == 8 || KC * (LSA + LSB) * 4 <= KC * (TM + TN + 2 * GPAD) * 8, "FP32 staging fits");
  constexpr int PERA = TM * KC / 256, PERB = TN * KC / 256;  // staged elements per thread
  TC *As = reinterpret_cast<TC *>(lds);  // [KC][LSA]
  TC *Bs = As + KC * LSA;                 // [KC][LSB]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave / GC, wc = wave % GC;
  const int li = lane & 15, lk = lane >> 4;
  const int mt = (m + TM - 1) / TM, nt = (n + TN - 1) / TN;
  // Staging: element q of this thread's share of a 64 x KC tile sits at (e + q STEP) along
  // the 64 edge and kk along K (K-fast layout), or at e along the edge and (kk + q STEP)
  // along K (edge-fast layout); the faster-running index follows the operand's memory
  // layout (coalesced loads).  Offsets are 32-bit (a cluster matrix has far fewer than 2^31
  // elements).
  constexpr bool B_KFAST = !((TRANS_B && !B_RM) || (!TRANS_B && B_RM));
  const int ef = tid % TM, kf = tid / TM;      // edge-fast position (A)
  const int efb = tid % TN, kfb = tid / TN;    // edge-fast position (B)
  const int ek = tid / KC, kk0 = tid % KC;     // K-fast position
  constexpr int STEP_E = 256 / TM, STEP_EB = 256 / TN, STEP_K = 256 / KC;
  const int b_e = B_KFAST ? ek : efb, b_k = B_KFAST ? kk0 : kfb;
  constexpr int B_STEP = B_KFAST ? STEP_K : STEP_EB;
  const int a_rs = A_RM ? lda : 1, a_ks = A_RM ? 1 : lda;
  const int b_cs = (TRANS_B != B_RM) ? 1 : ldb, b_ks = (TRANS_B != B_RM) ? ldb : 1;
  // layout of an A chunk: 1 = K-fast, 0 = edge-fast
  auto a_mode_of = [&](int r0, int k0) -> int {
    if (A_SYM) return (k0 >= r0 + TM) ? 1 : 0;
    return A_RM ? 1 : 0;
  };
  // Fetched chunks stay in FP64 registers (the loads are in flight while the previous chunk is
  // multiplied); they are rounded to the compute type only when staged in LDS.
  auto fetchA = [&](const double *Ap, int r0, int k0, int mode, double *ra) {
    const double *Asrc = DUAL ? Ap : A;
#pragma unroll
    for (int q = 0; q < PERA; ++q) {
      int gr, gk;
      if (mode) {
        gr = r0 + ek + q * STEP_K;
        gk = k0 + kk0;
      } else {
        gr = r0 + ef;
        gk = k0 + kf + q * STEP_E;
      }
      double val = 0.0;
      if (gr < m && gk < k) {
        if (A_SYM) {
          const int hi = gr > gk ? gr : gk, lo = gr > gk ? gk : gr;
          val = Asrc[lo * lda + hi];
        } else {
          val = Asrc[gr * a_rs + gk * a_ks];
        }
      }
      ra[q] = val;
    }
  };
  auto fetchB = [&](const double *Bp, int c0, int k0, double *rb) {
    const double *Bsrc = DUAL ? Bp : B;
#pragma unroll
    for (int q = 0; q < PERB; ++q) {
      const int gc = c0 + b_e + (B_KFAST ? q * B_STEP : 0);
      int gk = k0 + b_k + (B_KFAST ? 0 : q * B_STEP);
      const bool in = gc < n && gk < k;
      if (b_rot > 0) {
        gk += b_rot;
        if (gk >= k) gk -= k;
      }
      rb[q] = in ? Bsrc[gc * b_cs + gk * b_ks] : 0.0;
    }
  };
  auto stage = [&](int mode, const double *ra, const double *rb) {
    if (mode) {
#pragma unroll
      for (int q = 0; q < PERA; ++q) As[kk0 * LSA + ek + q * STEP_K] = (TC)ra[q];
    } else {
#pragma unroll
      for (int q = 0; q < PERA; ++q) As[(kf + q * STEP_E) * LSA + ef] = (TC)ra[q];
    }
#pragma unroll
    for (int q = 0; q < PERB; ++q)
      Bs[(b_k + (B_KFAST ? 0 : q * B_STEP)) * LSB + b_e + (B_KFAST ? q * B_STEP : 0)] = (TC)rb[q];
  };
  auto cidx = [&](int gr, int gc) { return C_RM ? gr * ldc + gc : gc * ldc + gr; };
  // tiles in row-major order (G_REV: reversed; G_LOWER: only tile row >= tile column); a
  // tile sequence index i maps to the tile index tile_of(i)
  auto tile_of = [&](int i) { return REV ? mt * nt - 1 - i : i; };
  auto next_tile = [&](int i) -> int {
    for (; i < mt * nt; ++i) {
      const int t = tile_of(i);
      if (!LOWER || t % nt <= t / nt) return i;
    }
    return -1;
  };
  auto k_end = [&](int r0) { return (a_diag >= 0) ? min(k, r0 + TM + a_diag) : k; };
  // a tile's K loop: [k_beg, k_stop); under G_DUAL the first product takes [0, k_half) and the
  // second [k_half, 2 k_half) (k_half a whole number of chunks)
  auto k_half = [&](int c0) { return ((min(k, c0 + TN) + KC - 1) / KC) * KC; };
  auto k_beg = [&](int c0) { return B_LOWER ? c0 : 0; };
  auto k_stop = [&](int r0, int c0) { return DUAL ? 2 * k_half(c0) : k_end(r0); };
  // operands and local K index of the chunk starting at k0 of the tile with column start c0
  auto chunk_src = [&](int c0, int k0, const double *&pa, const double *&pb) -> int {
    if (DUAL) {
      const int kh = k_half(c0);
      if (k0 >= kh) {
        pa = A2;
        pb = B2;
        return k0 - kh;
      }
    }
    pa = A;
    pb = B;
    return k0;
  };

  // Software pipeline over (tile, K chunk): the chunk after the one being multiplied is always
  // in flight, including the first chunk of the next tile while the last chunk of this one runs.
  double ra[PERA], rb[PERB];
  int tile = next_tile(0);
  int amode = 0;
  const double *pa = A, *pb = B;
  if (tile >= 0) {
    const int r0 = (tile_of(tile) / nt) * TM, c0 = (tile_of(tile) % nt) * TN;
    if (k_stop(r0, c0) > k_beg(c0)) {
      const int kk = chunk_src(c0, k_beg(c0), pa, pb);
      amode = a_mode_of(r0, kk);
      fetchA(pa, r0, kk, amode, ra);
      fetchB(pb, c0, kk, rb);
    }
  }
  while (tile >= 0) {
    const int ti = tile_of(tile) / nt, tj = tile_of(tile) % nt;
    const int r0 = ti * TM, c0 = tj * TN;
    const int kbeg = k_beg(c0), kend = k_stop(r0, c0);
    const int nxt = next_tile(tile + 1);
    const int r0n = (nxt >= 0) ? (tile_of(nxt) / nt) * TM : 0, c0n = (nxt >= 0) ? (tile_of(nxt) % nt) * TN : 0;
    const bool fetch_next = nxt >= 0 && k_stop(r0n, c0n) > k_beg(c0n);
    acc_t acc[2][BN];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < BN; ++b) acc[a][b] = acc_t{0, 0, 0, 0};
    double cold[2][BN][4];
    for (int k0 = kbeg; k0 < kend; k0 += KC) {
      __syncthreads();
      stage(amode, ra, rb);
      __syncthreads();
      if (k0 + KC < kend) {
        const int kk = chunk_src(c0, k0 + KC, pa, pb);
        amode = a_mode_of(r0, kk);
        fetchA(pa, r0, kk, amode, ra);
        fetchB(pb, c0, kk, rb);
      } else {
        if (fetch_next) {
          const int kk = chunk_src(c0n, k_beg(c0n), pa, pb);
          amode = a_mode_of(r0n, kk);
          fetchA(pa, r0n, kk, amode, ra);
          fetchB(pb, c0n, kk, rb);
        }
      }
      if (!OVERWRITE && PREFETCH_C && (EARLY_C ? k0 == kbeg : k0 + KC >= kend)) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < BN; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int gr = r0 + wr * 32 + a * 16 + li, gc = c0 + wc * WN + b * 16 + Mfma<TC>::row_of(r, lk);
              cold[a][b][r] = (gr < m && gc < n) ? C[cidx(gr, gc)] : 0.0;
            }
      }
#pragma unroll
      for (int s4 = 0; s4 < KC / 4; ++s4) {
        const int kra = (4 * s4 + lk) * LSA, krb = (4 * s4 + lk) * LSB;
        TC af[2], bf[BN];
#pragma unroll
        for (int a = 0; a < 2; ++a) af[a] = As[kra + wr * 32 + a * 16 + li];
#pragma unroll
        for (int b = 0; b < BN; ++b) bf[b] = Bs[krb + wc * WN + b * 16 + li];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < BN; ++b) acc[a][b] = Mfma<TC>::step(bf[b], af[a], acc[a][b]);
      }
    }
    if (kend <= kbeg && fetch_next) {
      const int kk = chunk_src(c0n, k_beg(c0n), pa, pb);
      amode = a_mode_of(r0n, kk);
      fetchA(pa, r0n, kk, amode, ra);
      fetchB(pb, c0n, kk, rb);
    }
    tile = nxt;
    if (kend <= kbeg && !OVERWRITE) continue;  // nothing to subtract
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const int gr = r0 + wr * 32 + a * 16 + li;
#pragma unroll
      for (int b = 0; b < BN; ++b) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int gc = c0 + wc * WN + b * 16 + Mfma<TC>::row_of(r, lk);
          if (gr < m && gc < n) {
            const double v = PLUS ? (double)acc[a][b][r] : -(double)acc[a][b][r];
            if (OVERWRITE) C[cidx(gr, gc)] = v;
            else if (PREFETCH_C) C[cidx(gr, gc)] = cold[a][b][r] + v;
            else C[cidx(gr, gc)] += v;
          }
        }
      }
    }
  }
  __syncthreads();
}

// C = -(A^T B) for a tall A (m x 32) and B (m x N, N <= 32), both row-major (row strides lda,
// ldb >= 32 resp. N), m >= 1; C is 32 x N, column-major (ldc) or row-major (C_RM).  The K
// range (the m rows) is split over the four waves in steps of 4 rows; each wave accumulates
// a full 32 x 32 partial product on the matrix cores (loads of 8 steps in flight) and the
// partial sums meet in LDS (4 x 32 x 33 doubles of lds).
constexpr int kAtbLds = 4 * 32 * 33;
template <bool C_RM>
__device__ void wg_atb32(double *C, int ldc, const double *A, int lda, const double *B, int ldb, int m, int N,
                         double *lds) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  constexpr int U = 8;
  ldc_double4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = ldc_double4{0.0, 0.0, 0.0, 0.0};
  const int nsteps = (m + 3) / 4;
  for (int s0 = wave; s0 < nsteps; s0 += 4 * U) {
    double av[U][2], bv[U][2];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int row = (s0 + 4 * u) * 4 + lk;
      const int rr = row < m ? row : m - 1;  // clamped: every load is in bounds
#pragma unroll
      for (int a = 0; a < 2; ++a) av[u][a] = A[rr * lda + a * 16 + li];
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int col = b * 16 + li;
        bv[u][b] = B[rr * ldb + (col < N ? col : N - 1)];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int row = (s0 + 4 * u) * 4 + lk;
#pragma unroll
      for (int a = 0; a < 2; ++a) av[u][a] = row < m ? av[u][a] : 0.0;
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(bv[u][b], av[u][a], acc[a][b], 0, 0, 0);
    }
  }
  // register r of block (a, b) holds the partial C[a 16 + li][b 16 + 4 r + lk]
  double *P = lds + wave * 32 * 33;
  __syncthreads();
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) P[(a * 16 + li) * 33 + b * 16 + 4 * r + lk] = acc[a][b][r];
  __syncthreads();
  for (int e = tid; e < 32 * N; e += blockDim.x) {
    const int i = C_RM ? e / N : e % 32, j = C_RM ? e % N : e / 32;
    const int o = i * 33 + j;
    const double v = (lds[o] + lds[32 * 33 + o]) + (lds[2 * 32 * 33 + o] + lds[3 * 32 * 33 + o]);
    C[C_RM ? i * ldc + j : j * ldc + i] = -v;
  }
  __syncthreads();
}

}  // namespace ldc
