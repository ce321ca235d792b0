// Two-stage Householder tridiagonalization of the standard-form cluster matrix
// A = L^{-1} H^(i) L^{-T} (Sec. II.C (iii)): Q^T A Q = T with Q = Q1 Q2.
//
// Stage 1 (sy2sb_kernel), reduction to band form of width b = kBand.  For every panel of b
// columns j0.. the block P = A(r:n, j0:j0+b), r = j0 + b, is QR-factorised (Householder,
// compact WY: Q_p = I - V T V^T) and the trailing matrix is updated two-sidedly:
//   X = A22 V T (symmetric product),  K = (V T)^T X,  W = X - V K / 2,
//   A22 <- A22 - V W^T - W V^T.
// All four products run on the FP64 matrix cores; only the QR of the tall-skinny panel is
// vector code (leaves of 8 columns factored in LDS).  The reflectors stay below the band
// (reflector k: unit at row k + b, the rest in A(k+b+1:, k)), tau in the tau vector and the
// T factors in the compact-WY area, one b x b block per panel; q2x_kernel applies Q1^T to the
// tracked columns afterwards.
//
// Stage 2 (sb2st_kernel), band to tridiagonal by bulge chasing on a band array holding the
// lower band and the bulge (2b + 1 diagonals).  Sweep s removes column s below its
// subdiagonal: the reflector of rows [r0, r0 + b), r0 = s + 1 + j b, comes from column s
// (j = 0) or from the first column of the bulge that step j - 1 created; step j applies it
// two-sidedly to the diagonal block and from the right to the band block below (which
// creates the next bulge), then forms the next reflector from that block and applies it from
// the left to the rest of the block.  Everything step j reads or writes lies in the columns
// [r0, r0 + b) of the band (column s too for j = 0), so step j of sweep s + 1 (columns
// [r0 + 1, r0 + 1 + b)) only needs steps j and j + 1 of sweep s.  One wavefront runs two sweeps
// (2p, 2p + 1), step j of the second right after step j + 1 of the first, the second sweep's
// window taken from the first's in registers (one window loaded and one stored per two steps);
// pairs of sweeps are pipelined across the wavefronts of the workgroup.  The reflectors are kept
// in the strictly upper triangle of A (sweep s in column n - 1 - s, rows j b..: tau first, then
// v(1:)); q2x_kernel then forms X <- Q2^T Q1^T X for the tracked columns.
#include "wg_blas.h"
#include "wg_qapply.h"

namespace ldc {

constexpr int LEAF = 8;                     // columns per LDS-resident leaf of the panel QR
constexpr int kRowRegs = kMaxDimTri / 64;   // rows of a panel column held per lane
constexpr int kLeafRows = (kMaxDimTri + kWG - 1) / kWG;  // leaf rows held per thread

// ---------------------------------------------------------------------------------------
// QR of the panel P = A(r:n, j0:j0+kBand) (column-major, ld), r = j0 + kBand, m = n - r.
// On return P holds R on and above its diagonal and the Householder vectors below it (unit
// diagonal implicit); tau_k goes to tt[j0 + k] (0 where the reflector has length <= 1).
// lf: LEAF * m doubles of LDS; sm: 2 * LEAF * LEAF + 4 * LEAF doubles; red: 10 * LEAF.
// The reflectors also go to VW (row-major, row stride 2 kBand, rows from r): V explicitly,
// unit diagonal and zeros above it.
// Needs blockDim.x == kWG (four waves).
__device__ void panel_qr(double *__restrict__ A, int ld, int n, int j0, double *__restrict__ tt, double *lf,
                         double *sm, double *red, double *__restrict__ VW) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nthr = blockDim.x, nw = nthr >> 6;
  const int r = j0 + kBand;
  double *Tl = sm;                  // [LEAF][LEAF] leaf T (row-major)
  double *Gl = sm + LEAF * LEAF;    // [LEAF][LEAF] leaf V^T V
  double *tl = Gl + LEAF * LEAF;    // [LEAF] leaf tau
  double *rk = red + 8 * LEAF;      // [2][LEAF] published row k
  for (int c0 = 0; c0 < kBand; c0 += LEAF) {
    const int R0 = r + c0, mp = n - R0;
    if (mp <= 0) {
      if (tid < LEAF) tt[j0 + c0 + tid] = 0.0;
      for (int i = tid; i < n - r; i += nthr)
#pragma unroll
        for (int c = 0; c < LEAF; ++c) VW[(long long)i * 2 * kBand + c0 + c] = 0.0;
      continue;
    }
    // leaf in registers: thread tid holds rows i = tid + kWG t (rows past mp read as zero;
    // the loads are clamped so that they issue back to back).  The barrier orders these reads
    // after the writes of the previous leaf or panel.
    __syncthreads();
    double x[LEAF][kLeafRows];
#pragma unroll
    for (int c = 0; c < LEAF; ++c)
#pragma unroll
      for (int t = 0; t < kLeafRows; ++t) {
        const int i = tid + kWG * t;
        const double v = A[(long long)(j0 + c0 + c) * ld + R0 + (i < mp ? i : mp - 1)];
        x[c][t] = i < mp ? v : 0.0;
      }
    // Column k of the leaf: one pass over the thread's rows applies reflector k - 1 and
    // accumulates the sums for reflector k (|x(k+1:)|^2 and the dots of x(k+1:) with the later
    // leaf columns); thread k publishes row k, so a single barrier per column suffices (red and
    // rk are double-buffered by k).  The loop is unrolled so that every column index is fixed.
    double tau_p = 0.0, beta_p = 0.0, sc_p = 0.0, wc_p[LEAF];
#pragma unroll
    for (int c = 0; c < LEAF; ++c) wc_p[c] = 0.0;
#pragma unroll
    for (int k = 0; k <= LEAF; ++k) {
      if (k >= 1) {
        const int kp = k - 1;
#pragma unroll
        for (int t = 0; t < kLeafRows; ++t) {
          const int i = tid + kWG * t;
          if (i >= kp) {  // rows above kp hold R
            const double v = (i == kp) ? 1.0 : x[kp][t] * sc_p;
#pragma unroll
            for (int c = kp + 1; c < LEAF; ++c) x[c][t] -= tau_p * v * wc_p[c - kp];
            x[kp][t] = (i == kp) ? beta_p : v;
          }
        }
      }
      if (k == LEAF) break;
      double *rkk = rk + (k & 1) * LEAF, *redk = red + (k & 1) * 4 * LEAF;
      if (tid == k && k < mp) {
#pragma unroll
        for (int c = 0; c < LEAF - k; ++c) rkk[c] = x[k + c][0];
      }
      double part[LEAF];
#pragma unroll
      for (int q = 0; q < LEAF; ++q) part[q] = 0.0;
#pragma unroll
      for (int t = 0; t < kLeafRows; ++t) {
        const int i = tid + kWG * t;
        const double a = i > k ? x[k][t] : 0.0;
        part[0] += a * a;
#pragma unroll
        for (int c = 1; c < LEAF - k; ++c) part[c] += a * x[k + c][t];
      }
#pragma unroll
      for (int q = 0; q < LEAF - k; ++q) {
        const double t = wave_sum(part[q]);
        if (lane == 0) redk[wave * LEAF + q] = t;
      }
      __syncthreads();
      double tot[LEAF];
#pragma unroll
      for (int q = 0; q < LEAF - k; ++q) {
        double a = 0.0;
        for (int w = 0; w < nw; ++w) a += redk[w * LEAF + q];
        tot[q] = a;
      }
      const double sigma = tot[0];
      const double alpha = (k < mp) ? rkk[0] : 0.0;
      if (mp - k < 2 || sigma == 0.0) {
        tau_p = 0.0;
        beta_p = alpha;
        sc_p = 0.0;
      } else {
        beta_p = -copysign(sqrt(alpha * alpha + sigma), alpha);
        tau_p = (beta_p - alpha) / beta_p;
        sc_p = 1.0 / (alpha - beta_p);
      }
#pragma unroll
      for (int c = 1; c < LEAF; ++c) wc_p[c] = (c < LEAF - k && k < mp) ? rkk[c] + sc_p * tot[c] : 0.0;
      if (tid == 0) {
        tt[j0 + c0 + k] = tau_p;
        tl[k] = tau_p;
      }
    }
    // leaf back to A, into LDS (column-major, stride mp) for the Gram matrix and the later
    // panel columns, and V's columns c0.. into VW (rows c0 + i; the rows above are zero)
#pragma unroll
    for (int c = 0; c < LEAF; ++c)
#pragma unroll
      for (int t = 0; t < kLeafRows; ++t) {
        const int i = tid + kWG * t;
        if (i < mp) {
          A[(long long)(j0 + c0 + c) * ld + R0 + i] = x[c][t];
          lf[c * mp + i] = x[c][t];
        }
      }
#pragma unroll
    for (int t = 0; t < kLeafRows; ++t) {
      const int i = tid + kWG * t;
      if (i < mp) {
        double *vr = VW + (long long)(c0 + i) * 2 * kBand + c0;
#pragma unroll
        for (int c = 0; c < LEAF; ++c) vr[c] = (i == c) ? 1.0 : (i > c ? x[c][t] : 0.0);
      }
    }
    if (tid < c0) {
#pragma unroll
      for (int c = 0; c < LEAF; ++c) VW[(long long)tid * 2 * kBand + c0 + c] = 0.0;
    }
    __syncthreads();
    if (c0 + LEAF >= kBand) break;  // no later panel columns
    // leaf Gram matrix G(a, b) = v_a . v_b (a < b): 8 lanes per pair, rows strided by 8
    {
      const int g = tid >> 3, sub = tid & 7;
      double acc = 0.0;
      int a = 0, b = 0;
      if (g < LEAF * (LEAF - 1) / 2) {
        int t = g;
        a = 0;
        while (t >= LEAF - 1 - a) {
          t -= LEAF - 1 - a;
          ++a;
        }
        b = a + 1 + t;
        for (int i = b + 1 + sub; i < mp; i += 8) acc += lf[a * mp + i] * lf[b * mp + i];
      }
      acc = group8_sum(acc);
      if (g < LEAF * (LEAF - 1) / 2 && sub == 0) Gl[a * LEAF + b] = acc + (b < mp ? lf[a * mp + b] : 0.0);
    }
    __syncthreads();
    if (tid < LEAF) {
      const int a = tid;
      for (int i = 0; i < LEAF; ++i) {
        double t;
        if (i < a) t = 0.0;
        else if (i == a) t = tl[i];
        else {
          double s = 0.0;
          for (int q = a; q < i; ++q) s += Tl[a * LEAF + q] * Gl[q * LEAF + i];
          t = -tl[i] * s;
        }
        Tl[a * LEAF + i] = t;
      }
    }
    __syncthreads();
    // later panel columns: P(:, c) <- (I - V T^T V^T) P(:, c), one column per wave at a time
    // (the column is held in kRowRegs registers per lane; rows past mp are clamped)
    for (int c = c0 + LEAF + wave; c < kBand; c += nw) {
      double *pc = A + (long long)(j0 + c) * ld + R0;
      double x[kRowRegs];
#pragma unroll
      for (int t = 0; t < kRowRegs; ++t) {
        const int i = lane + 64 * t;
        x[t] = pc[i < mp ? i : mp - 1];
      }
      double y[LEAF];
#pragma unroll
      for (int a = 0; a < LEAF; ++a) y[a] = 0.0;
#pragma unroll
      for (int t = 0; t < kRowRegs; ++t) {
        const int i = lane + 64 * t;
        if (i < mp) {
#pragma unroll
          for (int a = 0; a < LEAF; ++a) {
            const double va = (i == a) ? 1.0 : (i > a ? lf[a * mp + i] : 0.0);
            y[a] += va * x[t];
          }
        }
      }
#pragma unroll
      for (int a = 0; a < LEAF; ++a) y[a] = wave_sum(y[a]);
      double z[LEAF];
#pragma unroll
      for (int a = 0; a < LEAF; ++a) {
        double s = 0.0;
#pragma unroll
        for (int q = 0; q <= a; ++q) s += Tl[q * LEAF + a] * y[q];
        z[a] = s;
      }
#pragma unroll
      for (int t = 0; t < kRowRegs; ++t) {
        const int i = lane + 64 * t;
        if (i < mp) {
          double s = 0.0;
#pragma unroll
          for (int a = 0; a < LEAF; ++a) {
            const double va = (i == a) ? 1.0 : (i > a ? lf[a * mp + i] : 0.0);
            s += va * z[a];
          }
          pc[i] = x[t] - s;
        }
      }
    }
    __syncthreads();
  }
  __syncthreads();
}

// One panel of the reduction to band form: QR of A(r:n, j0:j0+b), its T factor (row-major
// into Tp) and the two-sided update of A(r:n, r:n).  Kept out of line so that the products'
// per-thread addressing is not held in registers across panels.
__device__ __noinline__ void band_panel(double *__restrict__ A, int ld, int n, int j0, double *__restrict__ tt,
                                        double *__restrict__ Tp, double *__restrict__ VW, double *__restrict__ VT,
                                        double *__restrict__ Kst, double *__restrict__ Gst, double *sh, double *sm,
                                        double *red) {
  // out of line: the matrix and workspace pointers are wave-uniform and point to global memory,
  // sh, sm and red to LDS
  A = global_ptr(uniform_ptr(A));
  tt = global_ptr(uniform_ptr(tt));
  Tp = global_ptr(uniform_ptr(Tp));
  VW = global_ptr(uniform_ptr(VW));
  VT = global_ptr(uniform_ptr(VT));
  Kst = global_ptr(uniform_ptr(Kst));
  Gst = global_ptr(uniform_ptr(Gst));
  sh = lds_ptr(sh);
  sm = lds_ptr(sm);
  red = lds_ptr(red);
  ld = __builtin_amdgcn_readfirstlane(ld);
  n = __builtin_amdgcn_readfirstlane(n);
  j0 = __builtin_amdgcn_readfirstlane(j0);
  const int tid = threadIdx.x, nthr = blockDim.x;
  constexpr int b = kBand;
  const int r = j0 + b, m = n - r;
  // QR of the panel; V (explicit, unit diagonal) into the first half of the rows of [V | W]
  panel_qr(A, ld, n, j0, tt, sh, sm, red, VW);
  // Gst = -V^T V
  wg_atb32<false>(Gst, b, VW, 2 * b, VW, 2 * b, m, b, sh);
  // T (row-major), T(a, i) = -tau_i sum_{a <= q < i} T(a, q) G(q, i) for i > a, T(a, a) = tau_a:
  // G = V^T V and tau in LDS, lane a keeps row a in registers (T(a, q) = 0 for q < a, so every
  // lane runs the same fully unrolled recurrence)
  {
    double *Gs = sh, *taus = sh + b * b;
    for (int e = tid; e < b * b; e += nthr) Gs[e] = -Gst[e];
    if (tid < b) taus[tid] = tt[j0 + tid];
    __syncthreads();
    if (tid < b) {
      const int a = tid;
      double trow[b];
#pragma unroll
      for (int i = 0; i < b; ++i) {
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < i; ++q) acc += trow[q] * Gs[q * b + i];
        const double ti = taus[i];
        trow[i] = (i < a) ? 0.0 : ((i == a) ? ti : -ti * acc);
      }
#pragma unroll
      for (int i = 0; i < b; ++i) Tp[a * b + i] = trow[i];
    }
    __syncthreads();
  }
  // VT = -V T
  wg_gemm<G_A_RM | G_B_RM | G_OVERWRITE | G_C_RM, 128, 32>(VT, b, VW, 2 * b, Tp, b, m, b, b, sh);
  // X = A22 V T  (into the W half of [V | W])
  double *A22 = A + (long long)r * ld + r;
  wg_gemm<G_A_SYM | G_B_RM | G_OVERWRITE | G_C_RM, 128, 32>(VW + b, 2 * b, A22, ld, VT, b, m, b, m, sh);
  // K = (V T)^T X, then K/2
  wg_atb32<false>(Kst, b, VT, b, VW + b, 2 * b, m, b, sh);
  for (int e = tid; e < b * b; e += nthr) Kst[e] *= 0.5;
  __syncthreads();
  // W = X - V K/2
  wg_gemm<G_A_RM | G_C_RM, 128, 32>(VW + b, 2 * b, VW, 2 * b, Kst, b, m, b, b, sh);
  // A22 -= V W^T + W V^T (lower triangle)
  wg_gemm<G_TRANS_B | G_LOWER | G_A_RM | G_B_RM | G_EARLY_C>(A22, ld, VW, 2 * b, VW, 2 * b, m, m, 2 * b, sh, -1, b);
}

// ---------------------------------------------------------------------------------------
// Stage 1: reduction to band form (see the top of the file).  Dynamic LDS: max(LEAF * nmax,
// kGemmLds, kGemmLdsTall, kAtbLds) doubles.
__global__ void __launch_bounds__(256, 2) sy2sb_kernel(int n_clusters, const int *__restrict__ order,
                                                       double *__restrict__ mat, const long long *__restrict__ mat_off,
                                                       double *__restrict__ vec, const long long *__restrict__ vec_off,
                                                       const int *__restrict__ dmax, const int *__restrict__ dim,
                                                       const int *__restrict__ n_orb, int *__restrict__ queue) {
  extern __shared__ __attribute__((aligned(16))) double sh[];
  __shared__ double sm[2 * LEAF * LEAF + 4 * LEAF];
  __shared__ double red[10 * LEAF];
  const int tid = threadIdx.x, nthr = blockDim.x;
  constexpr int b = kBand;
  for (int s = queue_next(queue); s < n_clusters; s = queue_next(queue)) {
    const int c = order[s];
    const int n = dim[c], ld = n;
    const int M = n_orb[c];
    double *A = mat + mat_off[c];
    const VecLayout vl = VecLayout::make(dmax[c]);
    double *cv = vec + vec_off[c];
    double *tt = cv + vl.tau, *Tq = cv + vl.u;
    double *VW = cv + vl.vw, *VT = cv + vl.vt, *Kst = cv + vl.kg, *Gst = Kst + b * b;
    int j0 = 0;
    for (; j0 + b < n; j0 += b) {
      const int r = j0 + b, m = n - r, p = j0 / b;
      double *Tp = Tq + (long long)p * b * b;
      if (m < 2) {
        // a single reflector of length 1: identity
        __syncthreads();
        for (int e = tid; e < b * b; e += nthr) Tp[e] = 0.0;
        if (tid == 0) tt[j0] = 0.0;
        continue;
      }
      band_panel(A, ld, n, j0, tt, Tp, VW, VT, Kst, Gst, sh, sm, red);
    }
  }
  queue_leave(queue);
}

// ---------------------------------------------------------------------------------------
// Stage 2: bulge chasing (see the top of the file).
__device__ inline int sweep_steps(int n, int s) { return (s > n - 3) ? 0 : (n - 3 - s) / kBand + 1; }

// Per-lane select with a wave-uniform 64-bit lane mask: bit l set -> lane l takes b.  One
// v_cndmask with the mask in an SGPR pair (the compiler would otherwise build the mask per lane
// from compares).
__device__ inline unsigned lane_select(unsigned long long mask, unsigned a, unsigned b) {
  unsigned r;
  asm("v_cndmask_b32_e64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(mask));
  return r;
}

// A lane mask from its two halves, each put in a scalar register by an opaque move: folded into
// one 64-bit scalar move, a mask that is not an inline constant had its high half read as zero
// on gfx950 (measured: the lanes 32..63 of such a mask were off).
__device__ inline unsigned long long lane_mask(unsigned lo, unsigned hi) {
  asm volatile("" : "+s"(lo), "+s"(hi));
  return ((unsigned long long)hi << 32) | lo;
}

__device__ inline double band_load(__amdgpu_buffer_rsrc_t band, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(band, (int)voff, (int)soff, 0));
}

__device__ inline void band_store(__amdgpu_buffer_rsrc_t band, double x, unsigned voff, unsigned soff) {
  using U2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(band, 0, 0, 0));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U2, x), band, (int)voff, (int)soff, 0);
}

// A byte offset past the end of every band array: a buffer store through it is dropped (the
// hardware range check of a raw buffer view; loads past the end read zero).
constexpr unsigned kBandOob = 0x80000000u;

// The band array: entry (r, c), r >= c, at c kBandLd + r - c, read and written through a raw
// buffer view of its n kBandLd doubles (entries of rows past the matrix are zero and are neither
// read nor written by the steps).
//
// Loads of bulge step (s, j): element k of the lane's row (D rows on lanes 0..31, R rows on
// lanes 32..63) sits at r0 kBandLd + k (kBandLd - 1) + lane, so one load per k serves both
// halves, the lane offset in a register and the window in a scalar register.  Only entries that
// exist are fetched: D on and below the diagonal inside the window, R rows and columns inside the
// matrix; the other lanes are sent past the end of the buffer and read zero (the D part above the
// diagonal is taken from the tile later).
__device__ inline void chase_fetch(__amdgpu_buffer_rsrc_t band, double (&row)[kBand], int n, int s, int j) {
  constexpr unsigned LB = kBandLd, LD1 = kBandLd - 1;
  const unsigned lane = threadIdx.x & 63u;
  const unsigned vl = lane * 8u;
  const int r0 = __builtin_amdgcn_readfirstlane(s + 1 + j * kBand);
  const int len = min(kBand, n - r0), nr = max(0, min(kBand, n - r0 - len));
  const unsigned in_win = len >= 32 ? 0xFFFFFFFFu : ((1u << len) - 1u);
  const unsigned in_r = nr >= 32 ? 0xFFFFFFFFu : ((1u << nr) - 1u);
  const unsigned base = (unsigned)r0 * LB * 8u;
#pragma unroll
  for (int k = 0; k < kBand; ++k) {
    const unsigned long long keep = lane_mask((0xFFFFFFFFu << k) & in_win, k < len ? in_r : 0u);
    row[k] = band_load(band, lane_select(keep, kBandOob, vl) + (unsigned)k * LD1 * 8u, base);
  }
}

// B(s + 1 + lane mod 32, s), column s below its diagonal (the input of step 0 of sweep s).
__device__ inline double chase_column(__amdgpu_buffer_rsrc_t band, int s) {
  const unsigned cs = __builtin_amdgcn_readfirstlane((unsigned)s * kBandLd * 8u);
  return band_load(band, (1u + (threadIdx.x & 31u)) * 8u, cs);
}

// One bulge step (sweep s, step j) by one wavefront, on the rows chase_fetch loaded.  The
// reflector H_j = I - tau v v^T of the rows [r0, r1), r0 = s + 1 + j b, r1 = min(r0 + b, n), is
// in the sweep's LDS slot (tau, then v with v(0) = 1); step 0 first forms it from column s.  The
// step then
//   (c) updates the diagonal block D = B(r0:r1, r0:r1) <- H_j D H_j and the block below it,
//       R = B(r1:r2, r0:r1) <- R H_j, r2 = min(r1 + b, n) (this creates the bulge in R);
//   (a) when r2 - r1 >= 2, forms H_{j+1} from the first column of R, which it reduces to
//       beta e_0, stores it (A's upper triangle and the slot), and
//   (b) applies H_{j+1} from the left to the other columns of R.
// (a) and (b) belong to step j + 1 of the sweep; nothing else touches R between the two
// steps, so they run here while R is still in registers.  The D rows take their part above the
// diagonal from the tile (wt: kBand x (kBand + 1) doubles of the wave's LDS; wsv: kBand doubles;
// slot: kBand + 1 doubles of the sweep) and leave the step as full symmetric rows.  Rows past
// the matrix hold zeros throughout (they read zeros, and v, w, p and v1 are zero on them); so do
// the columns past the matrix.  The caller stores the window (chase_store).
__device__ void bulge_step(__amdgpu_buffer_rsrc_t band, double (&row)[kBand], double x, double *__restrict__ A,
                           int ld, int n, int s, int j, double *slot, double *wsv, double *wt) {
  constexpr int b = kBand, TS = kBand + 1;
  constexpr unsigned LB = kBandLd;
  // the lane index and (s, j) through opaque moves: keeps the compiler from hoisting the
  // per-lane addresses of the fully unrolled loops below out of the time loop
  int tx;
  asm volatile("v_mov_b32 %0, %1" : "=v"(tx) : "v"((int)threadIdx.x));
  s = __builtin_amdgcn_readfirstlane(s);
  j = __builtin_amdgcn_readfirstlane(j);
  asm volatile("" : "+s"(s), "+s"(j));
  const int lane = tx & 63;
  const bool lo = lane < 32;
  const int i = lo ? lane : lane - 32;
  const int r0 = s + 1 + j * b, len = min(b, n - r0), r1 = r0 + len;
  const int nr = min(b, n - r1);  // rows of R (0 on the last step of a sweep)
  const bool isRow = lo && i < len, isR = !lo && i < nr;
  double *vs = slot + 1;
  double tau, v;
  if (j == 0) {
    // reflector from x = B(s + 1 + i, s)
    const double sigma = wave_sum(isRow && i >= 1 ? x * x : 0.0);
    const double alpha = __shfl(x, 0, 64);
    double beta, sc;
    if (sigma == 0.0) {
      tau = 0.0;
      beta = alpha;
      sc = 0.0;
    } else {
      beta = -copysign(sqrt(alpha * alpha + sigma), alpha);
      tau = (beta - alpha) / beta;
      sc = 1.0 / (alpha - beta);
    }
    v = isRow ? (i == 0 ? 1.0 : x * sc) : 0.0;
    // column s: beta on the subdiagonal, zeros below (the D lanes past the matrix rewrite zeros)
    band_store(band, (i == 0) ? beta : 0.0, lane_select(lane_mask(0xFFFFFFFFu, 0u), kBandOob, (unsigned)(1 + i) * 8u),
               (unsigned)s * LB * 8u);
    if (isRow) A[(long long)(n - 1 - s) * ld + i] = (i == 0) ? tau : v;
    if (lo) vs[i] = v;
  } else {
    tau = slot[0];
    v = isRow ? vs[i] : 0.0;
  }
  __builtin_amdgcn_wave_barrier();
  // (c) the D lanes park their rows in the tile and read back full symmetric rows: entry k of
  // row i is tile(max(i, k), min(i, k)), at 33 max + min = 32 max + i + k
  if (lo) {
#pragma unroll
    for (int k = 0; k < b; ++k) wt[i * TS + k] = row[k];
  }
  __builtin_amdgcn_wave_barrier();
  if (lo) {
#pragma unroll
    for (int k = 0; k < b; ++k) row[k] = wt[32 * max(i, k) + i + k];
  }
  double pd[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < b; ++k) pd[k & 3] = fma(row[k], vs[k], pd[k & 3]);
  const double p = tau * ((pd[0] + pd[1]) + (pd[2] + pd[3]));
  const double vp = wave_sum(isRow ? v * p : 0.0);
  const double w = p - 0.5 * tau * vp * v;
  if (lo) wsv[i] = isRow ? w : 0.0;
  __builtin_amdgcn_wave_barrier();
  // v is read again from LDS below rather than held in 64 more registers
  asm volatile("" ::: "memory");
  // one pass for both lane halves: D rows take D - v w^T - w v^T, R rows R - p v^T
  {
    const double ca = isRow ? v : 0.0, cb = isRow ? w : (isR ? p : 0.0);
#pragma unroll
    for (int k = 0; k < b; ++k) row[k] = fma(-cb, vs[k], fma(-ca, wsv[k], row[k]));
  }
  if (nr >= 2) {
    // (a) H_{j+1} from x = R(:, 0)
    const double x1 = isR ? row[0] : 0.0;
    const double sigma = wave_sum(isR && i >= 1 ? x1 * x1 : 0.0);
    const double alpha = __shfl(x1, 32, 64);
    double beta, tau1, sc;
    if (sigma == 0.0) {
      tau1 = 0.0;
      beta = alpha;
      sc = 0.0;
    } else {
      beta = -copysign(sqrt(alpha * alpha + sigma), alpha);
      tau1 = (beta - alpha) / beta;
      sc = 1.0 / (alpha - beta);
    }
    const double v1 = isR ? (i == 0 ? 1.0 : x1 * sc) : 0.0;
    if (!lo) row[0] = (i == 0) ? beta : 0.0;
    if (isR) A[(long long)(n - 1 - s) * ld + (j + 1) * b + i] = (i == 0) ? tau1 : v1;
    // the slot passes H_{j+1} to the next step (every read of H_j above comes first)
    __builtin_amdgcn_wave_barrier();
    if (!lo) vs[i] = v1;
    if (lane == 32) slot[0] = tau1;
    // (b) R(:, 1:) <- H_{j+1} R(:, 1:), column dots through the tile
    if (!lo) {
#pragma unroll
      for (int c = 1; c < b; ++c) wt[i * TS + c] = v1 * row[c];
    }
    __builtin_amdgcn_wave_barrier();
    if (lo && i >= 1) {
      double dq[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int q = 0; q < b; ++q) dq[q & 3] += wt[q * TS + i];
      wsv[i] = tau1 * ((dq[0] + dq[1]) + (dq[2] + dq[3]));
    }
    __builtin_amdgcn_wave_barrier();
    if (!lo) {
#pragma unroll
      for (int c = 1; c < b; ++c) row[c] -= v1 * wsv[c];
    }
  }
}

// What chase_store writes of a step's window.
enum ChaseStore {
  kStoreAll = 0,      // D rows on and below the diagonal inside the window, R rows and columns inside the matrix
  kStoreDiag = 1,     // only the diagonal entry of the window's first column
  kStoreCol0Tail = 2, // only the first column's R entries past the first R row
  kStoreAllButCol0 = 3  // every column but the first, and the first column's R entries past the first R row
};

// Stores the window of step (s, j) from the rows (D rows on lanes 0..31, R rows on lanes
// 32..63), one store per column; the lanes of entries that are not written are sent past the end
// of the buffer.
__device__ inline void chase_store(__amdgpu_buffer_rsrc_t band, const double (&row)[kBand], int n, int s, int j,
                                   int mode) {
  constexpr unsigned LB = kBandLd, LD1 = kBandLd - 1;
  const unsigned vl = (threadIdx.x & 63u) * 8u;
  n = __builtin_amdgcn_readfirstlane(n);
  mode = __builtin_amdgcn_readfirstlane(mode);
  const int r0 = __builtin_amdgcn_readfirstlane(s + 1 + j * kBand);
  const int len = min(kBand, n - r0), nr = max(0, min(kBand, n - r0 - len));
  const unsigned in_win = len >= 32 ? 0xFFFFFFFFu : ((1u << len) - 1u);
  const unsigned in_r = nr >= 32 ? 0xFFFFFFFFu : ((1u << nr) - 1u);
  const unsigned base = (unsigned)r0 * LB * 8u;
  const unsigned c0lo = __builtin_amdgcn_readfirstlane(mode == kStoreAll ? 0xFFFFFFFFu : (mode == kStoreDiag ? 1u : 0u));
  const unsigned c0hi =
      __builtin_amdgcn_readfirstlane(mode == kStoreAll ? 0xFFFFFFFFu : (mode == kStoreDiag ? 0u : 0xFFFFFFFEu));
  const bool rest = mode == kStoreAll || mode == kStoreAllButCol0;
  band_store(band, row[0], lane_select(lane_mask(in_win & c0lo, in_r & c0hi), kBandOob, vl), base);
  if (rest) {
#pragma unroll
    for (int k = 1; k < kBand; ++k) {
      const unsigned long long keep = lane_mask((0xFFFFFFFFu << k) & in_win, k < len ? in_r : 0u);
      band_store(band, row[k], lane_select(keep, kBandOob, vl) + (unsigned)k * LD1 * 8u, base);
    }
  }
}

// Wavefronts per chase workgroup, each running one pair of sweeps at a time, and waves per SIMD
// (a wave holds two windows, 195 VGPRs).  Two waves per cluster and four clusters per CU beat
// four or eight waves per cluster with fewer clusters in flight (the steps are latency-bound).
#ifndef LDC_CHASE_WAVES
#define LDC_CHASE_WAVES 2
#endif
constexpr int kChaseWaves = LDC_CHASE_WAVES;
constexpr int kChaseOcc = 2;
constexpr int kMaxPairs = (kMaxDimTri - 1) / 2;  // sweeps 0 .. n - 3 taken two at a time

// The last pair time of the pair of sweeps (2p, 2p + 1), counted from the pair's start: the
// second sweep's step j runs at pair time j + 1; a lone last sweep ends at its own last step.
__device__ inline int pair_last(int n, int p) {
  const int s = 2 * p;
  return s + 1 <= n - 3 ? sweep_steps(n, s + 1) : sweep_steps(n, s) - 1;
}

// Pair time tau of the sweeps s = 2p and s + 1 on one wavefront: step (s, tau), then step
// (s + 1, tau - 1), which needs (s, tau) and nothing later.  The window of (s + 1, tau - 1) is
// that of (s, tau - 1) moved down and right by one: its rows and columns 0 .. b - 2 are the
// rows 1 .. and columns 1 .. of the first sweep's previous window (P, kept in registers), its
// last column is the first column of (s, tau)'s window, and its last row is zero left of that
// column (the sweeps before s annihilated those entries).  So only the first sweep's windows are
// loaded and only the second sweep's are stored, except what no later step of the second sweep
// covers: the diagonal entry of column s + 1 (tau = 0), the first column's entries past the
// first R row (zeros after the annihilation), and the whole last window of the first sweep when
// the second ends a step earlier.  A lone last sweep stores its windows itself.
__device__ inline void chase_pair(__amdgpu_buffer_rsrc_t band, double (&P)[kBand], double *__restrict__ A, int ld,
                                  int n, int p, int tau, double *slot0, double *slot1, double *wsv, double *wt) {
  constexpr unsigned LB = kBandLd;
  const int lane = threadIdx.x & 63;
  n = __builtin_amdgcn_readfirstlane(n);
  p = __builtin_amdgcn_readfirstlane(p);
  tau = __builtin_amdgcn_readfirstlane(tau);
  const int s = 2 * p;
  const bool solo = s + 1 > n - 3;
  const int J0 = sweep_steps(n, s), J1 = solo ? 0 : sweep_steps(n, s + 1);
  const bool first = tau < J0;
  double C[kBand];
  if (first) {
    chase_fetch(band, C, n, s, tau);
    const double x = tau == 0 ? chase_column(band, s) : 0.0;
    bulge_step(band, C, x, A, ld, n, s, tau, slot0, wsv, wt);
    chase_store(band, C, n, s, tau,
                solo ? kStoreAll : (tau == 0 ? kStoreDiag : (tau == J0 - 1 && J1 <= tau ? kStoreAllButCol0 : kStoreCol0Tail)));
  }
  if (tau >= 1 && tau - 1 < J1) {
    // column r0c = s + 1 + tau b from its diagonal down, on lanes 0 .. b
    const int r0c = s + 1 + tau * kBand;
    double c0 = 0.0;
    if (first)
      c0 = C[0];
    else if (r0c <= n - 1)
      c0 = band_load(band, lane <= kBand ? (unsigned)lane * 8u : kBandOob, (unsigned)r0c * LB * 8u);
    // step 0 of sweep s + 1 takes column s + 1 below its diagonal: P's first column, one row down
    const double x1 = __shfl_down(P[0], 1, 64);
#pragma unroll
    for (int k = 0; k < kBand - 1; ++k) {
      const double v = __shfl_down(P[k + 1], 1, 64);
      P[k] = lane == 63 ? 0.0 : v;
    }
    const double v = __shfl(c0, max(lane - (kBand - 1), 0), 64);
    P[kBand - 1] = lane >= kBand - 1 ? v : 0.0;
    bulge_step(band, P, x1, A, ld, n, s + 1, tau - 1, slot1, wsv, wt);
    chase_store(band, P, n, s + 1, tau - 1, kStoreAll);
  }
  if (first) {
#pragma unroll
    for (int k = 0; k < kBand; ++k) P[k] = C[k];
  }
}

// Bulge chasing of one cluster per workgroup.  Sweeps go in pairs (2p, 2p + 1), pair p on wave
// p mod nw; pair p starts at pair time T_p = max(T_{p-1} + 3, T_{p-nw} + last(p - nw) + 1): step
// (2p, tau) needs (2p - 1, tau + 1), which the previous pair runs at its pair time tau + 2, and a
// wave takes its next pair only after the last one ends.  Every step of pair time T then touches
// columns no other step of T touches, and a barrier ends each pair time.
__global__ void __launch_bounds__(64 * kChaseWaves, kChaseOcc) sb2st_kernel(int n_clusters, const int *__restrict__ order,
                                                    double *__restrict__ mat, const long long *__restrict__ mat_off,
                                                    double *__restrict__ vec, const long long *__restrict__ vec_off,
                                                    const int *__restrict__ dmax, const int *__restrict__ dim, int *__restrict__ queue) {
  __shared__ double wsv[kChaseWaves][kBand];
  __shared__ double wtile[kChaseWaves][kBand * (kBand + 1)];
  __shared__ double slots[kChaseWaves][2][kBand + 1];
  __shared__ int tstart[kMaxPairs];
  __shared__ int tlast;
  // the wave index in a scalar register: the pair numbers and band offsets derived from it are
  // wave-uniform (buffer offsets in vector registers would need a loop over lanes)
  const int tid = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(tid >> 6), nthr = blockDim.x, nw = nthr >> 6;
  constexpr int LB = kBandLd;
  for (int sidx = queue_next(queue); sidx < n_clusters; sidx = queue_next(queue)) {
    const int c = order[sidx];
    const int n = dim[c], ld = n;
    double *A = mat + mat_off[c];
    const VecLayout vl = VecLayout::make(dmax[c]);
    double *cv = vec + vec_off[c];
    double *dd = cv + vl.d, *ee = cv + vl.e;
    // n x kBandLd from the first 128-byte boundary of the band-reduction workspace (n kBandLd + 15
    // <= 3 kBand dmax doubles)
    double *Bd = cv + vl.vw;
    Bd += (16 - (int)((reinterpret_cast<unsigned long long>(Bd) >> 3) & 15)) & 15;
    const int npairs = n >= 3 ? (n - 1) / 2 : 0;
    __syncthreads();
    for (long long e = tid; e < (long long)n * LB; e += nthr) {
      const int cc = (int)(e / LB), d = (int)(e % LB);
      Bd[e] = (d <= kBand && cc + d < n) ? A[(long long)cc * ld + cc + d] : 0.0;
    }
    if (tid == 0) {
      int tl = -1;
      for (int q = 0; q < npairs; ++q) {
        int t = q == 0 ? 0 : tstart[q - 1] + 3;
        if (q >= nw) t = max(t, tstart[q - nw] + pair_last(n, q - nw) + 1);
        tstart[q] = t;
        tl = max(tl, t + pair_last(n, q));
      }
      tlast = tl;
    }
    __syncthreads();
    // raw buffer view of the band array (word 3: the gfx9 buffer format for untyped access)
    const __amdgpu_buffer_rsrc_t band = __builtin_amdgcn_make_buffer_rsrc(Bd, (short)0, n * LB * 8, 0x00020000);
    const int tend = tlast;
    int p = wave;
    double P[kBand];
#pragma unroll
    for (int k = 0; k < kBand; ++k) P[k] = 0.0;
    for (int t = 0; t <= tend; ++t) {
      if (p < npairs) {
        const int tau = t - __builtin_amdgcn_readfirstlane(tstart[p]);
        if (tau >= 0) {
          chase_pair(band, P, A, ld, n, p, tau, slots[wave][0], slots[wave][1], wsv[wave], wtile[wave]);
          if (tau == pair_last(n, p)) p += nw;
        }
      }
      __syncthreads();
    }
    for (int i = tid; i < n; i += nthr) {
      dd[i] = Bd[(long long)i * LB];
      ee[i] = (i < n - 1) ? Bd[(long long)i * LB + 1] : 0.0;
    }
  }
  queue_leave(queue);
}

// The two halves of the tracked-column product, out of line (each holds X in registers in its own
// layout; inlined together they would share one register budget).
__device__ __noinline__ void q1t_tracked(const double *A, int n, const double *Tq, double *X, int nc, double *lds) {
  wg_apply_q1<true>(A, n, Tq, X, kTrack, nc, lds);
}
__device__ __noinline__ void q2t_tracked(const double *A, int n, double *X, int nc, double *runs, double *ex) {
  wg_apply_q2_regs<true>(A, n, X, kTrack, nc, runs, ex);
}

// X <- Q^T X = Q2^T Q1^T X for the tracked columns: one workgroup per half (M columns) of a
// cluster's 2M.  Q1^T on the matrix cores from the band reduction's panels and T factors
// (wg_apply_q1), then Q2^T with the rows in register windows (wg_apply_q2_regs).  Dynamic LDS:
// max(kQ1Lds, 3 q2_lds_stride(nmax) + 2 x 32 x 16) doubles.
__global__ void __launch_bounds__(256, 2) q2x_kernel(int n_clusters, const int *__restrict__ order,
                                                  const double *__restrict__ mat, const long long *__restrict__ mat_off,
                                                  double *__restrict__ vec, const long long *__restrict__ vec_off,
                                                  const int *__restrict__ dmax, const int *__restrict__ dim,
                                                  const int *__restrict__ n_orb, int *__restrict__ queue) {
  extern __shared__ __attribute__((aligned(16))) double q2l[];
  for (int item = queue_next(queue); item < 2 * n_clusters; item = queue_next(queue)) {
    const int c = order[item >> 1], half = item & 1;
    const int n = dim[c], nc = n_orb[c];
    const VecLayout vl = VecLayout::make(dmax[c]);
    double *cv = vec + vec_off[c];
    double *X = cv + vl.G0 + half * nc;  // n x nc of the n x kTrack row-major block
    const double *A = mat + mat_off[c];
    __syncthreads();
    q1t_tracked(A, n, cv + vl.u, X, nc, q2l);
    if (n < 3) continue;
    q2t_tracked(A, n, X, nc, q2l, q2l + 3LL * q2_lds_stride(n));
  }
  queue_leave(queue);
}

// ---------------------------------------------------------------------------------------
void launch_sy2sb(Plan &p) {
  const size_t lds = sizeof(double) * std::max({(size_t)LEAF * cur_dim(p), (size_t)kGemmLds, (size_t)kGemmLdsTall,
                                                (size_t)kAtbLds});
  const int n = cur_count(p);
  const int grid = std::max(1, std::min(stage_grid(p, kTSy2sb, p.workgroups), n));
  hipLaunchKernelGGL(sy2sb_kernel, dim3(grid), dim3(kWG), lds, p.stream, n, cur_order(p), p.d_mat, p.d_mat_off,
                     p.d_vec, p.d_vec_off, p.d_dmax, p.d_dim, p.d_n_orb, p.d_queue);
}

void launch_sb2st(Plan &p) {
  // default: as many workgroups as are resident (kChaseOcc waves per SIMD)
  const int n = cur_count(p);
  const int grid = std::max(1, std::min(stage_grid(p, kTSb2st, p.n_cu * 4 * kChaseOcc / kChaseWaves), n));
  hipLaunchKernelGGL(sb2st_kernel, dim3(grid), dim3(64 * kChaseWaves), 0, p.stream, n, cur_order(p), p.d_mat,
                     p.d_mat_off, p.d_vec, p.d_vec_off, p.d_dmax, p.d_dim, p.d_queue);
}

void launch_q2x(Plan &p) {
  const size_t lds = sizeof(double) * std::max((size_t)kQ1Lds, 3 * (size_t)q2_lds_stride(cur_dim(p)) + 2 * 16 * 32);
  const int n = cur_count(p);
  const int grid = std::max(1, std::min(stage_grid(p, kTQ2x, 2 * p.n_cu), 2 * n));
  hipLaunchKernelGGL(q2x_kernel, dim3(grid), dim3(kWG), lds, p.stream, n, cur_order(p), p.d_mat, p.d_mat_off, p.d_vec,
                     p.d_vec_off, p.d_dmax, p.d_dim, p.d_n_orb, p.d_queue);
}

}  // namespace ldc
