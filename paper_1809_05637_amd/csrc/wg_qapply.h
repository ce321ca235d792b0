// Products with an orthogonal factor Q = H_0 H_1 ... H_{n-1-sh} stored as Householder
// reflectors below a band of width sh: H_k = I - tau_k v_k v_k^T, v_k(0:k+sh) = 0,
// v_k(k+sh) = 1, v_k(k+sh+1:) stored in A(k+sh+1:, k) (column-major, leading dimension ld).
// sh = 1 is the one-stage tridiagonalization, sh = b the reduction to band form.  Reflectors
// are grouped in panels of QP columns; a panel's product is I - V T V^T with T upper
// triangular (compact WY form): T(a,a) = tau_a, T(0:a, a) = -tau_a T(0:a, 0:a) (V(:, 0:a)^T v_a).
#pragma once

#include "dev_common.h"

namespace ldc {

constexpr int QP = 32;      // reflectors per panel
constexpr int QCH = 32;     // rows of V staged in LDS per step
constexpr int QXC = 32;     // largest number of columns of X
constexpr int QS = QP + 1;  // LDS row stride

// LDS (doubles) needed by wg_apply_q.
constexpr int kQapplyLds = QCH * QS + 3 * QP * QS + QCH * (QXC + 1);

// X (n rows, ncol <= QXC columns, row-major with row stride ldx) <- Q^T X (transpose) or
// Q X.  With make_T the panels' T factors are formed and stored in Tq (QP*QP per panel,
// row-major); otherwise the stored ones are used.  Whole workgroup (256 threads); lds:
// kQapplyLds.
__device__ void wg_apply_q(const double *__restrict__ A, int ld, int n, const double *__restrict__ tau, double *Tq,
                           bool make_T, double *X, int ldx, int ncol, bool transpose, double *lds, int sh = 1) {
  const int tid = threadIdx.x, nthr = blockDim.x, lane = tid & 63, wave = tid >> 6;
  double *Vc = lds;              // [QCH][QS]
  double *G = Vc + QCH * QS;     // [QP][QS]  V^T V
  double *T = G + QP * QS;       // [QP][QS]
  double *Y = T + QP * QS;       // [QP][QS]  V^T X, then T' V^T X
  double *Xc = Y + QP * QS;      // [QCH][QXC+1] rows of X
  constexpr int NACC = (QP * QP + QP * QXC) / 256;  // entries per thread (8)
  constexpr int NST = QCH * QP / 256;               // staged V (and X) entries per thread (4)
  static_assert(QCH * QXC <= NST * 256, "X staging");
  const int nref = n - sh;                          // reflectors 0..n-1-sh
  const int npan = nref > 0 ? (nref + QP - 1) / QP : 0;
  for (int pi = 0; pi < npan; ++pi) {
    const int p = transpose ? pi : (npan - 1 - pi);
    const int p0 = p * QP, nbp = min(QP, nref - p0);
    const int nG = make_T ? QP * QP : 0;
    const int nE = nG + QP * ncol;
    // Staging of QCH rows from r0: V entry e = tid + 256 u at (row e % QCH, reflector e / QCH),
    // X entry e at (row e / ncol, column e % ncol).  Loads are clamped into range and
    // unconditional (the next chunk is fetched while the current one is used); values outside
    // the reflectors or past row n are masked.
    auto fetch = [&](int r0, double *rv, double *rx) {
#pragma unroll
      for (int u = 0; u < NST; ++u) {
        const int e = tid + u * nthr, rr = e % QCH, t = e / QCH;
        const int r = r0 + rr, k = p0 + t;
        const double a = A[(long long)min(k, p0 + nbp - 1) * ld + min(r, n - 1)];
        const bool in = t < nbp && r < n;
        rv[u] = (in && r > k + sh) ? a : ((in && r == k + sh) ? 1.0 : 0.0);
        const int xr = r0 + e / ncol, xq = e % ncol;
        const double x = X[(long long)min(xr, n - 1) * ldx + xq];
        rx[u] = (e < QCH * ncol && xr < n) ? x : 0.0;
      }
    };
    auto stage = [&](const double *rv, const double *rx) {
#pragma unroll
      for (int u = 0; u < NST; ++u) {
        const int e = tid + u * nthr;
        Vc[(e % QCH) * QS + e / QCH] = rv[u];
        if (e < QCH * ncol) Xc[(e / ncol) * (QXC + 1) + e % ncol] = rx[u];
      }
    };
    double rv[NST], rx[NST];
    double acc[NACC];
#pragma unroll
    for (int q = 0; q < NACC; ++q) acc[q] = 0.0;
    fetch(p0 + sh, rv, rx);
    for (int r0 = p0 + sh; r0 < n; r0 += QCH) {
      __syncthreads();
      stage(rv, rx);
      __syncthreads();
      if (r0 + QCH < n) fetch(r0 + QCH, rv, rx);
      // whole chunks (rows past n are staged as zeros): fixed trip counts keep the LDS reads
      // in flight together
#pragma unroll
      for (int q = 0; q < NACC; ++q) {
        const int e = tid + q * 256;
        if (e < nE) {
          double s = 0.0;
          if (e < nG) {
            const int a = e / QP, b = e % QP;
            if (a < b) {
#pragma unroll 8
              for (int rr = 0; rr < QCH; ++rr) s += Vc[rr * QS + a] * Vc[rr * QS + b];
            }
          } else {
            const int a = (e - nG) / ncol, qq = (e - nG) % ncol;
#pragma unroll 8
            for (int rr = 0; rr < QCH; ++rr) s += Vc[rr * QS + a] * Xc[rr * (QXC + 1) + qq];
          }
          acc[q] += s;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < NACC; ++q) {
      const int e = tid + q * 256;
      if (e < nE) {
        if (e < nG) G[(e / QP) * QS + e % QP] = acc[q];
        else Y[((e - nG) / ncol) * QS + (e - nG) % ncol] = acc[q];
      }
    }
    // the first chunk of the second pass is fetched while T and T'Y are formed
    fetch(p0 + sh, rv, rx);
    __syncthreads();
    double *Tp = Tq + (long long)p * QP * QP;
    if (make_T) {
      // lane a of wave 0 forms row a of T: T(a, i) = -tau_i sum_{b=a}^{i-1} T(a, b) G(b, i)
      if (wave == 0 && lane < QP) {
        const int a = lane;
        for (int i = 0; i < QP; ++i) {
          double t;
          if (i >= nbp || i < a) t = 0.0;
          else if (i == a) t = tau[p0 + i];
          else {
            double sacc = 0.0;
            for (int b = a; b < i; ++b) sacc += T[a * QS + b] * G[b * QS + i];
            t = -tau[p0 + i] * sacc;
          }
          T[a * QS + i] = t;
          Tp[a * QP + i] = t;
        }
      }
    } else {
      for (int e = tid; e < QP * QP; e += nthr) T[(e / QP) * QS + e % QP] = Tp[e];
    }
    __syncthreads();
    // Y <- T^T Y (transpose) or T Y
    double z[(QP * QXC) / 256];
#pragma unroll
    for (int q = 0; q < (QP * QXC) / 256; ++q) {
      const int e = tid + q * 256;
      double s = 0.0;
      if (e < QP * ncol) {
        const int a = e / ncol, qq = e % ncol;
        if (transpose) {
          for (int b = 0; b <= a; ++b) s += T[b * QS + a] * Y[b * QS + qq];
        } else {
          for (int b = a; b < QP; ++b) s += T[a * QS + b] * Y[b * QS + qq];
        }
      }
      z[q] = s;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < (QP * QXC) / 256; ++q) {
      const int e = tid + q * 256;
      if (e < QP * ncol) Y[(e / ncol) * QS + e % ncol] = z[q];
    }
    // X(r, :) <- X(r, :) - V(r, :) Y, V and X staged in LDS by chunks of QCH rows
    for (int r0 = p0 + sh; r0 < n; r0 += QCH) {
      __syncthreads();
      stage(rv, rx);
      __syncthreads();
      if (r0 + QCH < n) fetch(r0 + QCH, rv, rx);
      const int rmax = min(QCH, n - r0);
      for (int e = tid; e < rmax * ncol; e += nthr) {
        const int rr = e / ncol, q = e % ncol;
        double s = 0.0;
#pragma unroll 8
        for (int t = 0; t < QP; ++t) s += Vc[rr * QS + t] * Y[t * QS + q];
        X[(long long)(r0 + rr) * ldx + q] = Xc[rr * (QXC + 1) + q] - s;
      }
    }
    __syncthreads();
  }
}

// X (n rows, ncol <= 32 columns, row-major, row stride ldx) <- Q2^T X (transpose) or Q2 X for
// the bulge-chasing reflectors of the band-to-tridiagonal step: sweep s holds the reflectors
// of rows [s + 1 + j b, s + 1 + j b + len), len = min(b, n - r0), b = kBand, stored in
// column n - 1 - s of A above the diagonal at rows j b.. (tau first, then v(1:len)); the
// steps of one sweep act on disjoint rows, so each sweep is one parallel step (16 or 32 lanes
// per reflector, one column each), and Q2 = (sweep 0) (sweep 1) ... in that order.
__device__ void wg_apply_q2(const double *__restrict__ A, int ld, int n, double *X, int ldx, int ncol,
                            bool transpose) {
  constexpr int b = kBand;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int gsh = ncol > 16 ? 5 : 4;
  const int grp = tid >> gsh, q = tid & ((1 << gsh) - 1), ngrp = nthr >> gsh;
  const int nsw = n - 2;  // sweeps 0 .. n-3
  for (int it = 0; it < nsw; ++it) {
    const int s = transpose ? it : nsw - 1 - it;
    const int nst = (n - 3 - s) / b + 1;
    for (int j = grp; j < nst; j += ngrp) {
      const int r0 = s + 1 + j * b, len = min(b, n - r0);
      const double *vp = A + (long long)(n - 1 - s) * ld + j * b;
      const double *xp = X + (long long)r0 * ldx + (q < ncol ? q : ncol - 1);
      double vv[b], xv[b];
      // clamped unconditional loads (all in flight together); entries past len are masked
#pragma unroll
      for (int i = 0; i < b; ++i) {
        const int ii = min(i, len - 1);
        const double t = vp[ii];
        vv[i] = (i < len) ? t : 0.0;
        xv[i] = xp[(long long)ii * ldx];
      }
      const double tau = vv[0];
      vv[0] = 1.0;
      double d = 0.0;
#pragma unroll
      for (int i = 0; i < b; ++i) d += vv[i] * xv[i];
      d *= tau;
      if (q < ncol) {
#pragma unroll
        for (int i = 0; i < b; ++i)
          if (i < len) X[(long long)(r0 + i) * ldx + q] = xv[i] - d * vv[i];
      }
    }
    __syncthreads();
  }
}

// The same product with X held in LDS (n >= 3; nc <= 16 columns, column-major: column q at
// Xs + q P, P = q2_lds_stride(n)): the only global reads are the reflectors, one contiguous run
// per sweep (n - 1 - s doubles of column n - 1 - s of A from row 0: per step tau, then v(1:len)),
// fetched two sweeps ahead into registers and parked in a triple buffer of LDS (runs: 3 x P
// doubles), one barrier per sweep.  Groups of 16 lanes take one reflector each, lane q one
// column.  The rows n .. P - 1 of every column and the kBand entries past the end of every
// parked run are zero, so every reflector, the last of a sweep too, runs over kBand rows with
// no clamping or masking (its entries past the run are zero and its rows past n stay zero), and
// every LDS offset is a lane base plus a constant.  Q2^T runs the sweeps forwards, Q2 backwards.
// Zeroes the padding rows and starts with the run prefetch (so a fill of Xs needs no barrier of
// its own before the call); ends with a barrier.
constexpr int kQ2Run = (kMaxDimTri + kBand + kWG - 1) / kWG;  // run elements per thread

// column stride of the LDS copy of X: at least n + kBand rows, odd (the columns of a group then
// start in distinct banks)
__host__ __device__ inline int q2_lds_stride(int n) { return (n + kBand) | 1; }

__device__ inline void q2_fetch_run(double *nx, const double *A, int n, int s, int tid, int nthr) {
  // run of sweep s (clamped unconditional loads; a sweep outside 0..n-3 reads its nearest)
  const int ss = max(0, min(s, n - 3)), len = n - 1 - ss;
  const double *src = A + (long long)(n - 1 - ss) * n;
#pragma unroll
  for (int u = 0; u < kQ2Run; ++u) nx[u] = src[min(tid + u * nthr, len - 1)];
}

__device__ void wg_apply_q2_lds(const double *__restrict__ A, int n, double *Xs, int nc, double *runs,
                                bool transpose) {
  constexpr int b = kBand;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int grp = tid >> 4, q = tid & 15, ngrp = nthr >> 4;
  const int P = q2_lds_stride(n);
  const int qc = min(q, nc - 1);
  double *xcol = Xs + (long long)qc * P;
  const int nsw = n - 2;  // sweeps 0 .. n-3
  auto sweep = [&](int it) { return max(0, min(transpose ? it : nsw - 1 - it, n - 3)); };
  // a parked run: its n - 1 - s entries, then kBand zeros
  auto park = [&](double *dst, const double *nx, int it) {
    const int nlen = n - 1 - sweep(it);
#pragma unroll
    for (int u = 0; u < kQ2Run; ++u) {
      const int e = tid + u * nthr;
      if (e < nlen + b) dst[e] = e < nlen ? nx[u] : 0.0;
    }
  };
  for (int e = tid; e < nc * (P - n); e += nthr) Xs[(long long)(e / (P - n)) * P + n + e % (P - n)] = 0.0;
  double nx0[kQ2Run], nx1[kQ2Run];
  q2_fetch_run(nx0, A, n, sweep(0), tid, nthr);
  q2_fetch_run(nx1, A, n, sweep(1), tid, nthr);
  park(runs, nx0, 0);
  __syncthreads();
  for (int it = 0; it < nsw; ++it) {
    const int s = sweep(it);
    // nx1 holds the run of the next sweep; fetch the one after
    q2_fetch_run(nx0, A, n, sweep(it + 2), tid, nthr);
    const double *cur = runs + (it % 3) * P;
    const int nst = (n - 3 - s) / b + 1;
    for (int j = grp; j < nst; j += ngrp) {
      const int r0 = s + 1 + j * b;
      const double *vp = cur + j * b;
      double *xp = xcol + r0;
      double vv[b], xv[b];
#pragma unroll
      for (int i = 0; i < b; ++i) {
        vv[i] = vp[i];
        xv[i] = xp[i];
      }
      const double tau = vv[0];
      vv[0] = 1.0;
      double d = 0.0;
#pragma unroll
      for (int i = 0; i < b; ++i) d += vv[i] * xv[i];
      d *= tau;
      if (q < nc) {
#pragma unroll
        for (int i = 0; i < b; ++i) xp[i] = xv[i] - d * vv[i];
      }
    }
    park(runs + ((it + 1) % 3) * P, nx1, it + 1);
#pragma unroll
    for (int u = 0; u < kQ2Run; ++u) nx1[u] = nx0[u];
    __syncthreads();
  }
}

}  // namespace ldc
