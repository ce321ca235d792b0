// Small dense eigen-routines for the per-atom LNO step (Sec. II.B, Eq. 20-22), written for
// one thread per atom (M_j <= 16).  Host and device compile the same code, so the routines
// can be checked on the CPU.
//
//  * hessenberg(): orthogonal reduction to upper Hessenberg form by Householder reflectors,
//    accumulating the transformation;
//  * schur(): Francis double-shift QR iteration to real Schur form T = Z^T A Z (1x1 blocks
//    for real eigenvalues, 2x2 blocks for complex-conjugate pairs), accumulating Z; written
//    from the statement of the algorithm in Golub & Van Loan, Matrix Computations, Sec. 7.5
//    (small_reflector / apply_small_reflector for the bulge, settle_block2 for a deflated
//    2x2 block);
//  * schur_vector(): the eigenvector of one eigenvalue by back-substitution in T (mapped
//    back with Z by lno_atom); a complex pair contributes the real and imaginary parts of
//    one member;
//  * sym_jacobi(): cyclic Jacobi eigendecomposition of a small symmetric matrix (used for
//    the S_jj-Loewdin orthonormalisation of the kept span);
//  * lno_atom(): the whole per-atom step (rank rule, kept span, Loewdin basis).
// tests/test_small_eig_host.py compiles this header for the host and checks it against
// LAPACK's general eigensolver.
#pragma once

#include <math.h>

#ifndef LDC_HD
#if defined(__HIPCC__)
#define LDC_HD __host__ __device__
#else
#define LDC_HD
#endif
#endif

namespace ldc {
namespace small {

constexpr int LD = 16;

LDC_HD inline double sgn_copy(double a, double b) { return b >= 0.0 ? fabs(a) : -fabs(a); }

// a (n x n, row stride LD) -> upper Hessenberg; z = accumulated orthogonal transform.
LDC_HD inline void hessenberg(double *a, double *z, int n) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) z[i * LD + j] = (i == j) ? 1.0 : 0.0;
  double v[LD];
  for (int c = 0; c + 2 < n; ++c) {
    double alpha = a[(c + 1) * LD + c];
    double sig = 0.0;
    for (int r = c + 2; r < n; ++r) sig += a[r * LD + c] * a[r * LD + c];
    if (sig == 0.0) continue;
    double beta = -sgn_copy(sqrt(alpha * alpha + sig), alpha);
    double tau = (beta - alpha) / beta;
    double scal = 1.0 / (alpha - beta);
    v[c + 1] = 1.0;
    for (int r = c + 2; r < n; ++r) v[r] = a[r * LD + c] * scal;
    // A <- H A on rows c+1..n-1
    for (int j = c; j < n; ++j) {
      double s = 0.0;
      for (int r = c + 1; r < n; ++r) s += v[r] * a[r * LD + j];
      s *= tau;
      for (int r = c + 1; r < n; ++r) a[r * LD + j] -= s * v[r];
    }
    // A <- A H and Z <- Z H on columns c+1..n-1
    for (int i = 0; i < n; ++i) {
      double s = 0.0, t = 0.0;
      for (int r = c + 1; r < n; ++r) {
        s += a[i * LD + r] * v[r];
        t += z[i * LD + r] * v[r];
      }
      s *= tau;
      t *= tau;
      for (int r = c + 1; r < n; ++r) {
        a[i * LD + r] -= s * v[r];
        z[i * LD + r] -= t * v[r];
      }
    }
    a[(c + 1) * LD + c] = beta;
    for (int r = c + 2; r < n; ++r) a[r * LD + c] = 0.0;
  }
}

// Householder reflector of a 2- or 3-vector x (len = 2 or 3): P = I - tau v v^T with v(0) = 1
// and P x = beta e_0.  Returns false (P = I) when x(1:) is already zero.
LDC_HD inline bool small_reflector(const double *x, int len, double *v, double &tau, double &beta) {
  double tail = 0.0;
  for (int i = 1; i < len; ++i) tail += x[i] * x[i];
  v[0] = 1.0;
  if (tail == 0.0) {
    for (int i = 1; i < len; ++i) v[i] = 0.0;
    tau = 0.0;
    beta = x[0];
    return false;
  }
  const double nrm = sqrt(x[0] * x[0] + tail);
  beta = x[0] > 0.0 ? -nrm : nrm;  // sign opposite to x(0): no cancellation in x(0) - beta
  const double inv = 1.0 / (x[0] - beta);
  for (int i = 1; i < len; ++i) v[i] = x[i] * inv;
  tau = (beta - x[0]) / beta;
  return true;
}

// Applies P = I - tau v v^T (v of length len, acting on indices k..k+len-1) to the rows
// k.. of a on the columns [c0, c1), and to the columns k.. of a on the rows [0, r1) and of z
// on the rows [0, n).
LDC_HD inline void apply_small_reflector(double *a, double *z, int n, int k, int len, const double *v, double tau,
                                         int c0, int c1, int r1) {
  for (int c = c0; c < c1; ++c) {
    double s = 0.0;
    for (int i = 0; i < len; ++i) s += v[i] * a[(k + i) * LD + c];
    s *= tau;
    for (int i = 0; i < len; ++i) a[(k + i) * LD + c] -= s * v[i];
  }
  for (int r = 0; r < r1; ++r) {
    double s = 0.0;
    for (int i = 0; i < len; ++i) s += a[r * LD + k + i] * v[i];
    s *= tau;
    for (int i = 0; i < len; ++i) a[r * LD + k + i] -= s * v[i];
  }
  for (int r = 0; r < n; ++r) {
    double s = 0.0;
    for (int i = 0; i < len; ++i) s += z[r * LD + k + i] * v[i];
    s *= tau;
    for (int i = 0; i < len; ++i) z[r * LD + k + i] -= s * v[i];
  }
}

// Brings the trailing 2 x 2 block at rows/columns (p, p + 1) of the quasi-triangular a to its
// final form: with real eigenvalues it is rotated to upper-triangular form (first column of
// the rotation = an eigenvector of the block), otherwise it is left as it is.  wr/wi receive
// the two eigenvalues (a complex pair as mean +- i omega, the + member at p).
LDC_HD inline void settle_block2(double *a, double *z, int n, int p, double *wr, double *wi) {
  const double b00 = a[p * LD + p], b01 = a[p * LD + p + 1];
  const double b10 = a[(p + 1) * LD + p], b11 = a[(p + 1) * LD + p + 1];
  const double half = 0.5 * (b00 - b11);
  const double disc = half * half + b01 * b10;  // the eigenvalues are b11 + half +- sqrt(disc)
  if (disc < 0.0) {
    const double om = sqrt(-disc);
    wr[p] = wr[p + 1] = 0.5 * (b00 + b11);
    wi[p] = om;
    wi[p + 1] = -om;
    return;
  }
  wi[p] = wi[p + 1] = 0.0;
  if (b10 == 0.0) {  // already triangular
    wr[p] = b00;
    wr[p + 1] = b11;
    return;
  }
  // lam = b11 + g with g of the sign of half (the larger root in magnitude, no cancellation);
  // (g, b10) is an eigenvector of the block for lam
  const double g = half + (half >= 0.0 ? sqrt(disc) : -sqrt(disc));
  const double r = sqrt(g * g + b10 * b10);
  const double cs = g / r, sn = b10 / r;
  for (int c = p; c < n; ++c) {  // rows p, p + 1 <- G^T (rows)
    const double u = a[p * LD + c], w = a[(p + 1) * LD + c];
    a[p * LD + c] = cs * u + sn * w;
    a[(p + 1) * LD + c] = -sn * u + cs * w;
  }
  for (int rr = 0; rr <= p + 1; ++rr) {  // columns p, p + 1 <- (columns) G
    const double u = a[rr * LD + p], w = a[rr * LD + p + 1];
    a[rr * LD + p] = cs * u + sn * w;
    a[rr * LD + p + 1] = -sn * u + cs * w;
  }
  for (int rr = 0; rr < n; ++rr) {
    const double u = z[rr * LD + p], w = z[rr * LD + p + 1];
    z[rr * LD + p] = cs * u + sn * w;
    z[rr * LD + p + 1] = -sn * u + cs * w;
  }
  a[(p + 1) * LD + p] = 0.0;
  wr[p] = a[p * LD + p];
  wr[p + 1] = a[(p + 1) * LD + p + 1];
}

// Real Schur form T = Z^T A Z of an upper Hessenberg a (n <= LD), accumulating into z: the
// implicitly double-shifted QR iteration of Francis, as stated in Golub & Van Loan, Matrix
// Computations (Sec. 7.5: the Francis step and the QR algorithm with deflation).  The active
// window [lo, hi] is the trailing unreduced Hessenberg block; a subdiagonal entry below
// 2^-53 times its two diagonal neighbours is set to zero (deflation).  A 1 x 1 window is a
// real eigenvalue; a 2 x 2 window is settled by settle_block2.  Otherwise one Francis step:
// the shifts s1, s2 are the two eigenvalues of the window's trailing 2 x 2 block, the first
// column of (H - s1)(H - s2) restricted to the window starts a bulge that 3 x 3 reflectors
// chase down to the bottom.  Every 11th step of a window uses an ad hoc
// shift pair built from the window's last subdiagonal entries instead, which breaks the
// cycles that the standard shifts can fall into.  The reflectors act on whole rows and
// columns of a (not only the window), so a ends as the full quasi-triangular T needed for
// the eigenvectors.  wr/wi: eigenvalues in Schur order (a complex pair at two consecutive
// positions, +wi first).  Returns 0, or -1 if a window needed more than 100 steps.
LDC_HD inline int schur(double *a, double *z, double *wr, double *wi, int n) {
  double scale = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = (i > 0 ? i - 1 : 0); j < n; ++j) scale = fmax(scale, fabs(a[i * LD + j]));
  const double eps = 1.1102230246251565e-16;  // 2^-53
  int hi = n - 1, steps = 0;
  while (hi >= 0) {
    int lo = hi;
    for (; lo > 0; --lo) {
      double nb = fabs(a[(lo - 1) * LD + lo - 1]) + fabs(a[lo * LD + lo]);
      if (nb == 0.0) nb = scale;
      if (fabs(a[lo * LD + lo - 1]) <= eps * nb) {
        a[lo * LD + lo - 1] = 0.0;
        break;
      }
    }
    if (lo == hi) {
      wr[hi] = a[hi * LD + hi];
      wi[hi] = 0.0;
      --hi;
      steps = 0;
      continue;
    }
    if (lo == hi - 1) {
      settle_block2(a, z, n, hi - 1, wr, wi);
      hi -= 2;
      steps = 0;
      continue;
    }
    if (steps >= 100) return -1;
    ++steps;
    // First column of (H - s1)(H - s2) on the window, divided by h10 (a common factor that
    // leaves the reflector unchanged), written with differences of nearby diagonal entries so
    // that nothing cancels when the shifts lie close to h00:
    //   x = (h00 - s1)(h00 - s2) / h10 + h01,  y = (h11 - h00) + (h00 - s1) + (h00 - s2),  z = h21.
    const double h00 = a[lo * LD + lo], h01 = a[lo * LD + lo + 1];
    const double h10 = a[(lo + 1) * LD + lo], h11 = a[(lo + 1) * LD + lo + 1];
    const double h21 = a[(lo + 2) * LD + lo + 1];
    double prod, sum;  // (h00 - s1)(h00 - s2) and (h00 - s1) + (h00 - s2)
    if (steps % 11 == 0) {
      // ad hoc shifts: the complex pair h + w (0.6 +- 0.8 i) with h the last diagonal entry and
      // w the size of the last two subdiagonal entries (not symmetric about h, so that a
      // spectrum symmetric about h cannot hold the iteration in place)
      const double w = fabs(a[hi * LD + hi - 1]) + fabs(a[(hi - 1) * LD + hi - 2]);
      const double e = h00 - a[hi * LD + hi] - 0.6 * w;
      prod = e * e + 0.64 * w * w;
      sum = 2.0 * e;
    } else {
      // the eigenvalues of the window's trailing 2 x 2 block [p00 p01; p10 p11]
      const double p00 = a[(hi - 1) * LD + hi - 1], p01 = a[(hi - 1) * LD + hi];
      const double p10 = a[hi * LD + hi - 1], p11 = a[hi * LD + hi];
      const double e1 = h00 - p00, e2 = h00 - p11;
      prod = e1 * e2 - p01 * p10;
      sum = e1 + e2;
    }
    double x[3] = {prod / h10 + h01, (h11 - h00) + sum, h21};
    {
      const double sc = fabs(x[0]) + fabs(x[1]) + fabs(x[2]);
      if (sc > 0.0)
        for (int i = 0; i < 3; ++i) x[i] /= sc;
    }
    double v[3], tau, beta;
    for (int k = lo; k <= hi - 1; ++k) {
      const int len = (k <= hi - 2) ? 3 : 2;
      if (k > lo) {
        for (int i = 0; i < len; ++i) x[i] = a[(k + i) * LD + k - 1];
      }
      if (small_reflector(x, len, v, tau, beta)) {
        const int c0 = (k > lo) ? k - 1 : k;
        const int r1 = (k + 3 < hi ? k + 3 : hi) + 1;
        apply_small_reflector(a, z, n, k, len, v, tau, c0, n, r1);
        if (k > lo) {
          a[k * LD + k - 1] = beta;
          for (int i = 1; i < len; ++i) a[(k + i) * LD + k - 1] = 0.0;
        }
      }
    }
  }
  // entries below the subdiagonal are zero in exact arithmetic; clear the rounding residue
  for (int i = 2; i < n; ++i)
    for (int j = 0; j + 1 < i; ++j) a[i * LD + j] = 0.0;
  return 0;
}

struct cplx {
  double re, im;
};
LDC_HD inline cplx cmul(cplx a, cplx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
LDC_HD inline cplx csub(cplx a, cplx b) { return {a.re - b.re, a.im - b.im}; }
LDC_HD inline cplx cadd(cplx a, cplx b) { return {a.re + b.re, a.im + b.im}; }
LDC_HD inline cplx cdiv(cplx a, cplx b) {
  // Smith's algorithm
  if (fabs(b.re) >= fabs(b.im)) {
    double r = b.im / b.re, den = b.re + b.im * r;
    return {(a.re + a.im * r) / den, (a.im - a.re * r) / den};
  }
  double r = b.re / b.im, den = b.im + b.re * r;
  return {(a.re * r + a.im) / den, (a.im * r - a.re) / den};
}
LDC_HD inline double cabs1(cplx a) { return fabs(a.re) + fabs(a.im); }

// Eigenvector (complex in general) of the Schur-form T for the eigenvalue at Schur
// position p (the first position of a complex pair, eigenvalue wr + i|wi|).  x: n entries.
LDC_HD inline void schur_vector(const double *T, int n, int p, double lre, double lim, cplx *x, double smin) {
  for (int i = 0; i < n; ++i) x[i] = {0.0, 0.0};
  cplx lam = {lre, lim};
  int top;  // highest index already set
  if (lim == 0.0) {
    x[p] = {1.0, 0.0};
    top = p;
  } else {
    // 2x2 block at (p, p+1): rank-1 matrix (B - lam I); pick the better-scaled row
    double a11 = T[p * LD + p], a12 = T[p * LD + p + 1], a21 = T[(p + 1) * LD + p], a22 = T[(p + 1) * LD + p + 1];
    if (fabs(a21) >= fabs(a12)) {
      // row 2: a21 x_p + (a22 - lam) x_{p+1} = 0 with x_{p+1} = 1
      x[p + 1] = {1.0, 0.0};
      x[p] = cdiv(csub(lam, {a22, 0.0}), {a21, 0.0});
    } else {
      // row 1: (a11 - lam) x_p + a12 x_{p+1} = 0 with x_p = 1
      x[p] = {1.0, 0.0};
      x[p + 1] = cdiv(csub(lam, {a11, 0.0}), {a12, 0.0});
    }
    top = p + 1;
  }
  int q = p - 1;
  while (q >= 0) {
    bool block2 = (q > 0) && (T[q * LD + q - 1] != 0.0);
    if (!block2) {
      cplx r = {0.0, 0.0};
      for (int j = q + 1; j <= top; ++j) r = cadd(r, cmul({T[q * LD + j], 0.0}, x[j]));
      cplx dd = csub({T[q * LD + q], 0.0}, lam);
      if (cabs1(dd) < smin) dd = {smin, 0.0};
      x[q] = cdiv({-r.re, -r.im}, dd);
      q -= 1;
    } else {
      int q0 = q - 1;
      cplx r0 = {0.0, 0.0}, r1 = {0.0, 0.0};
      for (int j = q + 1; j <= top; ++j) {
        r0 = cadd(r0, cmul({T[q0 * LD + j], 0.0}, x[j]));
        r1 = cadd(r1, cmul({T[q * LD + j], 0.0}, x[j]));
      }
      cplx m11 = csub({T[q0 * LD + q0], 0.0}, lam), m12 = {T[q0 * LD + q], 0.0};
      cplx m21 = {T[q * LD + q0], 0.0}, m22 = csub({T[q * LD + q], 0.0}, lam);
      cplx det = csub(cmul(m11, m22), cmul(m12, m21));
      if (cabs1(det) < smin * smin) det = {smin * smin, 0.0};
      cplx b0 = {-r0.re, -r0.im}, b1 = {-r1.re, -r1.im};
      x[q0] = cdiv(csub(cmul(m22, b0), cmul(m12, b1)), det);
      x[q] = cdiv(csub(cmul(m11, b1), cmul(m21, b0)), det);
      q -= 2;
    }
  }
}

// Cyclic Jacobi eigendecomposition of a symmetric k x k matrix g (row stride LD):
// on return g holds the eigenvalues on its diagonal and v the eigenvectors (columns).
LDC_HD inline void sym_jacobi(double *g, double *v, int k) {
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) v[i * LD + j] = (i == j) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, dia = 0.0;
    for (int i = 0; i < k; ++i) {
      dia += g[i * LD + i] * g[i * LD + i];
      for (int j = i + 1; j < k; ++j) off += g[i * LD + j] * g[i * LD + j];
    }
    if (off <= 1e-34 * dia || off == 0.0) break;
    for (int p = 0; p < k; ++p)
      for (int q = p + 1; q < k; ++q) {
        double apq = g[p * LD + q];
        if (apq == 0.0) continue;
        double app = g[p * LD + p], aqq = g[q * LD + q];
        double theta = (aqq - app) / (2.0 * apq);
        double t = sgn_copy(1.0, theta) / (fabs(theta) + sqrt(theta * theta + 1.0));
        double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int r = 0; r < k; ++r) {
          double grp = g[r * LD + p], grq = g[r * LD + q];
          g[r * LD + p] = c * grp - s * grq;
          g[r * LD + q] = s * grp + c * grq;
        }
        for (int r = 0; r < k; ++r) {
          double gpr = g[p * LD + r], gqr = g[q * LD + r];
          g[p * LD + r] = c * gpr - s * gqr;
          g[q * LD + r] = s * gpr + c * gqr;
        }
        for (int r = 0; r < k; ++r) {
          double vrp = v[r * LD + p], vrq = v[r * LD + q];
          v[r * LD + p] = c * vrp - s * vrq;
          v[r * LD + q] = s * vrp + c * vrq;
        }
      }
  }
}

// Full LNO computation for one atom.
//   lam_in: Lambda (m x m, row stride LD); sjj: S_jj block (m x m, row stride LD).
//   rule: lambda_th, k_min, k_max (<0: m), fixed (>=0 overrides the count).
//   out u: m x k column-major with leading dimension m (u[r + c*m]).
// Returns k >= 0, or -1 (QR did not converge), -2 (kept span rank deficient).
LDC_HD inline int lno_atom(const double *lam_in, const double *sjj, int m, double lambda_th, int k_min, int k_max,
                           int fixed, double *u, double *work /* >= 6*LD*LD doubles */) {
  double *a = work;
  double *z = work + LD * LD;
  double *b = work + 2 * LD * LD;   // basis, m x k (row stride LD)
  double *g = work + 3 * LD * LD;
  double *vg = work + 4 * LD * LD;
  double *tmp = work + 5 * LD * LD;
  double wr[LD], wi[LD];
  int idx[LD];
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) a[i * LD + j] = lam_in[i * LD + j];
  hessenberg(a, z, m);
  if (schur(a, z, wr, wi, m) != 0) return -1;
  // rank eigenvalues by real part, descending; stable in Schur position
  for (int i = 0; i < m; ++i) idx[i] = i;
  for (int i = 1; i < m; ++i) {
    int v = idx[i];
    int j = i - 1;
    while (j >= 0 && wr[idx[j]] < wr[v]) {
      idx[j + 1] = idx[j];
      --j;
    }
    idx[j + 1] = v;
  }
  // conjugate-pair members: the +wi member first (they share the real part exactly)
  for (int i = 0; i + 1 < m; ++i) {
    int s0 = idx[i], s1 = idx[i + 1];
    if (wi[s0] != 0.0 && wr[s0] == wr[s1] && wi[s0] < 0.0 && wi[s1] > 0.0) {
      idx[i] = s1;
      idx[i + 1] = s0;
    }
  }
  int kmax = k_max < 0 ? m : (k_max > m ? m : k_max);
  int k;
  if (fixed >= 0) {
    k = fixed;
  } else {
    k = 0;
    for (int i = 0; i < m; ++i) k += (wr[i] >= lambda_th);
    if (k < k_min) k = k_min;
    if (k > kmax) k = kmax;
  }
  if (k < 0) k = 0;
  if (k > m) k = m;
  if (k > 0 && k < m) {
    int s0 = idx[k - 1], s1 = idx[k];
    bool same_pair = (wi[s0] != 0.0) && (wr[s0] == wr[s1]) && (wi[s0] == -wi[s1]);
    if (same_pair) k = (k + 1 <= kmax) ? k + 1 : k - 1;
  }
  // basis of the kept span
  double scale = 0.0;
  for (int i = 0; i < m; ++i) scale = fmax(scale, fabs(wr[i]) + fabs(wi[i]));
  double smin = fmax(2.2e-16 * scale, 1e-290);
  cplx x[LD];
  int col = 0;
  for (int t = 0; t < k;) {
    int s = idx[t];
    if (wi[s] == 0.0) {
      schur_vector(a, m, s, wr[s], 0.0, x, smin);
      double nrm = 0.0;
      for (int r = 0; r < m; ++r) {
        double acc = 0.0;
        for (int q = 0; q < m; ++q) acc += z[r * LD + q] * x[q].re;
        b[r * LD + col] = acc;
        nrm += acc * acc;
      }
      nrm = 1.0 / sqrt(nrm);
      for (int r = 0; r < m; ++r) b[r * LD + col] *= nrm;
      col += 1;
      t += 1;
    } else {
      // pair at Schur positions p, p+1 (p = the smaller of the two)
      int p = s;
      int s2 = idx[t + 1 < m ? t + 1 : t];
      if (s2 < p) p = s2;
      schur_vector(a, m, p, wr[s], fabs(wi[s]), x, smin);
      double n0 = 0.0, n1 = 0.0;
      for (int r = 0; r < m; ++r) {
        double re = 0.0, im = 0.0;
        for (int q = 0; q < m; ++q) {
          re += z[r * LD + q] * x[q].re;
          im += z[r * LD + q] * x[q].im;
        }
        b[r * LD + col] = re;
        b[r * LD + col + 1] = im;
        n0 += re * re;
        n1 += im * im;
      }
      n0 = 1.0 / sqrt(n0);
      n1 = 1.0 / sqrt(n1);
      for (int r = 0; r < m; ++r) {
        b[r * LD + col] *= n0;
        b[r * LD + col + 1] *= n1;
      }
      col += 2;
      t += 2;
    }
  }
  k = col;
  if (k == 0) return 0;
  // Loewdin: U = B (B^T S_jj B)^{-1/2}
  for (int i = 0; i < m; ++i)
    for (int c = 0; c < k; ++c) {
      double acc = 0.0;
      for (int q = 0; q < m; ++q) acc += sjj[i * LD + q] * b[q * LD + c];
      tmp[i * LD + c] = acc;  // S_jj B
    }
  for (int c1 = 0; c1 < k; ++c1)
    for (int c2 = 0; c2 < k; ++c2) {
      double acc = 0.0;
      for (int q = 0; q < m; ++q) acc += b[q * LD + c1] * tmp[q * LD + c2];
      g[c1 * LD + c2] = acc;
    }
  for (int c1 = 0; c1 < k; ++c1)
    for (int c2 = c1 + 1; c2 < k; ++c2) {
      double s = 0.5 * (g[c1 * LD + c2] + g[c2 * LD + c1]);
      g[c1 * LD + c2] = g[c2 * LD + c1] = s;
    }
  sym_jacobi(g, vg, k);
  double emax = 0.0;
  for (int c = 0; c < k; ++c) emax = fmax(emax, g[c * LD + c]);
  for (int c = 0; c < k; ++c)
    if (!(g[c * LD + c] > 1e-13 * emax)) return -2;
  // tmp = V diag(e^{-1/2}) V^T
  for (int c1 = 0; c1 < k; ++c1)
    for (int c2 = 0; c2 < k; ++c2) {
      double acc = 0.0;
      for (int q = 0; q < k; ++q) acc += vg[c1 * LD + q] * vg[c2 * LD + q] / sqrt(g[q * LD + q]);
      tmp[c1 * LD + c2] = acc;
    }
  for (int r = 0; r < m; ++r)
    for (int c = 0; c < k; ++c) {
      double acc = 0.0;
      for (int q = 0; q < k; ++q) acc += b[r * LD + q] * tmp[q * LD + c];
      u[r + c * m] = acc;
    }
  return k;
}

}  // namespace small
}  // namespace ldc
