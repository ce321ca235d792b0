// Small dense eigen-routines for the per-atom LNO step (Sec. II.B, Eq. 20-22), written for
// one thread per atom (M_j <= 16).  Host and device compile the same code, so the routines
// can be checked on the CPU.
//
//  * hessenberg(): orthogonal reduction to upper Hessenberg form by Householder reflectors,
//    accumulating the transformation;
//  * schur(): Francis double-shift QR iteration to real Schur form T = Z^T A Z (1x1 blocks
//    for real eigenvalues, 2x2 blocks for complex-conjugate pairs), accumulating Z;
//  * kept_basis(): eigenvectors of selected eigenvalues by back-substitution in T, mapped
//    back with Z; a complex pair contributes the real and imaginary parts of one member;
//  * sym_jacobi(): cyclic Jacobi eigendecomposition of a small symmetric matrix (used for
//    the S_jj-Loewdin orthonormalisation of the kept span).
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

// Real Schur form of an upper Hessenberg a, accumulating into z.  wr/wi: eigenvalues in
// Schur order (a complex pair occupies two consecutive positions, +wi first).  Returns 0 on
// success, -1 if an eigenvalue needed more than 200 iterations (an exceptional shift
// is taken every 10 iterations).
LDC_HD inline int schur(double *a, double *z, double *wr, double *wi, int n) {
  double anorm = 0.0;
  for (int i = 0; i < n; ++i)
    for (int j = (i > 0 ? i - 1 : 0); j < n; ++j) anorm += fabs(a[i * LD + j]);
  int nn = n - 1;
  double t = 0.0;
  int its = 0;
  while (nn >= 0) {
    int l;
    for (l = nn; l >= 1; --l) {
      double s = fabs(a[(l - 1) * LD + l - 1]) + fabs(a[l * LD + l]);
      if (s == 0.0) s = anorm;
      if (fabs(a[l * LD + l - 1]) + s == s) {
        a[l * LD + l - 1] = 0.0;
        break;
      }
    }
    double x = a[nn * LD + nn];
    if (l == nn) {  // one real root
      a[nn * LD + nn] = x + t;
      wr[nn] = x + t;
      wi[nn] = 0.0;
      --nn;
      its = 0;
      continue;
    }
    double y = a[(nn - 1) * LD + nn - 1];
    double w = a[nn * LD + nn - 1] * a[(nn - 1) * LD + nn];
    if (l == nn - 1) {  // a 2x2 block
      double p = 0.5 * (y - x);
      double q = p * p + w;
      double zz = sqrt(fabs(q));
      x += t;
      a[nn * LD + nn] = x;
      a[(nn - 1) * LD + nn - 1] = y + t;
      if (q >= 0.0) {  // real pair: rotate the block to triangular form
        zz = p + sgn_copy(zz, p);
        wr[nn - 1] = wr[nn] = x + zz;
        if (zz != 0.0) wr[nn] = x - w / zz;
        wi[nn - 1] = wi[nn] = 0.0;
        x = a[nn * LD + nn - 1];
        double s = fabs(x) + fabs(zz);
        p = x / s;
        q = zz / s;
        double r = sqrt(p * p + q * q);
        p /= r;
        q /= r;
        for (int j = nn - 1; j < n; ++j) {
          zz = a[(nn - 1) * LD + j];
          a[(nn - 1) * LD + j] = q * zz + p * a[nn * LD + j];
          a[nn * LD + j] = q * a[nn * LD + j] - p * zz;
        }
        for (int i = 0; i <= nn; ++i) {
          zz = a[i * LD + nn - 1];
          a[i * LD + nn - 1] = q * zz + p * a[i * LD + nn];
          a[i * LD + nn] = q * a[i * LD + nn] - p * zz;
        }
        for (int i = 0; i < n; ++i) {
          zz = z[i * LD + nn - 1];
          z[i * LD + nn - 1] = q * zz + p * z[i * LD + nn];
          z[i * LD + nn] = q * z[i * LD + nn] - p * zz;
        }
        a[nn * LD + nn - 1] = 0.0;
      } else {  // complex pair
        wr[nn - 1] = wr[nn] = x + p;
        wi[nn - 1] = zz;
        wi[nn] = -zz;
      }
      nn -= 2;
      its = 0;
      continue;
    }
    // no root yet: one double-shift QR sweep on rows/columns l..nn
    if (its >= 200) return -1;
    if (its > 0 && its % 10 == 0) {  // exceptional shift
      t += x;
      for (int i = 0; i <= nn; ++i) a[i * LD + i] -= x;
      double s = fabs(a[nn * LD + nn - 1]) + fabs(a[(nn - 1) * LD + nn - 2]);
      y = x = 0.75 * s;
      w = -0.4375 * s * s;
    }
    ++its;
    int m;
    double p = 0.0, q = 0.0, r = 0.0, zz;
    for (m = nn - 2; m >= l; --m) {
      zz = a[m * LD + m];
      r = x - zz;
      double s = y - zz;
      p = (r * s - w) / a[(m + 1) * LD + m] + a[m * LD + m + 1];
      q = a[(m + 1) * LD + m + 1] - zz - r - s;
      r = a[(m + 2) * LD + m + 1];
      s = fabs(p) + fabs(q) + fabs(r);
      p /= s;
      q /= s;
      r /= s;
      if (m == l) break;
      double u = fabs(a[m * LD + m - 1]) * (fabs(q) + fabs(r));
      double vv = fabs(p) * (fabs(a[(m - 1) * LD + m - 1]) + fabs(zz) + fabs(a[(m + 1) * LD + m + 1]));
      if (u + vv == vv) break;
    }
    for (int i = m + 2; i <= nn; ++i) {
      a[i * LD + i - 2] = 0.0;
      if (i != m + 2) a[i * LD + i - 3] = 0.0;
    }
    for (int k = m; k <= nn - 1; ++k) {
      if (k != m) {
        p = a[k * LD + k - 1];
        q = a[(k + 1) * LD + k - 1];
        r = 0.0;
        if (k != nn - 1) r = a[(k + 2) * LD + k - 1];
        x = fabs(p) + fabs(q) + fabs(r);
        if (x != 0.0) {
          p /= x;
          q /= x;
          r /= x;
        }
      }
      double s = sgn_copy(sqrt(p * p + q * q + r * r), p);
      if (s != 0.0) {
        if (k == m) {
          if (l != m) a[k * LD + k - 1] = -a[k * LD + k - 1];
        } else {
          a[k * LD + k - 1] = -s * x;
        }
        p += s;
        x = p / s;
        y = q / s;
        zz = r / s;
        q /= p;
        r /= p;
        for (int j = k; j < n; ++j) {
          p = a[k * LD + j] + q * a[(k + 1) * LD + j];
          if (k != nn - 1) {
            p += r * a[(k + 2) * LD + j];
            a[(k + 2) * LD + j] -= p * zz;
          }
          a[(k + 1) * LD + j] -= p * y;
          a[k * LD + j] -= p * x;
        }
        int mmin = nn < k + 3 ? nn : k + 3;
        for (int i = 0; i <= mmin; ++i) {
          p = x * a[i * LD + k] + y * a[i * LD + k + 1];
          if (k != nn - 1) {
            p += zz * a[i * LD + k + 2];
            a[i * LD + k + 2] -= p * r;
          }
          a[i * LD + k + 1] -= p * q;
          a[i * LD + k] -= p;
        }
        for (int i = 0; i < n; ++i) {
          p = x * z[i * LD + k] + y * z[i * LD + k + 1];
          if (k != nn - 1) {
            p += zz * z[i * LD + k + 2];
            z[i * LD + k + 2] -= p * r;
          }
          z[i * LD + k + 1] -= p * q;
          z[i * LD + k] -= p;
        }
      }
    }
  }
  // entries below the subdiagonal are logically zero (bulge remnants are never read)
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
