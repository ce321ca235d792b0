// Divide-and-conquer eigensolver for the symmetric tridiagonal T = Q^T A Q of a cluster.
//
// T is split at every position into 1x1 leaves (Cuppen): T = diag(T1, T2) + rho v v^T with
// rho = |beta| and the two touching diagonal entries lowered by |beta|.  Merges run bottom
// up, one level at a time; every merge solves diag(d) + rho z z^T (z = last row of the
// left child's eigenvectors, sign(beta) x first row of the right child's) by:
//   sort the children's eigenvalues; deflate tiny z components and nearly equal poles
//   (Givens rotation); find each remaining root of the secular equation
//   1 + rho sum z_j^2/(d_j - lambda) = 0 by a safeguarded rational ("middle way")
//   iteration from the nearer pole, keeping d_j - lambda_i as (d_j - d_origin) - tau_i;
//   recompute z by Loewner's formula so the eigenvectors z_j/(d_j - lambda_i) are
//   orthogonal to working accuracy.
// The eigenvector matrix Z is never formed.  The forward pass carries the projections
// Z^T X of the tracked columns X (plus the first and last rows of the current Z blocks,
// which feed the z vectors), and stores per merge what a later product Z y needs: the sort
// permutation, the rotations, the secular-equation data and the output order.
#include "dc_common.h"
#include "wg_blas.h"

#include <type_traits>

namespace ldc {

constexpr double kEps = 2.220446049250313e-16;

// Root t (0-based) of 1/rho + sum_j z_j^2/(d_j - lambda) = 0 for ascending poles d (k of
// them), given the squares z2 of the z entries, as lambda = d_o + tau with o the nearer pole.
// An interior root starts from the midpoint of its two poles, whose sums also decide the
// nearer pole; the last root from the middle of (d_k, d_k + rho |z|^2].  Each pass evaluates
// the sums once and takes one safeguarded rational ("middle way") step; the root is done when
// the equation holds to its rounding error, the bracket has closed, or the step has become a
// rounding-level change of tau.  The passes of one root are a fixed sequence, whichever lane
// runs them and whatever it ran before.
struct SecularRoot {
  const double *d, *z2;
  int k, t, o, it;
  bool start;  // the next pass is the one at the midpoint (d0 = d_t)
  double rinv, rho, a, b, tau, d0;

  __device__ void begin(const double *dk, const double *z2k, int kk, double rh, int tt) {
    d = dk;
    z2 = z2k;
    k = kk;
    t = tt;
    rho = rh;
    rinv = 1.0 / rh;
    it = 0;
    if (t < k - 1) {
      start = true;
      o = t;
      d0 = d[t];
      tau = 0.5 * (d[t + 1] - d[t]);
      a = b = 0.0;
    } else {
      start = false;
      o = t;
      d0 = d[t];
      double zz = 0.0;
      for (int j = 0; j < k; ++j) zz += z2[j];
      a = 0.0;
      b = rho * zz * (1.0 + 8.0 * kEps);  // the last root lies in (d_k, d_k + rho |z|^2]
      tau = 0.5 * (a + b);
    }
  }

  // psi = sum_{j <= t} z_j^2 / (d_j - lambda), phi = sum_{j > t} (the same), and their
  // derivatives, d_j - lambda = (d_j - d0) - tau, in one loop over all j: with lambda strictly
  // between d_t and d_t+1 (the last root: above d_k) the terms of j <= t are exactly the
  // negative ones, so every lane of a merge runs the same j whatever its root.  Two partial
  // sums each; four terms formed stage by stage (their chains in flight together; the
  // reciprocal and its two Newton steps as in rcp_nr).
  __device__ void sums(double &psi, double &dpsi, double &phi, double &dphi) const {
    double sn[2] = {0.0, 0.0}, sp[2] = {0.0, 0.0}, dn[2] = {0.0, 0.0}, dpv[2] = {0.0, 0.0};
    auto add = [&](int h, double term, double r) {
      const double tn = fmin(term, 0.0), tp = fmax(term, 0.0);
      sn[h] += tn;
      sp[h] += tp;
      dn[h] = fma(tn, r, dn[h]);
      dpv[h] = fma(tp, r, dpv[h]);
    };
    int j = 0;
    for (; j + 4 <= k; j += 4) {
      double x[4], r[4], e[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) x[u] = (d[j + u] - d0) - tau;
#pragma unroll
      for (int u = 0; u < 4; ++u) r[u] = __builtin_amdgcn_rcp(x[u]);
#pragma unroll
      for (int u = 0; u < 4; ++u) e[u] = fma(-x[u], r[u], 1.0);
#pragma unroll
      for (int u = 0; u < 4; ++u) r[u] = fma(r[u], e[u], r[u]);
#pragma unroll
      for (int u = 0; u < 4; ++u) e[u] = fma(-x[u], r[u], 1.0);
#pragma unroll
      for (int u = 0; u < 4; ++u) r[u] = fma(r[u], e[u], r[u]);
#pragma unroll
      for (int u = 0; u < 4; ++u) add(u & 1, z2[j + u] * r[u], r[u]);
    }
    for (; j < k; ++j) {
      const double r = rcp_nr((d[j] - d0) - tau);
      add(0, z2[j] * r, r);
    }
    psi = sn[0] + sn[1];
    phi = sp[0] + sp[1];
    dpsi = dn[0] + dn[1];
    dphi = dpv[0] + dpv[1];
  }

  // one pass; true when the root is done (o and tau final)
  __device__ bool pass() {
    double psi, dpsi, phi, dphi;
    sums(psi, dpsi, phi, dphi);
    if (start) {  // at the midpoint: the sign decides the nearer pole and the bracket
      start = false;
      const double half = tau;
      if (rinv + psi + phi >= 0.0) {  // the root lies in (d_t, midpoint]
        o = t;
        a = 0.0;
        b = half;
      } else {
        o = t + 1;
        a = -half;
        b = 0.0;
        tau = a;
      }
      d0 = d[o];
    }
    const double g = rinv + psi + phi;
    const double err = 8.0 * (fabs(psi) + fabs(phi) + rinv) + fabs(tau) * (dpsi + dphi);
    if (g < 0.0) a = tau;
    else b = tau;
    if (fabs(g) <= kEps * err || (b - a) <= 2.0 * kEps * fmax(fabs(a), fabs(b))) return true;
    const double dl = (d[t] - d0) - tau;
    double eta = 0.0;
    bool ok = true;
    if (t < k - 1) {
      const double dr = (d[t + 1] - d0) - tau;
      const double cc = g - dl * dpsi - dr * dphi;
      const double aa = (dl + dr) * g - dl * dr * (dpsi + dphi);
      const double bb = dl * dr * g;
      const double disc = sqrt(fmax(0.0, aa * aa - 4.0 * bb * cc));
      if (cc == 0.0) {
        if (aa != 0.0) eta = bb / aa;
        else ok = false;
      } else if (aa <= 0.0) {
        eta = (aa - disc) / (2.0 * cc);
      } else {
        eta = 2.0 * bb / (aa + disc);
      }
    } else {
      const double cc = g - dl * dpsi;
      if (cc > 0.0) eta = dl + dl * dl * dpsi / cc;
      else ok = false;
    }
    double tn = ok ? tau + eta : 0.5 * (a + b);
    if (!(tn > a && tn < b)) tn = 0.5 * (a + b);
    const bool done = fabs(tn - tau) <= 2.0 * kEps * fabs(tn);
    tau = tn;
    return done || ++it >= 100;
  }
};

// Total order on doubles (IEEE order for numbers; NaNs at the ends): sorting and ranking by
// this key gives a permutation whatever the data.
__device__ inline long long dc_key(double x) {
  const long long b = __double_as_longlong(x);
  return b >= 0 ? b : (b ^ 0x7fffffffffffffffLL);
}

// LDS copies of the current level's merge data (n entries each), read many times by the
// secular solver, the Loewner formula, the norms, the output ranking and the row transform.
struct DcLds {
  double *d, *z, *zt, *tau, *nrm, *Ds;
  int *orig, *kpos, *jinv;
  static constexpr int kBytesPerRow = 6 * sizeof(double) + 3 * sizeof(int);
};

__device__ inline DcLds dc_lds(void *base, int nmax) {
  DcLds L;
  double *b = static_cast<double *>(base);
  L.d = b;
  L.z = b + nmax;
  L.zt = b + 2 * nmax;
  L.tau = b + 3 * nmax;
  L.nrm = b + 4 * nmax;
  L.Ds = b + 5 * nmax;
  L.orig = reinterpret_cast<int *>(b + 6 * nmax);
  L.kpos = L.orig + nmax;
  L.jinv = L.kpos + nmax;
  return L;
}

// Forward pass for one cluster (whole workgroup).  In: d, e (T), G0 rows = tracked X with
// nx columns.  Out: lam ascending, G0 rows = Z^T X (columns 0..nx-1), records.
__device__ void dc_forward(int n, const double *__restrict__ dd, const double *__restrict__ ee, int nx, DcWs ws,
                           DcLds S, DevStatus *st, int cid) {
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int Fc = nx, Lc = nx + 1, nt = nx + 2;
  __shared__ int qnext;                          // the secular roots' work queue
  __shared__ int mono[(kMaxDimTri + 63) / 64];  // per merge of 64 rows or more: kept values in order
  double *lam = ws.lam, *G0 = ws.G0, *G1 = ws.G1;
  for (int i = tid; i < n; i += nthr) {
    double di = dd[i];
    if (i > 0) di -= fabs(ee[i - 1]);
    if (i + 1 < n) di -= fabs(ee[i]);
    lam[i] = di;
    G0[(long long)i * kTrack + Fc] = 1.0;
    G0[(long long)i * kTrack + Lc] = 1.0;
  }
  __syncthreads();
  int L = 0;
  while ((1 << L) < n) ++L;
  for (int l = 0; l < L; ++l) {
    const int size = 1 << l, span = 2 * size;
    const DcRec R = dc_rec(ws.dcd, ws.dci, n, l);
    const int nmerge = (n + span - 1) / span;
    // Phase A0: stage the children's eigenvalues and z entries (z = last row of the left
    // child's eigenvectors, sign(beta) x first row of the right child's: tracked columns Lc,
    // Fc) in LDS and clear those columns.  S.tau, S.nrm and S.zt serve as scratch here; they
    // are filled with their own data in the later phases.
    for (int q = tid; q < n; q += nthr) {
      const int lo = q - q % span, m = lo + size, hi = min(lo + span, n);
      if (m >= hi) continue;
      const double sg = ee[m - 1] >= 0.0 ? 1.0 : -1.0;
      S.tau[q] = lam[q];
      const int col = q < m ? Lc : Fc;
      S.nrm[q] = (q < m ? 1.0 : sg) * G0[(long long)q * kTrack + col];
      G0[(long long)q * kTrack + col] = 0.0;
    }
    __syncthreads();
    // Phase A1: merge the two sorted children by rank (binary search in the other child;
    // the left child's element first on equal keys).  Keys are a total order on the doubles,
    // so the ranks form a permutation for any data.
    for (int q = tid; q < n; q += nthr) {
      const int lo = q - q % span, m = lo + size, hi = min(lo + span, n);
      if (m >= hi) continue;
      const long long key = dc_key(S.tau[q]);
      int a, b2;
      const bool left = q < m;
      if (left) {  // right elements with key < key(x)
        a = m;
        b2 = hi;
        while (a < b2) {
          const int c = (a + b2) >> 1;
          if (dc_key(S.tau[c]) < key) a = c + 1;
          else b2 = c;
        }
      } else {  // left elements with key <= key(y)
        a = lo;
        b2 = m;
        while (a < b2) {
          const int c = (a + b2) >> 1;
          if (dc_key(S.tau[c]) <= key) a = c + 1;
          else b2 = c;
        }
      }
      const int pos = left ? (q - lo) + (a - m) : (q - m) + (a - lo);
      R.perm[lo + pos] = q - lo;
      S.Ds[lo + pos] = S.tau[q];
      S.zt[lo + pos] = S.nrm[q];
    }
    __syncthreads();
    // Phase A2: normalise z and deflate.  The deflation is a sequential chain over the merge's
    // sorted entries (one lane); around it, a merge of 64 rows or more takes a whole wave for
    // the sums, the scaling and the kept copies, a smaller one a single thread.
    // deflate: the chain of merge [lo, hi) (Ds, zs: its sorted poles and normalised z, in
    // LDS); returns the kept count and the rotation count
    auto deflate = [&](int lo, int hi, double *Ds, double *zs, double rho, double tol, int &kp_out, int &nrot_out) {
      const int k = hi - lo;
      // the pending entry pj (the last one not deflated) is kept in registers with its z and
      // pole, so the chain from one j to the next is only the pair test; the test
      // |(d_j - d_pj) c s| <= tol of the rotation (c, s) = (z_j, -z_pj) / r, r^2 = z_pj^2 + z_j^2,
      // is taken as |(d_j - d_pj) z_j z_pj| <= tol r^2, and the rotation is formed only when
      // the pair deflates
      int kp = 0, nd = 0, nrot = 0, pj = -1;
      double zp = 0.0, dp = 0.0;
      for (int j = 0; j < k; ++j) {
        const double zj = zs[j], dj = Ds[j];
        if (rho * fabs(zj) <= tol) {
          R.kpos[hi - 1 - nd] = j;
          S.kpos[hi - 1 - nd] = j;
          ++nd;
          continue;
        }
        if (pj < 0) {
          pj = j;
          zp = zj;
          dp = dj;
          continue;
        }
        const double tdiff = dj - dp;
        if (fabs(tdiff * zj * zp) <= tol * (zp * zp + zj * zj)) {
          const double tau = hypot(zj, zp);
          const double c_ = zj / tau, s_ = -zp / tau;
          zs[j] = tau;
          zs[pj] = 0.0;
          R.ra[lo + nrot] = pj;
          R.rb[lo + nrot] = j;
          R.rc[lo + nrot] = c_;
          R.rs[lo + nrot] = s_;
          ++nrot;
          const double t1 = dp * c_ * c_ + dj * s_ * s_;
          const double dn = dp * s_ * s_ + dj * c_ * c_;
          Ds[j] = dn;
          Ds[pj] = t1;
          R.kpos[hi - 1 - nd] = pj;
          S.kpos[hi - 1 - nd] = pj;
          ++nd;
          zp = tau;
          dp = dn;
        } else {
          R.kpos[lo + kp] = pj;
          S.kpos[lo + kp] = pj;
          ++kp;
          zp = zj;
          dp = dj;
        }
        pj = j;
      }
      if (pj >= 0) {
        R.kpos[lo + kp] = pj;
        S.kpos[lo + kp] = pj;
        ++kp;
      }
      kp_out = kp;
      nrot_out = nrot;
    };
    if (span >= 64) {
      const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
      for (int mi = wave; mi < nmerge; mi += nthr >> 6) {
        const int lo = mi * span, m = lo + size, hi = min(lo + span, n);
        if (m >= hi) {
          if (lane == 0) R.cnt[lo] = -1;
          continue;
        }
        const int k = hi - lo;
        double *Ds = S.Ds + lo, *zs = S.zt + lo;
        double a2 = 0.0, dm = 0.0;
        for (int p = lane; p < k; p += 64) {
          a2 += zs[p] * zs[p];
          dm = fmax(dm, fabs(Ds[p]));
        }
        const double zn2 = wave_sum(a2), dmaxabs = wave_max(dm);
        const double zinv = 1.0 / sqrt(zn2);
        double zm = 0.0;
        for (int p = lane; p < k; p += 64) {
          const double v = zs[p] * zinv;
          zs[p] = v;
          zm = fmax(zm, fabs(v));
        }
        const double zmax = wave_max(zm);
        const double rho = fabs(ee[m - 1]) * zn2;
        const double tol = 8.0 * kEps * fmax(dmaxabs, zmax);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");  // the scaled z of every lane
        int kp = 0, nrot = 0;
        if (lane == 0) deflate(lo, hi, Ds, zs, rho, tol, kp, nrot);
        kp = __shfl(kp, 0);
        nrot = __shfl(nrot, 0);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");  // the chain's LDS writes
        if (lane == 0) {
          R.cnt[lo] = kp;
          R.cnt[lo + 1] = nrot;
          ws.rhov[lo] = rho;
        }
        for (int t = lane; t < kp; t += 64) {
          const int pos = S.kpos[lo + t];
          const double dv = Ds[pos];
          R.dK[lo + t] = dv;
          S.d[lo + t] = dv;
          S.z[lo + t] = zs[pos];
        }
        for (int t = lane; t < k; t += 64) S.jinv[lo + S.kpos[lo + t]] = t;
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");  // S.z complete before zs is reused
        // S.zt[lo + t] takes z^2 for the secular solver (zs is no longer needed)
        for (int t = lane; t < kp; t += 64) {
          const double zv = S.z[lo + t];
          S.zt[lo + t] = zv * zv;
        }
      }
    } else {
      for (int mi = tid; mi < nmerge; mi += nthr) {
        const int lo = mi * span, m = lo + size, hi = min(lo + span, n);
        if (m >= hi) {
          R.cnt[lo] = -1;
          continue;
        }
        const int k = hi - lo;
        double rho = fabs(ee[m - 1]);
        double *Ds = S.Ds + lo, *zs = S.zt + lo;
        double zn2 = 0.0, dmaxabs = 0.0;
        for (int p = 0; p < k; ++p) {
          zn2 += zs[p] * zs[p];
          dmaxabs = fmax(dmaxabs, fabs(Ds[p]));
        }
        const double zinv = 1.0 / sqrt(zn2);
        double zmax = 0.0;
        for (int p = 0; p < k; ++p) {
          zs[p] *= zinv;
          zmax = fmax(zmax, fabs(zs[p]));
        }
        rho *= zn2;
        const double tol = 8.0 * kEps * fmax(dmaxabs, zmax);
        int kp = 0, nrot = 0;
        deflate(lo, hi, Ds, zs, rho, tol, kp, nrot);
        R.cnt[lo] = kp;
        R.cnt[lo + 1] = nrot;
        ws.rhov[lo] = rho;
        // kept poles and z in order; S.zt[lo + t] takes z^2 for the secular solver (position
        // kpos[t] >= t, so no entry of zs is overwritten before it is read)
        for (int t = 0; t < kp; ++t) {
          const int pos = S.kpos[lo + t];
          const double dv = Ds[pos], zv = zs[pos];
          R.dK[lo + t] = dv;
          S.d[lo + t] = dv;
          S.z[lo + t] = zv;
          S.zt[lo + t] = zv * zv;
        }
        for (int t = 0; t < k; ++t) S.jinv[lo + S.kpos[lo + t]] = t;
      }
    }
    __syncthreads();
    // Phase A3: G1 = rows of G0 in sorted order.  One thread of the 256 per row: every source
    // index of the level is loaded at once, then the rows eight columns at a time
    {
      constexpr int RPT = (kMaxDimTri + 255) / 256;
      int src[RPT];
#pragma unroll
      for (int u = 0; u < RPT; ++u) {
        const int q = tid + 256 * u;
        src[u] = -1;
        if (q < n) {
          const int lo = q & ~(span - 1);
          const int c = R.cnt[lo], pq = R.perm[q];
          src[u] = c < 0 ? -1 : lo + pq;
        }
      }
      for (int c0 = 0; c0 < nt; c0 += 8) {
        double v[RPT][8];
#pragma unroll
        for (int u = 0; u < RPT; ++u) {
          const double *g = G0 + (long long)max(src[u], 0) * kTrack;
#pragma unroll
          for (int c = 0; c < 8; ++c) v[u][c] = g[min(c0 + c, kTrack - 1)];
        }
#pragma unroll
        for (int u = 0; u < RPT; ++u)
          if (src[u] >= 0) {
            double *o = G1 + (long long)(tid + 256 * u) * kTrack;
#pragma unroll
            for (int c = 0; c < 8; ++c)
              if (c0 + c < nt) o[c0 + c] = v[u][c];
          }
      }
    }
    __syncthreads();
    // Phase A4: deflation rotations, one thread per (merge, column)
    for (int e = tid; e < nmerge * nt; e += nthr) {
      const int mi = e / nt, cc = e % nt;
      const int lo = mi * span;
      const int kk = R.cnt[lo];
      if (kk < 0) continue;
      const int nrot = R.cnt[lo + 1];
      for (int r = 0; r < nrot; ++r) {
        const long long pa = (long long)(lo + R.ra[lo + r]) * kTrack + cc;
        const long long pb = (long long)(lo + R.rb[lo + r]) * kTrack + cc;
        const double c_ = R.rc[lo + r], s_ = R.rs[lo + r];
        const double ga = G1[pa], gb = G1[pb];
        G1[pa] = c_ * ga + s_ * gb;
        G1[pb] = c_ * gb - s_ * ga;
      }
    }
    __syncthreads();
    // Phase B: secular roots.  Every lane works through the roots of the level from a shared
    // queue: a lane whose root is done stores it and takes the next one at once, so the few
    // slow roots of a wave do not hold its other lanes idle.
    {
      if (tid == 0) qnext = nthr;
      __syncthreads();
      auto is_root = [&](int q) {
        const int lo = q & ~(span - 1), kp = R.cnt[lo];
        return kp >= 0 && q - lo < kp;
      };
      auto next_root = [&](int q) {
        while (q < n && !is_root(q)) q = atomicAdd(&qnext, 1);
        return q;
      };
      SecularRoot sr;
      int q = next_root(tid);
      if (q < n) {
        const int lo = q & ~(span - 1);
        sr.begin(S.d + lo, S.zt + lo, R.cnt[lo], ws.rhov[lo], q - lo);
      }
      while (__any(q < n)) {
        if (q < n && sr.pass()) {
          R.orig[q] = sr.o;
          R.tau[q] = sr.tau;
          S.orig[q] = sr.o;
          S.tau[q] = sr.tau;
          q = next_root(atomicAdd(&qnext, 1));
          if (q < n) {
            const int lo2 = q & ~(span - 1);
            sr.begin(S.d + lo2, S.zt + lo2, R.cnt[lo2], ws.rhov[lo2], q - lo2);
          }
        }
      }
    }
    __syncthreads();
    // Phase C: Loewner z
    for (int q = tid; q < n; q += nthr) {
      const int lo = q - q % span;
      const int kp = R.cnt[lo];
      const int j = q - lo;
      if (kp < 0 || j >= kp) continue;
      const double *dK = S.d + lo;
      const int *org = S.orig + lo;
      const double *tu = S.tau + lo;
      const double dj = dK[j];
      const double rho = ws.rhov[lo];
      // four partial products over i = u mod 4, the factors of four i formed stage by stage
      // (their chains in flight together); the factor of i = j is one
      double p4[4] = {1.0, 1.0, 1.0, 1.0};
      int i = 0;
      for (; i + 4 <= kp; i += 4) {
        double num[4], x[4], r[4], e[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          num[u] = (dj - dK[org[i + u]]) - tu[i + u];
          x[u] = dj - dK[i + u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) r[u] = __builtin_amdgcn_rcp(x[u]);
#pragma unroll
        for (int u = 0; u < 4; ++u) e[u] = fma(-x[u], r[u], 1.0);
#pragma unroll
        for (int u = 0; u < 4; ++u) r[u] = fma(r[u], e[u], r[u]);
#pragma unroll
        for (int u = 0; u < 4; ++u) e[u] = fma(-x[u], r[u], 1.0);
#pragma unroll
        for (int u = 0; u < 4; ++u) r[u] = fma(r[u], e[u], r[u]);
#pragma unroll
        for (int u = 0; u < 4; ++u) p4[u] *= (i + u == j) ? 1.0 : num[u] * r[u];
      }
      for (; i < kp; ++i) {
        if (i == j) continue;
        const double num = (dj - dK[org[i]]) - tu[i];
        p4[0] *= num * rcp_nr(dj - dK[i]);
      }
      const double prod = (-((dj - dK[org[j]]) - tu[j]) / rho) * ((p4[0] * p4[1]) * (p4[2] * p4[3]));
      const double ztj = copysign(sqrt(fmax(prod, 0.0)), S.z[lo + j]);
      R.zt[lo + j] = ztj;
      S.zt[lo + j] = ztj;
    }
    __syncthreads();
    // Phase D: eigenvector norms
    for (int q = tid; q < n; q += nthr) {
      const int lo = q - q % span;
      const int kp = R.cnt[lo];
      const int t = q - lo;
      if (kp < 0 || t >= kp) continue;
      const double *dK = S.d + lo, *zt = S.zt + lo;
      const double dorig = dK[S.orig[lo + t]], tau = S.tau[lo + t];
      // four partial sums, the terms of four j formed stage by stage
      double s4[4] = {0.0, 0.0, 0.0, 0.0};
      int j = 0;
      for (; j + 4 <= kp; j += 4) {
        double x[4], r[4], e[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) x[u] = (dK[j + u] - dorig) - tau;
#pragma unroll
        for (int u = 0; u < 4; ++u) r[u] = __builtin_amdgcn_rcp(x[u]);
#pragma unroll
        for (int u = 0; u < 4; ++u) e[u] = fma(-x[u], r[u], 1.0);
#pragma unroll
        for (int u = 0; u < 4; ++u) r[u] = fma(r[u], e[u], r[u]);
#pragma unroll
        for (int u = 0; u < 4; ++u) e[u] = fma(-x[u], r[u], 1.0);
#pragma unroll
        for (int u = 0; u < 4; ++u) r[u] = fma(r[u], e[u], r[u]);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const double v = zt[j + u] * r[u];
          s4[u] += v * v;
        }
      }
      for (; j < kp; ++j) {
        const double v = zt[j] * rcp_nr((dK[j] - dorig) - tau);
        s4[0] += v * v;
      }
      const double nv = sqrt((s4[0] + s4[1]) + (s4[2] + s4[3]));
      R.nrm[lo + t] = nv;
      S.nrm[lo + t] = nv;
    }
    __syncthreads();
    // Phase F: output order (ascending eigenvalue; ties by element index).  The values go to
    // S.z first (free after phase C), then every element counts the smaller ones of its merge
    // (the threads of a merge read the same entry in step).
    for (int q = tid; q < n; q += nthr) {
      const int lo = q - q % span;
      const int kp = R.cnt[lo];
      if (kp < 0) continue;
      const int x = q - lo;
      S.z[q] = x < kp ? S.d[lo + S.orig[lo + x]] + S.tau[lo + x] : S.Ds[lo + S.kpos[lo + x]];
    }
    __syncthreads();
    // In a merge of 64 rows or more whose kept values (the secular roots, one per interval
    // between poles) are non-decreasing, as they are unless rounding crossed a pole, the kept
    // part is counted by bisection (its (key, index) pairs increase) and only the deflated part
    // is scanned; otherwise every element of the merge is scanned.
    const bool big = span >= 64;
    if (big) {
      if (tid < nmerge) mono[tid] = 1;
      __syncthreads();
      for (int q = tid; q < n; q += nthr) {
        const int lo = q & ~(span - 1);
        const int kp = R.cnt[lo];
        if (kp >= 0 && q + 1 < lo + kp && dc_key(S.z[q]) > dc_key(S.z[q + 1])) mono[q / span] = 0;
      }
      __syncthreads();
    }
    for (int q = tid; q < n; q += nthr) {
      const int lo = q - q % span;
      const int kp = R.cnt[lo];
      if (kp < 0) continue;
      const int hi = min(lo + span, n);
      const int e = q - lo;
      const double ve = S.z[q];
      const long long ke = dc_key(ve);
      int rank = 0, x0 = lo;
      if (big && mono[lo / span]) {
        int a = lo, b = lo + kp;
        while (a < b) {
          const int m = (a + b) >> 1;
          const long long km = dc_key(S.z[m]);
          if (km < ke || (km == ke && m < q)) a = m + 1;
          else b = m;
        }
        rank = a - lo;
        x0 = lo + kp;
      }
      for (int x = x0; x < hi; ++x) {
        const long long kx = dc_key(S.z[x]);
        rank += (kx < ke) || (kx == ke && x < q);
      }
      R.oo[lo + rank] = e;
      lam[lo + rank] = ve;
    }
    __syncthreads();
    // Phase E: transformed rows, written in output order.  Output row q (merge [lo, lo+k),
    // element e = oo[q]) is sum_j u(e, j) G1(lo + kpos[j]) over the kept j (e < kp), or its own
    // row G1(lo + kpos[e]) (deflated e).  Row p of G1 carries its pole and Loewner z in S.Ds[p]
    // and S.z[p] (the merge data of row p's j = jinv[p]; a deflated row has z = 0 and a far
    // pole, so its weight is exactly zero), so every output row of a merge sums over all the
    // merge's rows p in order.
    for (int pp = tid; pp < n; pp += nthr) {
      const int lo = pp - pp % span;
      const int kp = R.cnt[lo];
      if (kp < 0) continue;
      const int j = S.jinv[pp];
      const bool kj = j < kp;
      S.Ds[pp] = kj ? S.d[lo + j] : 1e300;
      S.z[pp] = kj ? S.zt[lo + j] : 0.0;
    }
    // Merges of fewer than 64 rows: one output row per thread, the rows of its merge read
    // straight from memory (the threads of a merge load the same row together) and summed in
    // order; the columns are summed unguarded up to a compile-time count NT >= nt (entries past
    // nt are never stored).
    auto transform_small = [&](auto ntc) {
      constexpr int NT = decltype(ntc)::value;
      for (int q = tid; q < n; q += nthr) {
        const int lo = q & ~(span - 1);
        const int kp = R.cnt[lo];
        if (kp < 0) continue;
        const int hi = min(lo + span, n);
        const int e = R.oo[q];
        double *out = G0 + (long long)q * kTrack;
        if (e >= kp) {
          const double *g = G1 + (long long)(lo + S.kpos[lo + e]) * kTrack;
          for (int cc = 0; cc < nt; ++cc) out[cc] = g[cc];
          continue;
        }
        const double dorig = S.d[lo + S.orig[lo + e]], tau = S.tau[lo + e], ninv = 1.0 / S.nrm[lo + e];
        double acc[NT];
#pragma unroll
        for (int cc = 0; cc < NT; ++cc) acc[cc] = 0.0;
#pragma unroll 2
        for (int pp = lo; pp < hi; ++pp) {
          const double w = S.z[pp] * rcp_nr((S.Ds[pp] - dorig) - tau) * ninv;
          const double *g = G1 + (long long)pp * kTrack;
#pragma unroll
          for (int cc = 0; cc < NT; ++cc) acc[cc] += w * g[cc];
        }
#pragma unroll
        for (int cc = 0; cc < NT; ++cc)
          if (cc < nt) out[cc] = acc[cc];
      }
    };
    // Merges of 64 rows or more on the FP64 matrix cores.  Each wave takes 64 output rows of one
    // merge as four 16-row tiles t; step s covers the staged rows pp = lo + 4 s + l/16: lane l
    // forms the weight u(q, pp) of row q = q0 + 16 t + l % 16 of every tile (the A operands)
    // and reads the 16-column blocks of G1 row pp (B operands, lane l: column 16 c + l % 16)
    // straight from memory, so the waves need no barrier.  Register r of the tile's result then
    // holds row q0 + 16 t + l/16 + 4 r.  The NL columns past the last full block are summed on
    // the vector units per lane and added over the four lane groups at the end.  Rows that are
    // not kept take zero weights (pole 0, shift -1e300, scale 0: every weight is an exact zero)
    // and are copies of their own G1 row.
    auto transform_mfma = [&](auto ntl_c, auto nl_c) {
      constexpr int NTL = decltype(ntl_c)::value, NL = decltype(nl_c)::value;
      const int lane = tid & 63, li = lane & 15, lg = lane >> 4;
      const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
      for (int q0 = 64 * wave; q0 < n; q0 += nthr) {
        const int lo = q0 - q0 % span, hi = min(lo + span, n);
        const int kp = R.cnt[lo];
        if (kp < 0) continue;
        double dor[4], tu[4], ni[4];
        unsigned long long keptm[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int q = q0 + 16 * t + li;
          const int e = q < n ? R.oo[q] : kp;
          const bool kq = e < kp;
          dor[t] = kq ? S.d[lo + S.orig[lo + e]] : 0.0;
          tu[t] = kq ? S.tau[lo + e] : -1e300;
          ni[t] = kq ? 1.0 / S.nrm[lo + e] : 0.0;
          keptm[t] = __ballot(kq);
        }
        ldc_double4 acc[4][NTL];
        double pl[4][NL];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
#pragma unroll
          for (int c = 0; c < NTL; ++c) acc[t][c] = ldc_double4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int c = 0; c < NL; ++c) pl[t][c] = 0.0;
        }
        // one step: the data of staged row pp (fetched two steps ahead), then its weights and
        // products; rows past the merge (the tail step only) take zero weights
        struct Row {
          double D, z, gb[NTL], gl[NL];
        };
        auto fetch = [&](Row &b, int pp) {
          const int pr = min(pp, hi - 1);
          b.D = S.Ds[pr];
          b.z = S.z[pr];
          const double *g = G1 + (long long)pr * kTrack;
#pragma unroll
          for (int c = 0; c < NTL; ++c) b.gb[c] = g[16 * c + li];
#pragma unroll
          for (int c = 0; c < NL; ++c) b.gl[c] = g[16 * NTL + c];
        };
        auto step = [&](const Row &b, bool in) {
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const double w0 = b.z * rcp_nr((b.D - dor[t]) - tu[t]) * ni[t];
            const double w = in ? w0 : 0.0;
#pragma unroll
            for (int c = 0; c < NTL; ++c) acc[t][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(w, b.gb[c], acc[t][c], 0, 0, 0);
#pragma unroll
            for (int c = 0; c < NL; ++c) pl[t][c] += w * b.gl[c];
          }
        };
        const int pend = lo + ((hi - lo) & ~3);
        Row b0, b1;
        fetch(b0, lo + lg);
        fetch(b1, lo + 4 + lg);
        for (int p0 = lo; p0 < pend; p0 += 4) {
          const Row cur = b0;
          b0 = b1;
          fetch(b1, p0 + 8 + lg);
          step(cur, true);
        }
        if (pend < hi) step(b0, pend + lg < hi);
        // results: kept rows of the blocks, then the remaining columns (lane l: row q0 + l,
        // tile l/16), then the copies
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int q = q0 + 16 * t + lg + 4 * r;
            if (q < n && ((keptm[t] >> (lg + 4 * r)) & 1ull)) {
#pragma unroll
              for (int c = 0; c < NTL; ++c)
                if (16 * c + li < nt) G0[(long long)q * kTrack + 16 * c + li] = acc[t][c][r];
            }
          }
        double own[NL];
#pragma unroll
        for (int c = 0; c < NL; ++c) own[c] = 0.0;
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int c = 0; c < NL; ++c) {
            double v = pl[t][c];
            v += __shfl_xor(v, 16);
            v += __shfl_xor(v, 32);
            if (lg == t) own[c] = v;
          }
        const int q = q0 + lane;
        if (q < n) {
          const int e = R.oo[q];
          if (e < kp) {
#pragma unroll
            for (int c = 0; c < NL; ++c)
              if (16 * NTL + c < nt) G0[(long long)q * kTrack + 16 * NTL + c] = own[c];
          } else {
            const double *g = G1 + (long long)(lo + S.kpos[lo + e]) * kTrack;
            for (int cc = 0; cc < nt; ++cc) G0[(long long)q * kTrack + cc] = g[cc];
          }
        }
      }
    };
    if (span >= 64) {
      __syncthreads();  // the staged poles and weights are complete
      if (nt <= 20) transform_mfma(std::integral_constant<int, 1>{}, std::integral_constant<int, 4>{});
      else transform_mfma(std::integral_constant<int, 2>{}, std::integral_constant<int, kTrack - 32>{});
    } else if (nt <= 20) {
      transform_small(std::integral_constant<int, 20>{});
    } else {
      transform_small(std::integral_constant<int, kTrack>{});
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(256, 3) stedc_kernel(int n_clusters, const int *__restrict__ order,
                                                    double *__restrict__ vec, const long long *__restrict__ vec_off,
                                                    int *__restrict__ ivec, const long long *__restrict__ ivec_off,
                                                    const int *__restrict__ dmax, const int *__restrict__ dim,
                                                    const int *__restrict__ n_orb, DevStatus *st, int nmax, int *__restrict__ queue) {
  extern __shared__ __attribute__((aligned(16))) double dsh[];
  const DcLds S = dc_lds(dsh, nmax);
  for (int s = queue_next(queue); s < n_clusters; s = queue_next(queue)) {
    const int c = order[s];
    const int n = dim[c];
    const int M = n_orb[c];
    double *cv = vec + vec_off[c];
    const VecLayout vl = VecLayout::make(dmax[c]);
    DcWs ws = dc_ws(cv, ivec + ivec_off[c], dmax[c]);
    __syncthreads();
    dc_forward(n, cv + vl.d, cv + vl.e, 2 * M, ws, S, st, c);
    // weights w_mu = sum_alpha (C^T E_i)_{mu alpha} ((S C)^T E_i)_{mu alpha}
    double *w = cv + vl.w;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      const double *g = ws.G0 + (long long)i * kTrack;
      double acc = 0.0;
      for (int a = 0; a < M; ++a) acc += g[a] * g[M + a];
      w[i] = acc;
    }
    __syncthreads();
  }
  queue_leave(queue);
}

void launch_stedc(Plan &p) {
  const int dm = cur_dim(p);
  const size_t lds = (size_t)dm * DcLds::kBytesPerRow;
  // above 64 KB the dynamic LDS limit must be raised (not reached below 1092 rows)
  if (lds > 64 * 1024)
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(stedc_kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
  // default three workgroups per CU (at most 168 VGPRs; the LDS of a 711-row cluster is 42 KB):
  // more waves in flight for the latency-bound merges
  const int n = cur_count(p);
  const int grid = std::max(1, std::min(stage_grid(p, kTStedc, 3 * p.n_cu), n));
  hipLaunchKernelGGL(stedc_kernel, dim3(grid), dim3(kWG), lds, p.stream, n, cur_order(p), p.d_vec, p.d_vec_off,
                     p.d_ivec, p.d_ivec_off, p.d_dmax, p.d_dim, p.d_n_orb, p.d_status, dm, p.d_queue);
}

}  // namespace ldc
