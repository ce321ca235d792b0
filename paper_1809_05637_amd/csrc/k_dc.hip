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

namespace ldc {

constexpr double kEps = 2.220446049250313e-16;

// Root t (0-based) of 1/rho + sum_j z_j^2/(d_j - lambda) = 0 for ascending poles d (k of
// them).  Returns the origin pole o and tau with lambda = d_o + tau.
__device__ void secular_root(const double *__restrict__ d, const double *__restrict__ z, int k, double rho, int t,
                             int *o_out, double *tau_out) {
  const double rinv = 1.0 / rho;
  int o;
  double a, b;
  if (t < k - 1) {
    const double delta = d[t + 1] - d[t];
    const double dt = d[t];
    double g = rinv;
    for (int j = 0; j < k; ++j) g += z[j] * z[j] / ((d[j] - dt) - 0.5 * delta);
    if (g >= 0.0) {
      o = t;
      a = 0.0;
      b = 0.5 * delta;
    } else {
      o = t + 1;
      a = -0.5 * delta;
      b = 0.0;
    }
  } else {
    o = t;
    double zz = 0.0;
    for (int j = 0; j < k; ++j) zz += z[j] * z[j];
    a = 0.0;
    b = rho * zz * (1.0 + 8.0 * kEps);  // the last root lies in (d_k, d_k + rho |z|^2]
  }
  const double dorig = d[o];
  double tau = 0.5 * (a + b);
  for (int it = 0; it < 100; ++it) {
    double psi = 0.0, dpsi = 0.0, phi = 0.0, dphi = 0.0;
    for (int j = 0; j < k; ++j) {
      const double diff = (d[j] - dorig) - tau;
      const double term = z[j] * z[j] / diff;
      if (j <= t) {
        psi += term;
        dpsi += term / diff;
      } else {
        phi += term;
        dphi += term / diff;
      }
    }
    const double g = rinv + psi + phi;
    const double err = 8.0 * (fabs(psi) + fabs(phi) + rinv) + fabs(tau) * (dpsi + dphi);
    if (g < 0.0) a = tau;
    else b = tau;
    if (fabs(g) <= kEps * err || (b - a) <= 2.0 * kEps * fmax(fabs(a), fabs(b))) break;
    const double dl = (d[t] - dorig) - tau;
    double eta;
    bool ok = true;
    if (t < k - 1) {
      const double dr = (d[t + 1] - dorig) - tau;
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
    tau = tn;
  }
  *o_out = o;
  *tau_out = tau;
}

// Forward pass for one cluster (whole workgroup).  In: d, e (T), G0 rows = tracked X with
// nx columns.  Out: lam ascending, G0 rows = Z^T X (columns 0..nx-1), records.
__device__ void dc_forward(int n, const double *__restrict__ dd, const double *__restrict__ ee, int nx, DcWs ws,
                           DevStatus *st, int cid) {
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int Fc = nx, Lc = nx + 1, nt = nx + 2;
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
    // Phase A: one thread per merge -- sort, normalise z, deflate
    for (int mi = tid; mi < nmerge; mi += nthr) {
      const int lo = mi * span, m = lo + size, hi = min(lo + span, n);
      if (m >= hi) {
        R.cnt[lo] = -1;
        continue;
      }
      const int k = hi - lo;
      const double beta = ee[m - 1];
      double rho = fabs(beta);
      const double sg = beta >= 0.0 ? 1.0 : -1.0;
      int i1 = lo, i2 = m;
      double zn2 = 0.0, dmaxabs = 0.0;
      for (int p = 0; p < k; ++p) {
        int take;
        if (i2 >= hi || (i1 < m && lam[i1] <= lam[i2])) take = i1++;
        else take = i2++;
        R.perm[lo + p] = take - lo;
        const double dv = lam[take];
        const double zv = take < m ? G0[(long long)take * kTrack + Lc] : sg * G0[(long long)take * kTrack + Fc];
        ws.Ds[lo + p] = dv;
        ws.zs[lo + p] = zv;
        zn2 += zv * zv;
        dmaxabs = fmax(dmaxabs, fabs(dv));
      }
      for (int r = lo; r < m; ++r) G0[(long long)r * kTrack + Lc] = 0.0;
      for (int r = m; r < hi; ++r) G0[(long long)r * kTrack + Fc] = 0.0;
      const double zinv = 1.0 / sqrt(zn2);
      double zmax = 0.0;
      for (int p = 0; p < k; ++p) {
        ws.zs[lo + p] *= zinv;
        zmax = fmax(zmax, fabs(ws.zs[lo + p]));
      }
      rho *= zn2;
      const double tol = 8.0 * kEps * fmax(dmaxabs, zmax);
      int kp = 0, nd = 0, nrot = 0, pj = -1;
      for (int j = 0; j < k; ++j) {
        const double zj = ws.zs[lo + j];
        if (rho * fabs(zj) <= tol) {
          R.kpos[hi - 1 - nd] = j;
          ++nd;
          continue;
        }
        if (pj < 0) {
          pj = j;
          continue;
        }
        double s_ = ws.zs[lo + pj], c_ = zj;
        const double tau = hypot(c_, s_);
        const double tdiff = ws.Ds[lo + j] - ws.Ds[lo + pj];
        c_ /= tau;
        s_ = -s_ / tau;
        if (fabs(tdiff * c_ * s_) <= tol) {
          ws.zs[lo + j] = tau;
          ws.zs[lo + pj] = 0.0;
          R.ra[lo + nrot] = pj;
          R.rb[lo + nrot] = j;
          R.rc[lo + nrot] = c_;
          R.rs[lo + nrot] = s_;
          ++nrot;
          const double dp = ws.Ds[lo + pj], dj = ws.Ds[lo + j];
          const double t1 = dp * c_ * c_ + dj * s_ * s_;
          ws.Ds[lo + j] = dp * s_ * s_ + dj * c_ * c_;
          ws.Ds[lo + pj] = t1;
          R.kpos[hi - 1 - nd] = pj;
          ++nd;
        } else {
          R.kpos[lo + kp] = pj;
          ++kp;
        }
        pj = j;
      }
      if (pj >= 0) {
        R.kpos[lo + kp] = pj;
        ++kp;
      }
      R.cnt[lo] = kp;
      R.cnt[lo + 1] = nrot;
      ws.rhov[lo] = rho;
      for (int t = 0; t < kp; ++t) {
        const int pos = R.kpos[lo + t];
        R.dK[lo + t] = ws.Ds[lo + pos];
        ws.zK[lo + t] = ws.zs[lo + pos];
      }
    }
    __syncthreads();
    // Phase A1: G1 = rows of G0 in sorted order
    for (long long e = tid; e < (long long)n * nt; e += nthr) {
      const int q = (int)(e / nt), cc = (int)(e % nt);
      const int lo = q - q % span;
      if (R.cnt[lo] < 0) continue;
      G1[(long long)q * kTrack + cc] = G0[(long long)(lo + R.perm[q]) * kTrack + cc];
    }
    __syncthreads();
    // Phase A2: deflation rotations, one thread per (merge, column)
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
    // Phase B: secular roots
    for (int q = tid; q < n; q += nthr) {
      const int lo = q - q % span;
      const int kp = R.cnt[lo];
      const int t = q - lo;
      if (kp < 0 || t >= kp) continue;
      int o;
      double tau;
      secular_root(R.dK + lo, ws.zK + lo, kp, ws.rhov[lo], t, &o, &tau);
      R.orig[lo + t] = o;
      R.tau[lo + t] = tau;
    }
    __syncthreads();
    // Phase C: Loewner z
    for (int q = tid; q < n; q += nthr) {
      const int lo = q - q % span;
      const int kp = R.cnt[lo];
      const int j = q - lo;
      if (kp < 0 || j >= kp) continue;
      const double *dK = R.dK + lo;
      const double dj = dK[j];
      const double rho = ws.rhov[lo];
      double prod = -((dj - dK[R.orig[lo + j]]) - R.tau[lo + j]) / rho;
      for (int i = 0; i < kp; ++i) {
        if (i == j) continue;
        const double num = (dj - dK[R.orig[lo + i]]) - R.tau[lo + i];
        prod *= num / (dj - dK[i]);
      }
      R.zt[lo + j] = copysign(sqrt(fmax(prod, 0.0)), ws.zK[lo + j]);
    }
    __syncthreads();
    // Phase D: eigenvector norms
    for (int q = tid; q < n; q += nthr) {
      const int lo = q - q % span;
      const int kp = R.cnt[lo];
      const int t = q - lo;
      if (kp < 0 || t >= kp) continue;
      const double *dK = R.dK + lo;
      const double dorig = dK[R.orig[lo + t]], tau = R.tau[lo + t];
      double s2 = 0.0;
      for (int j = 0; j < kp; ++j) {
        const double u = R.zt[lo + j] / ((dK[j] - dorig) - tau);
        s2 += u * u;
      }
      R.nrm[lo + t] = sqrt(s2);
    }
    __syncthreads();
    // Phase F: output order (ascending eigenvalue; ties by element index)
    for (int q = tid; q < n; q += nthr) {
      const int lo = q - q % span;
      const int kp = R.cnt[lo];
      if (kp < 0) continue;
      const int hi = min(lo + span, n), k = hi - lo;
      const int e = q - lo;
      auto val = [&](int x) -> double {
        return x < kp ? R.dK[lo + R.orig[lo + x]] + R.tau[lo + x] : ws.Ds[lo + R.kpos[lo + x]];
      };
      const double ve = val(e);
      int rank = 0;
      for (int x = 0; x < k; ++x) {
        const double vx = val(x);
        rank += (vx < ve) || (vx == ve && x < e);
      }
      R.oo[lo + rank] = e;
      lam[lo + rank] = ve;
    }
    __syncthreads();
    // Phase E: transformed rows, written in output order
    for (int q = tid; q < n; q += nthr) {
      const int lo = q - q % span;
      const int kp = R.cnt[lo];
      if (kp < 0) continue;
      const int e = R.oo[q];
      double acc[kTrack];
      if (e < kp) {
#pragma unroll
        for (int cc = 0; cc < kTrack; ++cc) acc[cc] = 0.0;
        const double *dK = R.dK + lo;
        const double dorig = dK[R.orig[lo + e]], tau = R.tau[lo + e];
        const double ninv = 1.0 / R.nrm[lo + e];
        for (int j = 0; j < kp; ++j) {
          const double u = R.zt[lo + j] / ((dK[j] - dorig) - tau) * ninv;
          const double *g = G1 + (long long)(lo + R.kpos[lo + j]) * kTrack;
#pragma unroll
          for (int cc = 0; cc < kTrack; ++cc)
            if (cc < nt) acc[cc] += u * g[cc];
        }
      } else {
        const double *g = G1 + (long long)(lo + R.kpos[lo + e]) * kTrack;
#pragma unroll
        for (int cc = 0; cc < kTrack; ++cc) acc[cc] = (cc < nt) ? g[cc] : 0.0;
      }
#pragma unroll
      for (int cc = 0; cc < kTrack; ++cc)
        if (cc < nt) G0[(long long)q * kTrack + cc] = acc[cc];
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(256) stedc_kernel(int n_clusters, const int *__restrict__ order,
                                                    double *__restrict__ vec, const long long *__restrict__ vec_off,
                                                    int *__restrict__ ivec, const long long *__restrict__ ivec_off,
                                                    const int *__restrict__ dmax, const int *__restrict__ dim,
                                                    const int *__restrict__ n_orb, DevStatus *st) {
  for (int s = blockIdx.x; s < n_clusters; s += gridDim.x) {
    const int c = order[s];
    const int n = dim[c];
    const int M = n_orb[c];
    double *cv = vec + vec_off[c];
    const VecLayout vl = VecLayout::make(dmax[c]);
    DcWs ws = dc_ws(cv, ivec + ivec_off[c], dmax[c]);
    __syncthreads();
    dc_forward(n, cv + vl.d, cv + vl.e, 2 * M, ws, st, c);
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
}

void launch_stedc(Plan &p) {
  hipLaunchKernelGGL(stedc_kernel, dim3(p.workgroups), dim3(kWG), 0, p.stream, p.n_atoms, p.d_order, p.d_vec,
                     p.d_vec_off, p.d_ivec, p.d_ivec_off, p.d_dmax, p.d_dim, p.d_n_orb, p.d_status);
}

}  // namespace ldc
