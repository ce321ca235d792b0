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

#include <type_traits>

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
    for (int j = 0; j < k; ++j) g += z[j] * z[j] * rcp_nr((d[j] - dt) - 0.5 * delta);
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
  // sum of z_j^2 / (d_j - lambda) and of its derivative over [j0, j1), four independent
  // partial sums (the terms' latency chains overlap)
  auto sums = [&](int j0, int j1, double &sv, double &dv) {
    double s4[4] = {0.0, 0.0, 0.0, 0.0}, d4[4] = {0.0, 0.0, 0.0, 0.0};
    int j = j0;
    for (; j + 4 <= j1; j += 4) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double r = rcp_nr((d[j + u] - dorig) - tau);
        const double term = z[j + u] * z[j + u] * r;
        s4[u] += term;
        d4[u] += term * r;
      }
    }
    for (; j < j1; ++j) {
      const double r = rcp_nr((d[j] - dorig) - tau);
      const double term = z[j] * z[j] * r;
      s4[0] += term;
      d4[0] += term * r;
    }
    sv = (s4[0] + s4[1]) + (s4[2] + s4[3]);
    dv = (d4[0] + d4[1]) + (d4[2] + d4[3]);
  };
  for (int it = 0; it < 100; ++it) {
    double psi, dpsi, phi, dphi;
    sums(0, t + 1, psi, dpsi);
    sums(t + 1, k, phi, dphi);
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

// Total order on doubles (IEEE order for numbers; NaNs at the ends): sorting and ranking by
// this key gives a permutation whatever the data.
__device__ inline long long dc_key(double x) {
  const long long b = __double_as_longlong(x);
  return b >= 0 ? b : (b ^ 0x7fffffffffffffffLL);
}

// LDS copies of the current level's merge data (n entries each), read many times by the
// secular solver, the Loewner formula, the norms, the output ranking and the row transform.
struct DcLds {
  double *d, *z, *zt, *tau, *nrm, *Ds, *g;
  int *orig, *kpos, *jinv;
  static constexpr int kBytesPerRow = 6 * sizeof(double) + 3 * sizeof(int);
  static constexpr int kChunk = 32;  // rows of G1 staged per step of the row transform
  static constexpr int kFixedBytes = kChunk * kTrack * sizeof(double);
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
  L.g = b + 6 * nmax;  // kChunk x kTrack
  L.orig = reinterpret_cast<int *>(b + 6 * nmax + DcLds::kChunk * kTrack);
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
    // Phase A2: one thread per merge -- normalise z, deflate (sequential chain on LDS data)
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
      int kp = 0, nd = 0, nrot = 0, pj = -1;
      for (int j = 0; j < k; ++j) {
        const double zj = zs[j];
        if (rho * fabs(zj) <= tol) {
          R.kpos[hi - 1 - nd] = j;
          S.kpos[hi - 1 - nd] = j;
          ++nd;
          continue;
        }
        if (pj < 0) {
          pj = j;
          continue;
        }
        double s_ = zs[pj], c_ = zj;
        const double tau = hypot(c_, s_);
        const double tdiff = Ds[j] - Ds[pj];
        c_ /= tau;
        s_ = -s_ / tau;
        if (fabs(tdiff * c_ * s_) <= tol) {
          zs[j] = tau;
          zs[pj] = 0.0;
          R.ra[lo + nrot] = pj;
          R.rb[lo + nrot] = j;
          R.rc[lo + nrot] = c_;
          R.rs[lo + nrot] = s_;
          ++nrot;
          const double dp = Ds[pj], dj = Ds[j];
          const double t1 = dp * c_ * c_ + dj * s_ * s_;
          Ds[j] = dp * s_ * s_ + dj * c_ * c_;
          Ds[pj] = t1;
          R.kpos[hi - 1 - nd] = pj;
          S.kpos[hi - 1 - nd] = pj;
          ++nd;
        } else {
          R.kpos[lo + kp] = pj;
          S.kpos[lo + kp] = pj;
          ++kp;
        }
        pj = j;
      }
      if (pj >= 0) {
        R.kpos[lo + kp] = pj;
        S.kpos[lo + kp] = pj;
        ++kp;
      }
      R.cnt[lo] = kp;
      R.cnt[lo + 1] = nrot;
      ws.rhov[lo] = rho;
      for (int t = 0; t < kp; ++t) {
        const int pos = S.kpos[lo + t];
        const double dv = Ds[pos], zv = zs[pos];
        R.dK[lo + t] = dv;
        S.d[lo + t] = dv;
        S.z[lo + t] = zv;
      }
      for (int t = 0; t < k; ++t) S.jinv[lo + S.kpos[lo + t]] = t;
    }
    __syncthreads();
    // Phase A3: G1 = rows of G0 in sorted order
    for (long long e = tid; e < (long long)n * nt; e += nthr) {
      const int q = (int)(e / nt), cc = (int)(e % nt);
      const int lo = q - q % span;
      if (R.cnt[lo] < 0) continue;
      G1[(long long)q * kTrack + cc] = G0[(long long)(lo + R.perm[q]) * kTrack + cc];
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
    // Phase B: secular roots
    for (int q = tid; q < n; q += nthr) {
      const int lo = q - q % span;
      const int kp = R.cnt[lo];
      const int t = q - lo;
      if (kp < 0 || t >= kp) continue;
      int o;
      double tau;
      secular_root(S.d + lo, S.z + lo, kp, ws.rhov[lo], t, &o, &tau);
      R.orig[lo + t] = o;
      R.tau[lo + t] = tau;
      S.orig[lo + t] = o;
      S.tau[lo + t] = tau;
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
      double prod = -((dj - dK[org[j]]) - tu[j]) / rho;
      for (int i = 0; i < kp; ++i) {
        if (i == j) continue;
        const double num = (dj - dK[org[i]]) - tu[i];
        prod *= num * rcp_nr(dj - dK[i]);
      }
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
      double s2 = 0.0;
      for (int j = 0; j < kp; ++j) {
        const double u = zt[j] * rcp_nr((dK[j] - dorig) - tau);
        s2 += u * u;
      }
      const double nv = sqrt(s2);
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
    for (int q = tid; q < n; q += nthr) {
      const int lo = q - q % span;
      const int kp = R.cnt[lo];
      if (kp < 0) continue;
      const int hi = min(lo + span, n);
      const int e = q - lo;
      const double ve = S.z[q];
      const long long ke = dc_key(ve);
      int rank = 0;
      for (int x = lo; x < hi; ++x) {
        const long long kx = dc_key(S.z[x]);
        rank += (kx < ke) || (kx == ke && x < q);
      }
      R.oo[lo + rank] = e;
      lam[lo + rank] = ve;
    }
    __syncthreads();
    // Phase E: transformed rows, written in output order.  Output row q (merge [lo, lo+k),
    // element e = oo[q]) is sum_j u(e, j) G1(lo + kpos[j]) over the kept j (e < kp), or its own
    // row G1(lo + kpos[e]) (deflated e).  One output row per thread and pass; G1 is staged
    // through LDS kChunk rows at a time.  A staged row p carries its pole and Loewner z in
    // S.Ds[p] and S.z[p] (the merge data of row p's j = jinv[p]; a deflated row has z = 0 and a
    // far pole, so its weight is exactly zero), so the threads of one merge read the same LDS
    // entries in step (broadcast) and, when merges span whole chunks, run a fixed 32-row loop.
    for (int pp = tid; pp < n; pp += nthr) {
      const int lo = pp - pp % span;
      const int kp = R.cnt[lo];
      if (kp < 0) continue;
      const int j = S.jinv[pp];
      const bool kj = j < kp;
      S.Ds[pp] = kj ? S.d[lo + j] : 1e300;
      S.z[pp] = kj ? S.zt[lo + j] : 0.0;
    }
    // the columns are summed unguarded up to a compile-time count NT >= nt (entries past nt are
    // never stored): a guard per column would serialize the LDS reads
    auto transform = [&](auto ntc) {
      constexpr int NT = decltype(ntc)::value;
      for (int qb = 0; qb < n; qb += nthr) {
        constexpr int CH = DcLds::kChunk;
        const int q = qb + tid;
        int lo = 0, hi = 0, kp = -1, e = 0;
        double dorig = 0.0, tau = 0.0, ninv = 0.0;
        if (q < n) {
          lo = q - q % span;
          hi = min(lo + span, n);
          kp = R.cnt[lo];
          if (kp >= 0) {
            e = R.oo[q];
            if (e < kp) {
              dorig = S.d[lo + S.orig[lo + e]];
              tau = S.tau[lo + e];
              ninv = 1.0 / S.nrm[lo + e];
            }
          }
        }
        const bool kept = q < n && kp >= 0 && e < kp;
        double acc[NT];
#pragma unroll
        for (int cc = 0; cc < NT; ++cc) acc[cc] = 0.0;
        // the rows any thread of this pass needs: [first merge start, last merge end)
        const int rlo = qb - qb % span, rhi = min(n, ((min(qb + nthr, n) - 1) / span + 1) * span);
        for (int c0 = rlo; c0 < rhi; c0 += CH) {
          __syncthreads();
          for (int t = tid; t < CH * nt; t += nthr) {
            const int r = t / nt, cc = t % nt;
            S.g[r * kTrack + cc] = (c0 + r < n) ? G1[(long long)(c0 + r) * kTrack + cc] : 0.0;
          }
          __syncthreads();
          if (!kept || c0 + CH <= lo || c0 >= hi) continue;
          if (span >= CH) {
            // the chunk lies inside this merge (merges start at multiples of span >= CH); rows
            // past the end of the matrix are masked
#pragma unroll 4
            for (int r = 0; r < CH; ++r) {
              const int pp = min(c0 + r, n - 1);
              const double w0 = S.z[pp] * rcp_nr((S.Ds[pp] - dorig) - tau) * ninv;
              const double w = (c0 + r < hi) ? w0 : 0.0;
              const double *g = S.g + r * kTrack;
#pragma unroll
              for (int cc = 0; cc < NT; ++cc) acc[cc] += w * g[cc];
            }
          } else {
            const int pa = max(c0, lo), pb = min(c0 + CH, hi);
            for (int pp = pa; pp < pb; ++pp) {
              const double w = S.z[pp] * rcp_nr((S.Ds[pp] - dorig) - tau) * ninv;
              const double *g = S.g + (pp - c0) * kTrack;
#pragma unroll
              for (int cc = 0; cc < NT; ++cc) acc[cc] += w * g[cc];
            }
          }
        }
        if (q < n && kp >= 0) {
          if (!kept) {
            const double *g = G1 + (long long)(lo + S.kpos[lo + e]) * kTrack;
#pragma unroll
            for (int cc = 0; cc < NT; ++cc)
              if (cc < nt) acc[cc] = g[cc];
          }
#pragma unroll
          for (int cc = 0; cc < NT; ++cc)
            if (cc < nt) G0[(long long)q * kTrack + cc] = acc[cc];
        }
      }
    };
    if (nt <= 20) transform(std::integral_constant<int, 20>{});
    else transform(std::integral_constant<int, kTrack>{});
    __syncthreads();
  }
}

__global__ void __launch_bounds__(256, 3) stedc_kernel(int n_clusters, const int *__restrict__ order,
                                                    double *__restrict__ vec, const long long *__restrict__ vec_off,
                                                    int *__restrict__ ivec, const long long *__restrict__ ivec_off,
                                                    const int *__restrict__ dmax, const int *__restrict__ dim,
                                                    const int *__restrict__ n_orb, DevStatus *st, int nmax) {
  extern __shared__ double dsh[];
  const DcLds S = dc_lds(dsh, nmax);
  for (int s = blockIdx.x; s < n_clusters; s += gridDim.x) {
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
}

void launch_stedc(Plan &p) {
  const int dm = cur_dim(p);
  const size_t lds = (size_t)dm * DcLds::kBytesPerRow + DcLds::kFixedBytes;
  // above 64 KB (clusters of more than about 940 rows) the dynamic LDS limit must be raised
  if (lds > 64 * 1024)
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(stedc_kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
  // default three workgroups per CU (at most 168 VGPRs; the LDS of a 711-row cluster is 51 KB):
  // more waves in flight for the latency-bound merges
  const int n = cur_count(p);
  const int grid = std::max(1, std::min(stage_grid(p, kTStedc, 3 * p.n_cu), n));
  hipLaunchKernelGGL(stedc_kernel, dim3(grid), dim3(kWG), lds, p.stream, n, cur_order(p), p.d_vec, p.d_vec_off,
                     p.d_ivec, p.d_ivec_off, p.d_dmax, p.d_dim, p.d_n_orb, p.d_status, dm);
}

}  // namespace ldc
