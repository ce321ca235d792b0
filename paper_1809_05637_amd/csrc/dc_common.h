// Records and the product Z y of the divide-and-conquer tridiagonal eigensolver (shared
// by the forward pass and the density step).
#pragma once

#include "dev_common.h"

namespace ldc {

struct DcRec {
  // per-level base pointers (length n each)
  double *rc, *rs, *dK, *zt, *tau, *nrm;
  int *perm, *kpos, *oo, *ra, *rb, *orig, *cnt;
};

__device__ inline DcRec dc_rec(double *dcd, int *dci, int n, int l) {
  DcRec r;
  double *b = dcd + 6LL * n * l;
  r.rc = b;
  r.rs = b + n;
  r.dK = b + 2 * n;
  r.zt = b + 3 * n;
  r.tau = b + 4 * n;
  r.nrm = b + 5 * n;
  int *ib = dci + 7LL * n * l;
  r.perm = ib;
  r.kpos = ib + n;
  r.oo = ib + 2 * n;
  r.ra = ib + 3 * n;
  r.rb = ib + 4 * n;
  r.orig = ib + 5 * n;
  r.cnt = ib + 6 * n;
  return r;
}

// Workspace of the tridiagonal solver inside a cluster's vector region.
struct DcWs {
  double *lam, *G0, *G1, *Ds, *zs, *zK, *rhov, *dcd;
  int *dci;
};

__device__ inline DcWs dc_ws(double *cv, int *ci, int nb) {
  const VecLayout vl = VecLayout::make(nb);
  DcWs w;
  w.lam = cv + vl.lam;
  w.G0 = cv + vl.G0;
  w.G1 = cv + vl.G1;
  w.Ds = cv + vl.y0;
  w.zs = cv + vl.y0 + nb;
  w.zK = cv + vl.y0 + 2 * nb;
  w.rhov = cv + vl.y0 + 3 * nb;
  w.dcd = cv + vl.dc;
  w.dci = ci;
  return w;
}

// Row q of x (ny <= NC columns, row stride kMaxOrb) to row lo + idx[q] of y, lo the start of
// q's merge (merges of span rows); rows of blocks that are not merged at this level
// (cnt < 0) stay in place.  One thread of the 256 per row: every index of the level is loaded at once,
// then every row, then the stores (two rounds of memory latency per level).
template <int NC>
__device__ inline void permute_rows(int n, int span, int ny, const int *__restrict__ idx, const double *x, double *y,
                                    const int *__restrict__ cnt) {
  constexpr int RPT = (kMaxDimTri + 255) / 256;
  int dst[RPT];
#pragma unroll
  for (int u = 0; u < RPT; ++u) {
    const int q = threadIdx.x + 256 * u;
    dst[u] = -1;
    if (q < n) {
      const int lo = q & ~(span - 1);
      const int c = cnt[lo], iq = idx[q];
      dst[u] = c < 0 ? q : lo + iq;
    }
  }
  double v[RPT][NC];
#pragma unroll
  for (int u = 0; u < RPT; ++u) {
    const double *xr = x + (long long)min((int)threadIdx.x + 256 * u, n - 1) * kMaxOrb;
#pragma unroll
    for (int cc = 0; cc < NC; ++cc) v[u][cc] = xr[cc];
  }
#pragma unroll
  for (int u = 0; u < RPT; ++u)
    if (dst[u] >= 0) {
#pragma unroll
      for (int cc = 0; cc < NC; ++cc)
        if (cc < ny) y[(long long)dst[u] * kMaxOrb + cc] = v[u][cc];
    }
}

// y (n rows, ny columns, row stride kMaxOrb) in final eigenvalue order -> Z y in the
// tridiagonal index order.  ya/yb: ping-pong buffers; the result ends in the returned one.
// lds: at least 4.5 n + kApplyChunk * kMaxOrb doubles: a level's secular data (poles, z,
// roots, norms, origins) and a chunk of y rows are staged there, so the row sums read LDS.
constexpr int kApplyChunk = 32;
__device__ inline int dc_apply_lds_doubles(int n) { return 4 * n + (n + 1) / 2 + kApplyChunk * kMaxOrb; }

template <int NC>
__device__ inline double *dc_apply_nc(int n, int ny, DcWs ws, double *ya, double *yb, double *lds) {
  const int tid = threadIdx.x, nthr = blockDim.x;
  double *sdK = lds, *szt = lds + n, *stau = lds + 2 * n, *snrm = lds + 3 * n;
  int *sorig = reinterpret_cast<int *>(lds + 4 * n);
  double *sy = lds + 4 * n + (n + 1) / 2;  // kApplyChunk x kMaxOrb
  int L = 0;
  while ((1 << L) < n) ++L;
  for (int l = L - 1; l >= 0; --l) {
    const int size = 1 << l, span = 2 * size;
    const DcRec R = dc_rec(ws.dcd, ws.dci, n, l);
    const int nmerge = (n + span - 1) / span;
    // T1: output order -> element order; stage the level's secular data
    permute_rows<NC>(n, span, ny, R.oo, ya, yb, R.cnt);
    for (int q = tid; q < n; q += nthr) {
      const int lo = q - q % span;
      const int kp = R.cnt[lo];
      if (kp < 0 || q - lo >= kp) continue;
      sdK[q] = R.dK[q];
      szt[q] = R.zt[q];
      stau[q] = R.tau[q];
      snrm[q] = R.nrm[q];
      sorig[q] = R.orig[q];
    }
    __syncthreads();
    // T2: secular eigenvectors (and deflated identities) -> sorted-pole order.  Row j < kp of a
    // merge is sum_t zt_j / ((d_j - d_orig(t) - tau_t) nrm_t) y_t, summed over t in order.
    // Merges under 64 rows: one row per thread, the y rows read straight from memory (the
    // threads of a merge load the same row together).  Larger merges: the y rows come through
    // LDS kApplyChunk at a time (the threads of one merge read the same row: broadcast).
    if (span < 64) {
      for (int q = tid; q < n; q += nthr) {
        const int lo = q & ~(span - 1);
        const int kp = R.cnt[lo];
        const int j = q - lo;
        if (kp < 0) {
          for (int cc = 0; cc < ny; ++cc) ya[(long long)q * kMaxOrb + cc] = yb[(long long)q * kMaxOrb + cc];
          continue;
        }
        double acc[NC];
        if (j < kp) {
          const double dj = sdK[q], zj = szt[q];
#pragma unroll
          for (int cc = 0; cc < NC; ++cc) acc[cc] = 0.0;
#pragma unroll 2
          for (int t = lo; t < lo + kp; ++t) {
            const double u = zj * rcp_nr(((dj - sdK[lo + sorig[t]]) - stau[t]) * snrm[t]);
            const double *y = yb + (long long)t * kMaxOrb;
#pragma unroll
            for (int cc = 0; cc < NC; ++cc) acc[cc] += u * y[cc];
          }
        } else {
          const double *y = yb + (long long)q * kMaxOrb;
#pragma unroll
          for (int cc = 0; cc < NC; ++cc) acc[cc] = (cc < ny) ? y[cc] : 0.0;
        }
        const int pos = R.kpos[q];
#pragma unroll
        for (int cc = 0; cc < NC; ++cc)
          if (cc < ny) ya[(long long)(lo + pos) * kMaxOrb + cc] = acc[cc];
      }
    } else {
      for (int qb = 0; qb < n; qb += nthr) {
        const int q = qb + tid;
        int lo = 0, kp = -1, j = 0;
        double dj = 0.0, zj = 0.0;
        if (q < n) {
          lo = q - q % span;
          kp = R.cnt[lo];
          j = q - lo;
          if (kp >= 0 && j < kp) {
            dj = sdK[q];
            zj = szt[q];
          }
        }
        const bool kept = q < n && kp >= 0 && j < kp;
        double acc[NC];
#pragma unroll
        for (int cc = 0; cc < NC; ++cc) acc[cc] = 0.0;
        const int rlo = qb - qb % span, rhi = min(n, ((min(qb + nthr, n) - 1) / span + 1) * span);
        // each chunk of y rows is fetched into registers while the previous one is used
        constexpr int PER = (kApplyChunk * kMaxOrb + 255) / 256;
        double pre[PER];
        auto fetch_chunk = [&](int c0) {
#pragma unroll
          for (int u = 0; u < PER; ++u) {
            const int e = tid + u * nthr, r = e / ny, cc = e % ny;
            pre[u] = (e < kApplyChunk * ny && c0 + r < n) ? yb[(long long)(c0 + r) * kMaxOrb + cc] : 0.0;
          }
        };
        if (rlo < rhi) fetch_chunk(rlo);
        for (int c0 = rlo; c0 < rhi; c0 += kApplyChunk) {
          __syncthreads();
#pragma unroll
          for (int u = 0; u < PER; ++u) {
            const int e = tid + u * nthr;
            if (e < kApplyChunk * ny) sy[(e / ny) * kMaxOrb + e % ny] = pre[u];
          }
          __syncthreads();
          if (c0 + kApplyChunk < rhi) fetch_chunk(c0 + kApplyChunk);
          if (kept) {
            const int ta = max(c0, lo), tb = min(c0 + kApplyChunk, lo + kp);
            for (int t = ta; t < tb; ++t) {
              const double u = zj * rcp_nr(((dj - sdK[lo + sorig[t]]) - stau[t]) * snrm[t]);
              const double *y = sy + (t - c0) * kMaxOrb;
              // all NC columns, unguarded (a guard per column would serialize the LDS reads);
              // the entries past ny are never stored
#pragma unroll
              for (int cc = 0; cc < NC; ++cc) acc[cc] += u * y[cc];
            }
          }
        }
        if (q < n) {
          if (kp < 0) {
            for (int cc = 0; cc < ny; ++cc) ya[(long long)q * kMaxOrb + cc] = yb[(long long)q * kMaxOrb + cc];
          } else {
            if (!kept) {
              const double *y = yb + (long long)(lo + j) * kMaxOrb;
#pragma unroll
              for (int cc = 0; cc < NC; ++cc) acc[cc] = (cc < ny) ? y[cc] : 0.0;
            }
            const int pos = R.kpos[lo + j];
#pragma unroll
            for (int cc = 0; cc < NC; ++cc)
              if (cc < ny) ya[(long long)(lo + pos) * kMaxOrb + cc] = acc[cc];
          }
        }
      }
    }
    __syncthreads();
    // T3: deflation rotations, reverse order
    for (int e = tid; e < nmerge * ny; e += nthr) {
      const int mi = e / ny, cc = e % ny;
      const int lo = mi * span;
      if (R.cnt[lo] < 0) continue;
      const int nrot = R.cnt[lo + 1];
      for (int r = nrot - 1; r >= 0; --r) {
        const long long pa = (long long)(lo + R.ra[lo + r]) * kMaxOrb + cc;
        const long long pb = (long long)(lo + R.rb[lo + r]) * kMaxOrb + cc;
        const double c_ = R.rc[lo + r], s_ = R.rs[lo + r];
        const double a = ya[pa], b = ya[pb];
        ya[pa] = c_ * a - s_ * b;
        ya[pb] = s_ * a + c_ * b;
      }
    }
    __syncthreads();
    // T4: undo the sort
    permute_rows<NC>(n, span, ny, R.perm, ya, yb, R.cnt);
    __syncthreads();
    double *t = ya;
    ya = yb;
    yb = t;
  }
  return ya;
}

// NC >= ny columns in the row sums: 9 covers s, p and d shells (the 16-column form costs 1.9 ms
// more per build on the 3920-atom slab)
__device__ inline double *dc_apply(int n, int ny, DcWs ws, double *ya, double *yb, double *lds) {
  return ny <= 9 ? dc_apply_nc<9>(n, ny, ws, ya, yb, lds) : dc_apply_nc<kMaxOrb>(n, ny, ws, ya, yb, lds);
}

}  // namespace ldc
