// Records and the product Z y of the divide-and-conquer tridiagonal eigensolver (shared
// by the forward pass and the density step).
#pragma once

#include "dev_common.h"
#include "wg_blas.h"

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

// The row sums of the merge product for merges of 64 rows or more, on the FP64 matrix cores.
// Each wave takes 64 output rows j of one merge as four 16-row tiles; K step s covers the roots
// t = lo + 4 s + l/16: lane l forms the weight u(j, t) = zt_j / (((d_j - d_orig(t)) - tau_t)
// nrm_t) of row j = q0 + 16 c + l % 16 of every tile c (the A operands) and reads column l % 16
// of y_t from memory (the B operand), so the waves need no barrier; register r of tile c's
// result then holds row q0 + 16 c + l/16 + 4 r.  Weights of rows that are not kept, and of
// roots past the last, are zero (selected, not multiplied); columns ny.. of y only reach columns
// that are not stored.  Rows j >= kp are copies of their own y row, blocks that are not merged
// (cnt < 0) copies in place.  Out of line (its registers apart from the kernel's); the LDS
// arrays hold the level's secular data as staged by the caller.
__device__ __noinline__ void dc_apply_rows_mfma(int n, int span, int ny, const int *__restrict__ cnt,
                                                const int *__restrict__ kpos, const double *sdK_, const double *szt_,
                                                const double *stau_, const double *snrm_, const int *sorig_,
                                                const double *__restrict__ yb, double *__restrict__ ya) {
  n = __builtin_amdgcn_readfirstlane(n);
  span = __builtin_amdgcn_readfirstlane(span);
  ny = __builtin_amdgcn_readfirstlane(ny);
  cnt = global_ptr(cnt);
  kpos = global_ptr(kpos);
  yb = global_ptr(yb);
  ya = global_ptr(ya);
  // the secular data lives in LDS: address it as such (out of line the pointers are generic)
  typedef __attribute__((address_space(3))) const double lds_double;
  typedef __attribute__((address_space(3))) const int lds_int;
  lds_double *sdK = (lds_double *)sdK_, *szt = (lds_double *)szt_, *stau = (lds_double *)stau_,
             *snrm = (lds_double *)snrm_;
  lds_int *sorig = (lds_int *)sorig_;
  const int lane = threadIdx.x & 63, li = lane & 15, lg = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (int q0 = 64 * wave; q0 < n; q0 += 256) {
    const int lo = q0 & ~(span - 1);
    const int kp = cnt[lo];
    const int q = q0 + lane;
    if (kp < 0) {
      if (q < n)
        for (int cc = 0; cc < ny; ++cc) ya[(long long)q * kMaxOrb + cc] = yb[(long long)q * kMaxOrb + cc];
      continue;
    }
    double dj[4], zj[4];
    bool kj[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int j = q0 + 16 * c + li;
      kj[c] = j < n && j - lo < kp;
      dj[c] = kj[c] ? sdK[j] : 0.0;
      zj[c] = kj[c] ? szt[j] : 0.0;
    }
    ldc_double4 acc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = ldc_double4{0.0, 0.0, 0.0, 0.0};
    const int tend = lo + kp;
    for (int t0 = lo; t0 < tend; t0 += 4) {
      const int t = t0 + lg;
      const bool in = t < tend;
      const int tc = in ? t : tend - 1;
      const double dor = sdK[lo + sorig[tc]], ta = stau[tc], nr = snrm[tc];
      const double yv = yb[(long long)tc * kMaxOrb + li];
      double x[4], r[4], e[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) x[c] = ((dj[c] - dor) - ta) * nr;
#pragma unroll
      for (int c = 0; c < 4; ++c) r[c] = __builtin_amdgcn_rcp(x[c]);
#pragma unroll
      for (int c = 0; c < 4; ++c) e[c] = fma(-x[c], r[c], 1.0);
#pragma unroll
      for (int c = 0; c < 4; ++c) r[c] = fma(r[c], e[c], r[c]);
#pragma unroll
      for (int c = 0; c < 4; ++c) e[c] = fma(-x[c], r[c], 1.0);
#pragma unroll
      for (int c = 0; c < 4; ++c) r[c] = fma(r[c], e[c], r[c]);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const double w = (in && kj[c]) ? zj[c] * r[c] : 0.0;
        acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(w, yv, acc[c], 0, 0, 0);
      }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int j = q0 + 16 * c + lg + 4 * rr;
        if (j < n && j - lo < kp && li < ny) ya[(long long)(lo + kpos[j]) * kMaxOrb + li] = acc[c][rr];
      }
    if (q < n && q - lo >= kp) {
      const int pos = kpos[q];
      for (int cc = 0; cc < ny; ++cc) ya[(long long)(lo + pos) * kMaxOrb + cc] = yb[(long long)q * kMaxOrb + cc];
    }
  }
}

// y (n rows, ny columns, row stride kMaxOrb) in final eigenvalue order -> Z y in the
// tridiagonal index order.  ya/yb: ping-pong buffers; the result ends in the returned one.
// lds: at least 4.5 n doubles: a level's secular data (poles, z, roots, norms, origins) is
// staged there, so the row sums read it from LDS.
__device__ inline int dc_apply_lds_doubles(int n) { return 4 * n + (n + 1) / 2; }

template <int NC>
__device__ inline double *dc_apply_nc(int n, int ny, DcWs ws, double *ya, double *yb, double *lds) {
  const int tid = threadIdx.x, nthr = blockDim.x;
  double *sdK = lds, *szt = lds + n, *stau = lds + 2 * n, *snrm = lds + 3 * n;
  int *sorig = reinterpret_cast<int *>(lds + 4 * n);
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
    // threads of a merge load the same row together).  Larger merges: on the matrix cores.
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
      dc_apply_rows_mfma(n, span, ny, R.cnt, R.kpos, sdK, szt, stau, snrm, sorig, yb, ya);
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
