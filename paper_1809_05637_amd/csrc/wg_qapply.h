// Products with the orthogonal factors of the two-stage tridiagonalization, Q = Q1 Q2.
//
// Q1 (reduction to band form, b = kBand): H_0 H_1 ... H_{n-1-b}, H_k = I - tau_k v_k v_k^T,
// v_k(0:k+b) = 0, v_k(k+b) = 1, v_k(k+b+1:) stored in A(k+b+1:, k) (column-major, leading
// dimension n).  The reflectors come in panels of b, panel p = reflectors 32 p .. 32 p + 31,
// whose product is I - V T V^T (compact WY) with T upper triangular, stored row-major by the
// band reduction, one b x b block per panel.
#pragma once

#include "dev_common.h"
#include "wg_blas.h"

namespace ldc {

constexpr int kQ1Slots = (kMaxDimTri + 63) / 64;  // 16-row chunks of X per wave
constexpr int kQ1Lds = 2 * 4 * 512;                // two buffers of the four waves' partial Y

// 8-byte load and store through a raw buffer view: byte offset voff (per lane) + soff (wave-
// uniform); a load at or past the view's size reads zero and a store there is dropped.
__device__ inline double view_load(__amdgpu_buffer_rsrc_t v, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(v, (int)voff, (int)soff, 0));
}
__device__ inline void view_store(__amdgpu_buffer_rsrc_t v, double x, unsigned voff, unsigned soff) {
  using U2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(v, 0, 0, 0));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U2, x), v, (int)voff, (int)soff, 0);
}

// A pointer that is the same in every lane, moved to scalar registers.
template <typename T>
__device__ inline T *uniform_ptr(T *p) {
  const unsigned long long u = reinterpret_cast<unsigned long long>(p);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)u), hi = __builtin_amdgcn_readfirstlane((unsigned)(u >> 32));
  return reinterpret_cast<T *>(((unsigned long long)hi << 32) | lo);
}

// X (n rows, M <= 16 columns, row-major with row stride ldx) <- Q1 X (TRANS false) or Q1^T X
// (TRANS true) on the FP64 matrix cores, panel by panel (Q1: from the last, with T; Q1^T: from
// the first, with T^T):  Y = V^T X,  Y <- T Y (T^T Y),  X <- X - V Y.
// X stays in registers for the whole product: 16-row chunk c belongs to wave c mod 4 and is
// held in the result layout of v_mfma_f64_16x16x4 (register r of lane l: X(16 c + l/16 + 4 r,
// l % 16)).  The K steps of every product are ordered so that each operand already sits in
// the register the instruction takes: step r of V^T X runs over the chunk's rows l/16 + 4 r
// (its B operand is register r of the chunk), the steps of T Y and of V Y over the reflectors
// 16 h + l/16 + 4 r (B operand: register r of block h of Y).  Rows below 2 b + 32 p are not
// touched by panel p, and rows 0 .. b - 1 by none.  The reflectors are read from A straight
// into the A operands (buffer loads: a lane offset and a wave-uniform one), the next chunk's
// while the current one is multiplied; entries that are not stored (above and on the unit
// diagonal, past row n, past the last reflector) are formed only in the panel's first two
// chunks, the chunk that holds row n - 1 and a short last panel.  The waves' partial Y meet in
// LDS (two buffers, so one barrier per panel), and every wave forms T Y itself in the same
// order.  Whole workgroup (4 waves); lds: kQ1Lds doubles; ends with a barrier.
template <bool TRANS>
__device__ void wg_apply_q1(const double *__restrict__ A, int n, const double *__restrict__ Tq, double *X, int ldx,
                            int M, double *lds) {
  static_assert(kBand == 32 && kMaxOrb == 16, "panels of two 16-wide blocks, X one 16-wide block");
  // the arguments are wave-uniform (out of line they arrive in vector registers)
  A = global_ptr(uniform_ptr(A));
  Tq = global_ptr(uniform_ptr(Tq));
  X = global_ptr(uniform_ptr(X));
  lds = lds_ptr(lds);
  n = __builtin_amdgcn_readfirstlane(n);
  ldx = __builtin_amdgcn_readfirstlane(ldx);
  M = __builtin_amdgcn_readfirstlane(M);
  const int lane = threadIdx.x & 63, li = lane & 15, lg = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nref = n - kBand;
  if (nref <= 0) return;
  const int nch = (n + 15) >> 4, npan = (nref + 31) >> 5;
  const unsigned n8 = 8u * (unsigned)n;
  const __amdgpu_buffer_rsrc_t av = __builtin_amdgcn_make_buffer_rsrc(const_cast<double *>(A), (short)0, (int)(n8 * n), 0x00020000);
  const unsigned lx8 = 8u * (unsigned)ldx;
  const __amdgpu_buffer_rsrc_t xv = __builtin_amdgcn_make_buffer_rsrc(X, (short)0, (int)(lx8 * n), 0x00020000);
  // X rows past n read zero (view size), columns M.. are sent past the view
  const unsigned xo = li < M ? 8u * (unsigned)(ldx * lg + li) : 0x80000000u;
  ldc_double4 x[kQ1Slots];
#pragma unroll
  for (int j = 0; j < kQ1Slots; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) x[j][r] = view_load(xv, xo + 4u * lx8 * r, 16u * lx8 * (4 * j + wave));
  // lane offsets of the two operand layouts: V(row0 + lg + 4 r, 16 h + li) and
  // V(row0 + li, 16 h + lg + 4 r)
  const unsigned o1 = 8u * (unsigned)(li * n + lg), o2 = 8u * (unsigned)(lg * n + li);
  for (int pi = 0; pi < npan; ++pi) {
    const int p = TRANS ? pi : npan - 1 - pi;
    const int nbp = min(32, nref - 32 * p), cf = 2 * p + 2;
    const unsigned vb0 = 32u * p * n8;  // column 32 p
    // the wave's chunks of the panel, c = 4 j + wave in [cf, nch)
    const int jlo = (cf - wave + 3) >> 2, jhi = (nch - 1 - wave) >> 2;
    // entries of the operand blocks that are not stored: t is the row offset from the panel's
    // first row (32 p + b) minus the reflector index
    // (rl = rows of the chunk inside the matrix, made opaque so that the compares are formed
    // here rather than hoisted out of the panel loop for every chunk)
    auto mask1 = [&](double (&v)[8], int c) {
      if (c < cf + 2 || 16 * c + 16 > n || nbp < 32) {
        int rl = n - 16 * c;
        asm volatile("" : "+s"(rl));
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int t = 16 * (c - cf - h) + 4 * r + lg - li;
            const bool in = li + 16 * h < nbp;
            v[4 * h + r] = (in && t > 0 && lg + 4 * r < rl) ? v[4 * h + r] : ((in && t == 0) ? 1.0 : 0.0);
          }
      }
    };
    auto mask2 = [&](double (&v)[8], int c) {
      if (c < cf + 2 || 16 * c + 16 > n || nbp < 32) {
        int rl = n - 16 * c;
        asm volatile("" : "+s"(rl));
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int t = 16 * (c - cf - h) - 4 * r + li - lg;
            const bool in = lg + 4 * r + 16 * h < nbp;
            v[4 * h + r] = (in && t > 0 && li < rl) ? v[4 * h + r] : ((in && t == 0) ? 1.0 : 0.0);
          }
      }
    };
    auto load1 = [&](double (&v)[8], int c) {
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int r = 0; r < 4; ++r) v[4 * h + r] = view_load(av, o1 + 32u * r, vb0 + 16u * h * n8 + 128u * c);
    };
    auto load2 = [&](double (&v)[8], int c) {
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int r = 0; r < 4; ++r) v[4 * h + r] = view_load(av, o2, vb0 + (16u * h + 4u * r) * n8 + 128u * c);
    };
    // Y = V^T X, two 16-row blocks
    ldc_double4 y0 = {0.0, 0.0, 0.0, 0.0}, y1 = {0.0, 0.0, 0.0, 0.0};
    double va[8], vb[8] = {};
    if (jlo <= jhi) load1(va, 4 * jlo + wave);
#pragma unroll
    for (int j = 0; j < kQ1Slots; ++j) {
      if (j >= jlo && j <= jhi) {
        const int c = 4 * j + wave;
        if (j < jhi) load1(vb, c + 4);
        mask1(va, c);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          y0 = __builtin_amdgcn_mfma_f64_16x16x4f64(va[r], x[j][r], y0, 0, 0, 0);
          y1 = __builtin_amdgcn_mfma_f64_16x16x4f64(va[4 + r], x[j][r], y1, 0, 0, 0);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) va[u] = vb[u];
      }
    }
    // T operands of T Y: T(16 g + li, 16 h + lg + 4 r), the block g = 1, h = 0 zero; of T^T Y:
    // T(16 h + lg + 4 r, 16 g + li), the block g = 0, h = 1 zero
    const double *Tp = Tq + (long long)p * 1024;
    double ta[8], tb[8];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int k = 16 * h + lg + 4 * r;
        ta[4 * h + r] = TRANS ? (h == 0 ? Tp[k * 32 + li] : 0.0) : Tp[li * 32 + k];
        tb[4 * h + r] = TRANS ? Tp[k * 32 + 16 + li] : (h == 1 ? Tp[(16 + li) * 32 + k] : 0.0);
      }
    double *Yb = lds + (p & 1) * 2048;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      Yb[wave * 512 + r * 64 + lane] = y0[r];
      Yb[wave * 512 + (4 + r) * 64 + lane] = y1[r];
    }
    __syncthreads();
    // Y summed over the waves in a fixed order, then T Y (T^T Y): z0 = rows 0..15, z1 = rows 16..31
    ldc_double4 z0 = {0.0, 0.0, 0.0, 0.0}, z1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const double ys = ((Yb[u * 64 + lane] + Yb[512 + u * 64 + lane]) + Yb[1024 + u * 64 + lane]) + Yb[1536 + u * 64 + lane];
      if (!TRANS || u < 4) z0 = __builtin_amdgcn_mfma_f64_16x16x4f64(ta[u], ys, z0, 0, 0, 0);
      if (TRANS || u >= 4) z1 = __builtin_amdgcn_mfma_f64_16x16x4f64(tb[u], ys, z1, 0, 0, 0);
    }
    // X <- X - V (T Y)
    if (jlo <= jhi) load2(va, 4 * jlo + wave);
#pragma unroll
    for (int j = 0; j < kQ1Slots; ++j) {
      if (j >= jlo && j <= jhi) {
        const int c = 4 * j + wave;
        if (j < jhi) load2(vb, c + 4);
        mask2(va, c);
#pragma unroll
        for (int r = 0; r < 4; ++r) x[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(va[r], -z0[r], x[j], 0, 0, 0);
#pragma unroll
        for (int r = 0; r < 4; ++r) x[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(va[4 + r], -z1[r], x[j], 0, 0, 0);
#pragma unroll
        for (int u = 0; u < 8; ++u) va[u] = vb[u];
      }
    }
  }
  // rows past n and columns M.. are dropped by the view
#pragma unroll
  for (int j = 0; j < kQ1Slots; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) view_store(xv, x[j][r], xo + 4u * lx8 * r, 16u * lx8 * (4 * j + wave));
  __syncthreads();
}

// Q2, band to tridiagonal by bulge chasing: sweep s holds the reflectors of rows
// [s + 1 + j b, s + 1 + j b + len), len = min(b, n - r0), b = kBand, stored in column n - 1 - s
// of A above the diagonal at rows j b.. (tau first, then v(1:len)); the steps of one sweep act
// on disjoint rows, and Q2 = (sweep 0) (sweep 1) ... in that order.  The only global reads of a
// product with Q2 are the reflectors, one contiguous run per sweep (n - 1 - s doubles of column
// n - 1 - s of A from row 0), fetched two sweeps ahead into registers and parked in a triple
// buffer of LDS (3 P doubles, P = q2_lds_stride(n)) with kBand zeros past the end of every run,
// so every reflector, the last of a sweep too, runs over kBand rows with no clamping or masking.
constexpr int kQ2Run = (kMaxDimTri + kBand + kWG - 1) / kWG;  // run elements per thread

// stride of the parked runs: at least n + kBand entries, even (every run and every step's
// reflector start on a 16-byte boundary, so the reflector entries are read in pairs)
__host__ __device__ inline int q2_lds_stride(int n) { return (n + kBand + 1) & ~1; }

__device__ inline void q2_fetch_run(double *nx, const double *A, int n, int s, int tid, int nthr) {
  // run of sweep s (clamped unconditional loads; a sweep outside 0..n-3 reads its nearest)
  const int ss = max(0, min(s, n - 3)), len = n - 1 - ss;
  const double *src = A + (long long)(n - 1 - ss) * n;
#pragma unroll
  for (int u = 0; u < kQ2Run; ++u) nx[u] = src[min(tid + u * nthr, len - 1)];
}

// Q2 X (FWD false) or Q2^T X (FWD true) with X held in registers: X (n >= 3 rows, nc <= 16
// columns, row-major with row stride ldx) in memory, the reflector runs parked in LDS (runs:
// 3 P doubles), ex: 2 x 32 x 16 doubles of LDS.  At sweep s the rows
// s + 1 .. of X are held in windows of 32 rows, window j = rows s + 1 + 32 j .. s + 32 j + 32
// (rows past n zero), window j in lane q of group j mod 16 (two windows per lane, j and j + 16).
// Step j of sweep s acts on exactly window j, so a sweep reads its reflector entries from LDS
// and touches no other memory.  Between sweeps every window moves by one row, and one row
// passes from each window to its neighbour through ex (double-buffered by sweep parity): Q2^T
// runs the sweeps forwards and the windows move down (window 0's first row is then final and
// goes back to X), Q2 runs them backwards and the windows move up (window 0 takes row s + 1 of
// X, which no later sweep has touched, fetched a sweep ahead).  At the end the windows go back
// to X (row 0 is not touched).  One barrier per sweep.  Whole workgroup (256 threads); ends with
// a barrier.
template <bool FWD>
__device__ void wg_apply_q2_regs(const double *__restrict__ A, int n, double *X, int ldx, int nc, double *runs,
                                 double *ex) {
  constexpr int b = kBand;
  // the arguments are wave-uniform (out of line they arrive in vector registers)
  A = global_ptr(uniform_ptr(A));
  X = global_ptr(uniform_ptr(X));
  runs = lds_ptr(runs);
  ex = lds_ptr(ex);
  n = __builtin_amdgcn_readfirstlane(n);
  ldx = __builtin_amdgcn_readfirstlane(ldx);
  nc = __builtin_amdgcn_readfirstlane(nc);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int grp = tid >> 4, q = tid & 15;
  const int P = q2_lds_stride(n);
  const int nsw = n - 2;  // sweeps 0 .. n-3
  auto sweep = [&](int it) { return max(0, min(FWD ? it : nsw - 1 - it, n - 3)); };
  auto park = [&](double *dst, const double *nx, int it) {
    const int nlen = n - 1 - sweep(it);
#pragma unroll
    for (int u = 0; u < kQ2Run; ++u) {
      const int e = tid + u * nthr;
      if (e < nlen + b) dst[e] = e < nlen ? nx[u] : 0.0;
    }
  };
  double *xc = X + min(q, nc - 1);
  const bool wr = q < nc;
  // the windows at the first sweep
  const int s0 = sweep(0);
  double xw[2][b];
#pragma unroll
  for (int w = 0; w < 2; ++w)
#pragma unroll
    for (int i = 0; i < b; ++i) {
      const int row = s0 + 1 + b * (grp + 16 * w) + i;
      const double v = xc[(long long)min(row, n - 1) * ldx];
      xw[w][i] = row < n ? v : 0.0;
    }
  double nx0[kQ2Run], nx1[kQ2Run];
  q2_fetch_run(nx0, A, n, sweep(0), tid, nthr);
  q2_fetch_run(nx1, A, n, sweep(1), tid, nthr);
  park(runs, nx0, 0);
  // backwards: row s + 1 of X for the next sweep's window 0
  double top = FWD ? 0.0 : xc[(long long)(sweep(1) + 1) * ldx];
  __syncthreads();
  for (int it = 0; it < nsw; ++it) {
    const int s = sweep(it);
    q2_fetch_run(nx0, A, n, sweep(it + 2), tid, nthr);
    if (it > 0) {
      const double *exr = ex + ((it - 1) & 1) * (2 * 16 * 16);
#pragma unroll
      for (int w = 0; w < 2; ++w) {
        const int j = grp + 16 * w;
        if (FWD) {
          // down by one row: the first row leaves (window 0's is final: row s), the next
          // window's first row arrives
          if (j == 0 && wr) X[(long long)s * ldx + q] = xw[w][0];
          const double in = j == 31 ? 0.0 : exr[(j + 1) * 16 + q];
#pragma unroll
          for (int i = 0; i < b - 1; ++i) xw[w][i] = xw[w][i + 1];
          xw[w][b - 1] = in;
        } else {
          // up by one row: the previous window's last row arrives (window 0: row s + 1 of X)
          const double in = j == 0 ? top : exr[(j - 1) * 16 + q];
#pragma unroll
          for (int i = b - 1; i > 0; --i) xw[w][i] = xw[w][i - 1];
          xw[w][0] = in;
        }
      }
      if (!FWD) top = xc[(long long)(sweep(it + 1) + 1) * ldx];
    }
    const double *cur = runs + (it % 3) * P;
    const int nst = (n - 3 - s) / b + 1;
#pragma unroll
    for (int w = 0; w < 2; ++w) {
      const int j = grp + 16 * w;
      if (j < nst) {
        typedef __attribute__((ext_vector_type(2))) double dpair;
        const dpair *vp = reinterpret_cast<const dpair *>(cur + j * b);
        double vv[b];
#pragma unroll
        for (int i = 0; i < b / 2; ++i) {
          const dpair t = vp[i];
          vv[2 * i] = t.x;
          vv[2 * i + 1] = t.y;
        }
        const double tau = vv[0];
        vv[0] = 1.0;
        double d4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int i = 0; i < b; ++i) d4[i & 3] += vv[i] * xw[w][i];
        const double d = ((d4[0] + d4[1]) + (d4[2] + d4[3])) * tau;
#pragma unroll
        for (int i = 0; i < b; ++i) xw[w][i] -= d * vv[i];
      }
    }
    // the row every window passes to its neighbour at the next sweep
    double *exw = ex + (it & 1) * (2 * 16 * 16);
#pragma unroll
    for (int w = 0; w < 2; ++w) exw[(grp + 16 * w) * 16 + q] = FWD ? xw[w][0] : xw[w][b - 1];
    park(runs + ((it + 1) % 3) * P, nx1, it + 1);
#pragma unroll
    for (int u = 0; u < kQ2Run; ++u) nx1[u] = nx0[u];
    __syncthreads();
  }
  // the windows of the last sweep
  const int sl = sweep(nsw - 1);
  if (wr) {
#pragma unroll
    for (int w = 0; w < 2; ++w)
#pragma unroll
      for (int i = 0; i < b; ++i) {
        const int row = sl + 1 + b * (grp + 16 * w) + i;
        if (row < n) X[(long long)row * ldx + q] = xw[w][i];
      }
  }
  __syncthreads();
}

}  // namespace ldc
