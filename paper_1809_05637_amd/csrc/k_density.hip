// Common chemical potential and density rows (Sec. II.C (iv)-(v); Eq. 13, 16, 24, 27).
//
// N(mu) = g sum_i sum_mu f((eps_mu - mu)/kT) w_mu is evaluated by a grid of workgroups
// (one partial per workgroup, fixed cluster assignment) and combined in order by the last
// workgroup to finish, which also performs the bisection update, so every run takes the same
// decisions.  One launch advances the bisection by kMuLevels halvings: the grid evaluates N at
// every node of the next kMuLevels levels of the bisection tree (each node the midpoint the
// halving rule would form on that path), and the combine walks the tree.  The host enqueues a
// fixed number of launches; those after convergence return at once.
//
// Density rows of atom i: with C = L^{-T} Q Z the cluster eigenvectors,
//   rho^(i)(:, i) = C f C_i^T = L^{-T} Q Z (f o u),  u = Z^T Q^T L^{-1} E_i = C_i^T,
// so only the tracked u, the merge records (Z y), the stored reflectors (Q r) and the
// trailing rows of L (P = F_i placed last) are needed.
#include "dc_common.h"
#include "wg_qapply.h"

namespace ldc {

// dynamic LDS: the secular data of the product Z y, then the reflector runs and row exchange of
// Q2 r, then the partial products of Q1 r
constexpr int kDensityLds = std::max(4 * kMaxDimTri + (kMaxDimTri + 1) / 2, kQ1Lds);
// the Q2 product's three reflector runs and its row exchange fit the same area
static_assert(3 * ((kMaxDimTri + kBand + 1) & ~1) + 2 * 16 * 32 <= kDensityLds, "Q2 runs and exchange");

// Q2 r with the rows of r held in registers, kept out of line: inlined into the density kernel it
// raises the register pressure of the whole kernel and spills
__device__ __noinline__ void density_q2(const double *A, int n, double *r, int nc, double *runs, double *ex) {
  wg_apply_q2_regs<false>(A, n, r, kMaxOrb, nc, runs, ex);
}

// Q1 r, kept out of line for the same reason: it holds r in registers
__device__ __noinline__ void density_q1(const double *A, int n, const double *Tq, double *r, int M, double *lds) {
  wg_apply_q1<false>(A, n, Tq, r, kMaxOrb, M, lds);
}

// x(g, a) = sum_{t >= g} Linv(t, g) r(t, a) for the rows g in [b0, n) on the FP64 matrix cores
// (Linv column-major with leading dimension ld; r and x row-major with row stride kMaxOrb, M
// columns).  Wave w takes the 16-row output tiles g0 = b0 + 16 i, i = w, w + 4, ...; K step k
// covers the rows t = g0 + 4 k + l/16: lane l's A operand is Linv(t, g0 + l % 16) (zero for
// t < g or t >= n), its B operand r(t, l % 16) (zero for t >= n); register j of the result
// then holds x(g0 + l/16 + 4 j, l % 16).  Eight K steps per round, their loads issued together.
// Columns M.. of r only reach columns M.. of the result, which are not stored.  Kept out of line
// (inlined, it changes the register allocation of the merge product and slows it).
__device__ __noinline__ void density_lt(const double *__restrict__ L, int ld, int n, int b0, const double *__restrict__ r,
                                        double *__restrict__ x, int M) {
  // the arguments are wave-uniform (out of line they arrive in vector registers)
  L = global_ptr(uniform_ptr(L));
  r = global_ptr(uniform_ptr(r));
  x = global_ptr(uniform_ptr(x));
  ld = __builtin_amdgcn_readfirstlane(ld);
  n = __builtin_amdgcn_readfirstlane(n);
  b0 = __builtin_amdgcn_readfirstlane(b0);
  M = __builtin_amdgcn_readfirstlane(M);
  const int lane = threadIdx.x & 63, li = lane & 15, lg = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int ntile = (n - b0 + 15) >> 4;
  for (int i = wave; i < ntile; i += 4) {
    const int g0 = b0 + 16 * i, g = g0 + li;
    const double *lc = L + (long long)min(g, n - 1) * ld;
    ldc_double4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int t0 = g0; t0 < n; t0 += 32) {
      double av[8], bv[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int t = t0 + 4 * k + lg, tc = min(t, n - 1);
        av[k] = (t >= g && t < n) ? lc[tc] : 0.0;
        bv[k] = t < n ? r[(long long)tc * kMaxOrb + li] : 0.0;
      }
#pragma unroll
      for (int k = 0; k < 8; ++k) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[k], bv[k], acc, 0, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int gr = g0 + lg + 4 * j;
      if (gr < n && li < M) x[(long long)gr * kMaxOrb + li] = acc[j];
    }
  }
}

// state layout of Plan::d_mu
enum { MU_LO = 0, MU_HI, MU_DONE, MU_IT, MU_SUMW, MU_NE, MU_KT, MU_G, MU_MU, MU_BAD };

// the tree's node count and the per-workgroup partial stride (kMuLevels halvings per launch)
constexpr int kMuNodes = (1 << kMuLevels) - 1, kMuStride = 16;
static_assert(kMuNodes < kMuStride, "tree partials fit the stride");

// Combine of the per-workgroup partials in a fixed order (lane l adds partials l, l + 64, ...,
// then a fixed DPP tree) and the bisection update; one wavefront, every lane takes the same
// decisions and lane 0 writes the state.  Runs in the last workgroup of mu_step_kernel to
// finish; the partials are read with coherent loads after the device-scope fence that
// follows that workgroup's ticket.
__device__ void mu_combine(int mode, int nparts, double *__restrict__ state, const double *partial, DevStatus *st) {
  const int lane = threadIdx.x & 63;
  const volatile double *vp = partial;
  const double kT = state[MU_KT], g = state[MU_G], ne = state[MU_NE];
  double lo, hi;
  if (mode == 0) {
    double s = 0.0, mn = 1e300, mx = -1e300;
    for (int b = lane; b < nparts; b += 64) {
      s += vp[b * kMuStride + 2];
      mn = fmin(mn, vp[b * kMuStride + 0]);
      mx = fmax(mx, vp[b * kMuStride + 1]);
    }
    s = wave_sum(s);
    mn = -wave_max(-mn);
    mx = wave_max(mx);
    lo = mn - 40.0 * kT;
    hi = mx + 40.0 * kT;
    const bool bad = !(ne > 0.0 && ne < g * s);
    const double mid = 0.5 * (lo + hi);
    if (lane == 0) {
      state[MU_SUMW] = s;
      state[MU_IT] = 0.0;
      state[MU_DONE] = 0.0;
      state[MU_BAD] = 0.0;
      if (bad) {
        state[MU_BAD] = 1.0;
        state[MU_DONE] = 1.0;
        report(st, LDC_ERR_MU_BRACKET, -1);
      }
      state[MU_LO] = lo;
      state[MU_HI] = hi;
      state[MU_MU] = mid;
      if (hi - lo <= 4e-16 * fmax(1.0, fabs(mid))) state[MU_DONE] = 1.0;
    }
    return;
  }
  // N at every node of the evaluated tree, then kMuLevels halvings down it, each with the
  // stopping test
  double sn[kMuNodes];
#pragma unroll
  for (int k = 0; k < kMuNodes; ++k) sn[k] = 0.0;
  for (int b = lane; b < nparts; b += 64) {
#pragma unroll
    for (int k = 0; k < kMuNodes; ++k) sn[k] += vp[b * kMuStride + k];
  }
#pragma unroll
  for (int k = 0; k < kMuNodes; ++k) sn[k] = wave_sum(sn[k]);
  lo = state[MU_LO];
  hi = state[MU_HI];
  double it = state[MU_IT];
  bool done = false;
  int node = 0;
  for (int level = 0; level < kMuLevels; ++level) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kMuNodes; ++k) s = (k == node) ? sn[k] : s;
    const double mid = 0.5 * (lo + hi);
    if (g * s < ne) {
      lo = mid;
      node = 2 * node + 2;
    } else {
      hi = mid;
      node = 2 * node + 1;
    }
    it += 1.0;
    const double mid2 = 0.5 * (lo + hi);
    if (hi - lo <= 4e-16 * fmax(1.0, fabs(mid2)) || it >= 200.0) {
      done = true;
      break;
    }
  }
  if (lane == 0) {
    state[MU_IT] = it;
    if (done) state[MU_DONE] = 1.0;
    state[MU_LO] = lo;
    state[MU_HI] = hi;
    state[MU_MU] = 0.5 * (lo + hi);
  }
}

// One step of the bisection over all clusters (mode 1), or its set-up (mode 0: the spectrum's
// range and the total weight).  Every workgroup forms its partial sums over a fixed set of
// clusters; the last workgroup to finish (atomic ticket on counter, which it resets) combines
// them.  Once the state says done, a launch returns at once, so the host can enqueue a fixed
// number of steps (enough for the 200-halving limit) without waiting for the result.
__global__ void __launch_bounds__(256) mu_step_kernel(int mode, int n_clusters, const double *__restrict__ vec,
                                                      const long long *__restrict__ vec_off,
                                                      const int *__restrict__ dmax, const int *__restrict__ dim,
                                                      double *__restrict__ state, double *__restrict__ partial,
                                                      int *__restrict__ counter, DevStatus *st) {
  __shared__ double red[8];
  __shared__ int last;
  if (mode == 1 && state[MU_DONE] != 0.0) return;
  const double kT = state[MU_KT];
  if (mode == 0) {
    double a0 = 1e300, a1 = -1e300, a2 = 0.0;
    for (int c = blockIdx.x; c < n_clusters; c += gridDim.x) {
      const VecLayout vl = VecLayout::make(dmax[c]);
      const double *lam = vec + vec_off[c] + vl.lam;
      const double *w = vec + vec_off[c] + vl.w;
      const int n = dim[c];
      for (int i = threadIdx.x; i < n; i += blockDim.x) {
        a0 = fmin(a0, lam[i]);
        a1 = fmax(a1, lam[i]);
        a2 += w[i];
      }
    }
    const double s = block_sum(a2, red);
    const double mn = -block_max(-a0, red);
    const double mx = block_max(a1, red);
    if (threadIdx.x == 0) {
      partial[blockIdx.x * kMuStride + 0] = mn;
      partial[blockIdx.x * kMuStride + 1] = mx;
      partial[blockIdx.x * kMuStride + 2] = s;
    }
  } else {
    // the tree's nodes in heap order: node k covers (nl, nh), its children 2k + 1 (hi = mid)
    // and 2k + 2 (lo = mid), each evaluated at its midpoint
    double nl[kMuNodes], nh[kMuNodes], m[kMuNodes], acc[kMuNodes];
    nl[0] = state[MU_LO];
    nh[0] = state[MU_HI];
    m[0] = 0.5 * (nl[0] + nh[0]);
#pragma unroll
    for (int k = 1; k < kMuNodes; ++k) {
      const int p = (k - 1) / 2;
      nl[k] = (k == 2 * p + 1) ? nl[p] : m[p];
      nh[k] = (k == 2 * p + 1) ? m[p] : nh[p];
      m[k] = 0.5 * (nl[k] + nh[k]);
    }
#pragma unroll
    for (int k = 0; k < kMuNodes; ++k) acc[k] = 0.0;
    for (int c = blockIdx.x; c < n_clusters; c += gridDim.x) {
      const VecLayout vl = VecLayout::make(dmax[c]);
      const double *lam = vec + vec_off[c] + vl.lam;
      const double *w = vec + vec_off[c] + vl.w;
      const int n = dim[c];
      for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const double li = lam[i], wi = w[i];
#pragma unroll
        for (int k = 0; k < kMuNodes; ++k) acc[k] += fermi_fast((li - m[k]) / kT) * wi;
      }
    }
#pragma unroll
    for (int k = 0; k < kMuNodes; ++k) {
      const double s = block_sum(acc[k], red);
      if (threadIdx.x == 0) partial[blockIdx.x * kMuStride + k] = s;
    }
  }
  // ticket: the partial stores above are made visible before the increment
  __threadfence();
  if (threadIdx.x == 0) last = (atomicAdd(counter, 1) == (int)gridDim.x - 1);
  __syncthreads();
  if (!last) return;
  __threadfence();
  if (threadIdx.x < 64) {
    mu_combine(mode, gridDim.x, state, partial, st);
    if (threadIdx.x == 0) atomicExch(counter, 0);
  }
}

// Rows of every cluster at mu = state[MU_MU] with weights by mode: density rows (Eq. 24 with
// Eq. 27, weights f), energy density rows (Eq. 25 with Eq. 27, weights f eps), or windowed
// density rows for energy-window LNOs (Sec. II.B: the projector over another energy window,
// weights f((eps - w_hi)/w_kT) - f((eps - w_lo)/w_kT)).
__global__ void __launch_bounds__(256, 2) density_kernel(
    int mode, double w_lo, double w_hi, double w_kT, int n_clusters, const int *__restrict__ order, double *__restrict__ mat, const long long *__restrict__ mat_off,
    double *__restrict__ vec, const long long *__restrict__ vec_off, int *__restrict__ ivec,
    const long long *__restrict__ ivec_off, const int *__restrict__ dmax, const int *__restrict__ dim,
    const int *__restrict__ n_orb, const int *__restrict__ p_rows, const int *__restrict__ mem_ptr,
    const int *__restrict__ mem_atom, const int *__restrict__ fna_ptr, const int *__restrict__ fna_blk,
    const long long *__restrict__ blk_off, const double *__restrict__ state, const double *__restrict__ H,
    const double *__restrict__ S, double *__restrict__ Dout, double *__restrict__ partial, int max_dim, int *__restrict__ queue) {
  __shared__ double red[16 * 17];
  __shared__ double sred[8];
  __shared__ int foff[kMaxMembers + 1];
  // dynamic LDS (kDensityLds doubles): the merge product's secular data, then Q2's reflector
  // runs and row exchange, then Q1's partial products
  extern __shared__ __attribute__((aligned(16))) double qlds[];
  const int tid = threadIdx.x, nthr = blockDim.x;
  const double mu = state[MU_MU], kT = state[MU_KT];
  for (int s = queue_next(queue); s < n_clusters; s = queue_next(queue)) {
    const int c = order[s];
    const int n = dim[c], ld = n;
    const int M = n_orb[c];
    const int p = p_rows[c];
    double *cv = vec + vec_off[c];
    const VecLayout vl = VecLayout::make(dmax[c]);
    DcWs ws;
    ws.lam = cv + vl.lam;
    ws.G0 = cv + vl.G0;
    ws.G1 = cv + vl.G1;
    ws.Ds = ws.zs = ws.zK = ws.rhov = nullptr;
    ws.dcd = cv + vl.dc;
    ws.dci = ivec + ivec_off[c];
    const double *A = mat + mat_off[c];
    const double *L = A + (long long)dmax[c] * dmax[c];
    double *ya = cv + vl.y0, *yb = cv + vl.y1;
    __syncthreads();
    // y = w o u with the mode's weights w
    for (long long e = tid; e < (long long)n * M; e += nthr) {
      const int i = (int)(e / M), a = (int)(e % M);
      const double li = ws.lam[i];
      const double wt = mode == kRowsWindow ? fermi((li - w_hi) / w_kT) - fermi((li - w_lo) / w_kT)
                                            : fermi((li - mu) / kT) * (mode == kRowsEnergy ? li : 1.0);
      ya[(long long)i * kMaxOrb + a] = wt * ws.G0[(long long)i * kTrack + a];
    }
    __syncthreads();
    double *r = dc_apply(n, M, ws, ya, yb, qlds);
    // r <- Q r = Q1 (Q2 r): the bulge-chasing reflectors, then the band reduction's compact-WY
    // panels (T factors stored by the band reduction)
    if (n >= 3) {
      __syncthreads();  // the merge data in the same LDS is no longer read
      double *runs = qlds, *ex = qlds + 3LL * q2_lds_stride(n);
      density_q2(A, n, r, M, runs, ex);
    }
    density_q1(A, n, cv + vl.u, r, M, qlds);
    // x_P = L_PP^{-T} r_P = ((L^{-1})_PP)^T r_P (P = the last p rows; the S slot holds L^{-1}):
    // x(g) = sum_{t >= g} Linv(t, g) r(t), written to the other buffer
    const int b0 = n - p;
    double *xo = (r == ya) ? yb : ya;
    density_lt(L, ld, n, b0, r, xo, M);
    __syncthreads();
    r = xo;
    // scatter D(i, j) for j in F_i (members F \ {i} then i, last in the member list)
    const int fb = fna_ptr[c], nf = fna_ptr[c + 1] - fb;
    const int mend = mem_ptr[c + 1];
    if (tid == 0) {
      foff[0] = 0;
      for (int q = 0; q < nf; ++q) foff[q + 1] = foff[q] + n_orb[mem_atom[mend - nf + q]];
    }
    __syncthreads();
    double eh = 0.0, es = 0.0;
    for (int e = tid; e < p * M; e += nthr) {
      const int prow = e / M, a = e % M;
      int q = 0;
      while (foff[q + 1] <= prow) ++q;
      const int j = mem_atom[mend - nf + q];
      const int mj = n_orb[j];
      const int be = prow - foff[q];
      const long long o = blk_off[fna_blk[fb + q]] + (long long)a * mj + be;
      const double dv = r[(long long)(b0 + prow) * kMaxOrb + a];
      Dout[o] = dv;
      eh += dv * H[o];
      es += dv * S[o];
    }
    eh = block_sum(eh, sred);
    es = block_sum(es, sred);
    if (tid == 0) {
      partial[2 * c] = eh;
      partial[2 * c + 1] = es;
    }
  }
  queue_leave(queue);
}

__global__ void sum_pairs_kernel(int n, const double *__restrict__ partial, double *__restrict__ out) {
  __shared__ double red[8];
  double a = 0.0, b = 0.0;
  // fixed order: thread t sums clusters t, t + 256, ...; then a fixed tree
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    a += partial[2 * c];
    b += partial[2 * c + 1];
  }
  a = block_sum(a, red);
  b = block_sum(b, red);
  if (threadIdx.x == 0) {
    out[0] = a;
    out[1] = b;
  }
}

void launch_mu_init(Plan &p, double kT) {
  (void)kT;
  hipLaunchKernelGGL(mu_step_kernel, dim3(p.workgroups), dim3(kWG), 0, p.stream, 0, p.n_atoms, p.d_vec,
                     p.d_vec_off, p.d_dmax, p.d_dim, p.d_mu, p.d_partial, p.d_counter, p.d_status);
}

void launch_mu_step(Plan &p, double, double, double) {
  hipLaunchKernelGGL(mu_step_kernel, dim3(p.workgroups), dim3(kWG), 0, p.stream, 1, p.n_atoms, p.d_vec,
                     p.d_vec_off, p.d_dmax, p.d_dim, p.d_mu, p.d_partial, p.d_counter, p.d_status);
}

void launch_density(Plan &p, int mode, double *d_D, const double *d_H, const double *d_S, double w_lo, double w_hi,
                    double w_kT) {
  double *cl_partial = p.d_partial + kMuStride * p.workgroups;
  const int dm = cur_dim(p);
  const size_t lds = sizeof(double) * kDensityLds;
  const int n = cur_count(p);
  const int grid = std::max(1, std::min(stage_grid(p, kTDensity, p.workgroups), n));
  hipLaunchKernelGGL(density_kernel, dim3(grid), dim3(kWG), lds, p.stream, mode, w_lo, w_hi, w_kT, n, cur_order(p),
                     p.d_mat, p.d_mat_off, p.d_vec, p.d_vec_off, p.d_ivec, p.d_ivec_off, p.d_dmax, p.d_dim, p.d_n_orb,
                     p.d_p_rows, p.d_mem_ptr, p.d_mem_atom, p.d_fna_ptr, p.d_fna_blk, p.d_blk_off, p.d_mu, d_H, d_S,
                     d_D, cl_partial, dm, p.d_queue);
}

void launch_density_sums(Plan &p, int mode) {
  double *cl_partial = p.d_partial + kMuStride * p.workgroups;
  hipLaunchKernelGGL(sum_pairs_kernel, dim3(1), dim3(kWG), 0, p.stream, p.n_atoms, cl_partial,
                     p.d_mu + (mode == kRowsWindow ? 20 : (mode == kRowsEnergy ? 18 : 16)));
}

// State of a density: fixed == 0 prepares a bisection (n_e, kT, g), fixed != 0 sets mu and
// marks the bisection done.
__global__ void state_init_kernel(double *state, double n_e, double kT, double g, int fixed, double mu) {
  const int t = threadIdx.x;
  if (t < 32) state[t] = 0.0;
  __syncthreads();
  if (t == 0) {
    state[MU_NE] = n_e;
    state[MU_KT] = kT;
    state[MU_G] = g;
    if (fixed) {
      state[MU_DONE] = 1.0;
      state[MU_MU] = mu;
    }
  }
}

void launch_state_init(Plan &p, double n_e, double kT, double g, int fixed, double mu) {
  hipLaunchKernelGGL(state_init_kernel, dim3(1), dim3(64), 0, p.stream, p.d_mu, n_e, kT, g, fixed, mu);
}

__global__ void fill_int_kernel(int *d, int n, int v) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) d[i] = v;
}

void launch_fill_int(Plan &p, int *d, int n, int v) {
  const int blocks = std::max(1, std::min(256, (n + 255) / 256));
  hipLaunchKernelGGL(fill_int_kernel, dim3(blocks), dim3(256), 0, p.stream, d, n, v);
}

}  // namespace ldc
