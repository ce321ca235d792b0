// Device helpers shared by the kernels of libldc (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include "ldc_internal.h"

namespace ldc {

// Out of line, a device function receives generic pointers and addresses them with flat
// instructions, which also count against the LDS counter (so a wait for an LDS read waits for
// outstanding memory loads too).  These restate where a pointer points (global memory or LDS), so
// that its accesses compile to global or ds instructions.  Only for pointers known to point there.
// The typed pointer is rebuilt from the address (an LDS pointer's flat address holds its LDS
// offset in the low half), so that only one cast, to generic, remains for the compiler to see
// through.
template <typename T>
__device__ inline T *global_ptr(T *p) {
  typedef __attribute__((address_space(1))) T gT;
  return (T *)(gT *)reinterpret_cast<unsigned long long>(p);
}
template <typename T>
__device__ inline T *lds_ptr(T *p) {
  typedef __attribute__((address_space(3))) T lT;
  return (T *)(lT *)(unsigned)reinterpret_cast<unsigned long long>(p);
}

// Clusters handed to workgroups as they become free: each workgroup takes the next index of the
// processing order (largest clusters first), so the last, smallest clusters go to whichever
// workgroups finish first instead of to a fixed stride.  q[0] is the next index, q[1] the number of
// workgroups that have left the loop; the last to leave resets both, so the queue reads zero at the
// next launch (the plan zeroes it once, when it is created).  Every workgroup calls queue_next
// until it returns an index past the end, then queue_leave once.  The result does not depend on
// which workgroup takes which cluster (each cluster's work is its workgroup's alone).
__device__ inline int queue_next(int *q) {
  __shared__ int next;
  __syncthreads();
  if (threadIdx.x == 0) next = atomicAdd(&q[0], 1);
  __syncthreads();
  return next;
}
__device__ inline void queue_leave(int *q) {
  if (threadIdx.x == 0) {
    __threadfence();
    if (atomicAdd(&q[1], 1) == (int)gridDim.x - 1) {
      atomicExch(&q[0], 0);
      atomicExch(&q[1], 0);
    }
  }
}

// First error wins; later errors are dropped.
__device__ inline void report(DevStatus *st, int code, int where) {
  if (atomicCAS(&st->code, 0, code) == 0) atomicExch(&st->where, where);
}

// Lane permutations of DPP moves within rows of 16 lanes: exchange with lane ^ 1 and lane ^ 2
// inside each quad, mirror each 8-lane half row, mirror each row.
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140;

template <int CTRL>
__device__ inline double dpp_perm(double v) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)u, CTRL, 0xF, 0xF, false);
  const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(u >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ inline double lane_value(double v, int l) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Sum over the 8 consecutive lanes of each group (every lane of the group gets its sum).
__device__ inline double group8_sum(double v) {
  v += dpp_perm<kDppXor1>(v);
  v += dpp_perm<kDppXor2>(v);
  v += dpp_perm<kDppHalfMirror>(v);
  return v;
}

// Sum over a 64-lane wavefront (every lane gets the total; all lanes must be active).
// Row sums by DPP moves, then the four rows through scalar reads.
__device__ inline double wave_sum(double v) {
  v = group8_sum(v);
  v += dpp_perm<kDppMirror>(v);
  return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
}

__device__ inline double wave_max(double v) {
  v = fmax(v, dpp_perm<kDppXor1>(v));
  v = fmax(v, dpp_perm<kDppXor2>(v));
  v = fmax(v, dpp_perm<kDppHalfMirror>(v));
  v = fmax(v, dpp_perm<kDppMirror>(v));
  return fmax(fmax(lane_value(v, 0), lane_value(v, 16)), fmax(lane_value(v, 32), lane_value(v, 48)));
}

// Workgroup sum of one value per thread; scratch: >= blockDim.x/64 doubles of LDS.
// Deterministic (fixed tree).  Every thread receives the total.
__device__ inline double block_sum(double v, double *scratch) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) scratch[wid] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < nw; ++w) t += scratch[w];
  return t;
}

__device__ inline double block_max(double v, double *scratch) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v = wave_max(v);
  __syncthreads();
  if (lane == 0) scratch[wid] = v;
  __syncthreads();
  double t = scratch[0];
  for (int w = 1; w < nw; ++w) t = fmax(t, scratch[w]);
  return t;
}

// 1/x by the hardware reciprocal and two Newton steps (a few ulp; x finite, nonzero and of
// normal magnitude -- the D&C denominators d_j - lambda are never zero for kept poles).
__device__ inline double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// Fermi-Dirac occupation f(x) = 1/(1+e^x), evaluated as (1 - tanh(x/2))/2.
__device__ inline double fermi(double x) { return 0.5 * (1.0 - tanh(0.5 * x)); }
// The same values without the tanh far from the step: for |x| > 80, tanh(x / 2) rounds to +-1
// in double precision (1 - tanh(40) < 1e-34), so f is exactly 0 or 1 there.
__device__ inline double fermi_fast(double x) {
  return x > 80.0 ? 0.0 : (x < -80.0 ? 1.0 : 0.5 * (1.0 - tanh(0.5 * x)));
}

// Per-cluster workspace pointers.
struct ClusterWs {
  double *H, *S;      // column-major, leading dimension = current dimension
  double *vec;
  int *ivec;
  int dmax;
};

__device__ inline ClusterWs cluster_ws(double *mat, const long long *mat_off, double *vec, const long long *vec_off,
                                      int *ivec, const long long *ivec_off, const int *dmax, int c) {
  ClusterWs w;
  w.dmax = dmax[c];
  w.H = mat + mat_off[c];
  w.S = w.H + (long long)w.dmax * w.dmax;
  w.vec = vec + vec_off[c];
  w.ivec = ivec + ivec_off[c];
  return w;
}

}  // namespace ldc
