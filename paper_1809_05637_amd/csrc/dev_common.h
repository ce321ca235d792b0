// Device helpers shared by the kernels of libldc (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include "ldc_internal.h"

namespace ldc {

// First error wins; later errors are dropped.
__device__ inline void report(DevStatus *st, int code, int where) {
  if (atomicCAS(&st->code, 0, code) == 0) atomicExch(&st->where, where);
}

// Sum over a 64-lane wavefront (every lane gets the total).
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
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
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  __syncthreads();
  if (lane == 0) scratch[wid] = v;
  __syncthreads();
  double t = scratch[0];
  for (int w = 1; w < nw; ++w) t = fmax(t, scratch[w]);
  return t;
}

// Fermi-Dirac occupation f(x) = 1/(1+e^x), evaluated as (1 - tanh(x/2))/2.
__device__ inline double fermi(double x) { return 0.5 * (1.0 - tanh(0.5 * x)); }

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
