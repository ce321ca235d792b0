// Allocation-free density entry point (ldc_density_noalloc): the same chemical-potential
// bisection and density rows as ldc_density, with every buffer that ldc_density keeps in
// plan-allocated memory between its kernels -- the bisection state, the workgroups' ticket
// counter, their partial sums and the per-cluster row sums -- taken from one file-scope device
// array instead, and the results (mu, E_band, N_e) written to device memory, so that the call
// neither allocates nor waits for the device.
#include <mutex>
#include <string>

#include "dev_common.h"
#include "ldc_internal.h"

namespace ldc {

// Limits of the array: atoms (clusters) of a plan and persistent workgroups of its launches.
constexpr int kNoallocMaxAtoms = 65536;
constexpr int kNoallocMaxGrid = 2048;
// Layout (doubles): the 32-double bisection state, the ticket counter (one int, alone on its
// own 64-byte line), the per-workgroup bisection partials (16 per workgroup, the stride of the
// bisection kernel), then two row sums per cluster.
constexpr long long kNaState = 0, kNaCounter = 32, kNaPartial = 40;
constexpr long long kNaDoubles = kNaPartial + 16LL * kNoallocMaxGrid + 2LL * kNoallocMaxAtoms;  // 1.3 MB

static __device__ __align__(256) double scratch[kNaDoubles];

namespace {
std::mutex g_na_mutex;
constexpr int kNaDevices = 64;
double *g_na_ptr[kNaDevices] = {};
}  // namespace

ldc_status noalloc_setup(int device, std::string &msg) {
  std::lock_guard<std::mutex> lock(g_na_mutex);
  if (device < 0 || device >= kNaDevices) {
    msg = "device index out of range for the allocation-free scratch";
    return LDC_ERR_LIMIT;
  }
  if (g_na_ptr[device]) return LDC_OK;
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    (void)hipGetLastError();
    msg = std::string("hipGetSymbolAddress of the scratch array failed: ") + hipGetErrorString(e);
    return LDC_ERR_DEVICE;
  }
  g_na_ptr[device] = static_cast<double *>(ptr);
  return LDC_OK;
}

double *noalloc_scratch(int device) {
  std::lock_guard<std::mutex> lock(g_na_mutex);
  return (device >= 0 && device < kNaDevices) ? g_na_ptr[device] : nullptr;
}

// The ticket counter starts every call at zero (a kernel, not a memset: the call may be
// captured into a graph).
__global__ void noalloc_clear_kernel(int *counter) {
  if (threadIdx.x == 0) counter[0] = 0;
}

// Results to the caller's device array and the state to the plan's own state buffer (so that
// ldc_energy_density after this call uses this density's mu and kT).
__global__ void noalloc_finish_kernel(const double *__restrict__ state, double g, double *__restrict__ result,
                                      double *__restrict__ plan_state) {
  const int t = threadIdx.x;
  if (t < 32) plan_state[t] = state[t];
  if (t == 0) {
    result[0] = state[8];        // mu
    result[1] = g * state[16];   // E_band = g sum tr(D H)
    result[2] = g * state[17];   // N_e = g Tr(D S)
  }
}

}  // namespace ldc

extern "C" ldc_status ldc_density_noalloc(ldc_plan_t plan, double n_electrons, double kT, double *d_D_out,
                                          double *d_result) {
  if (!plan || !d_D_out || !d_result || !(kT > 0.0)) return LDC_ERR_ARG;
  ldc::Plan &p = plan->p;
  if (!p.solved) {
    p.msg = "ldc_density_noalloc called before ldc_solve";
    return LDC_ERR_STATE;
  }
  if (p.n_atoms > ldc::kNoallocMaxAtoms || p.workgroups > ldc::kNoallocMaxGrid) {
    p.msg = "ldc_density_noalloc: the plan has " + std::to_string(p.n_atoms) + " atoms and " +
            std::to_string(p.workgroups) + " workgroups; the scratch array holds at most " +
            std::to_string(ldc::kNoallocMaxAtoms) + " atoms and " + std::to_string(ldc::kNoallocMaxGrid) +
            " workgroups";
    return LDC_ERR_LIMIT;
  }
  double *base = ldc::noalloc_scratch(p.device);
  if (!base) {
    // the set-up at plan creation failed: retry once on the plan's device
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != p.device) {
      (void)hipGetLastError();
      p.msg = "ldc_density_noalloc: the plan's device is not current";
      return LDC_ERR_DEVICE;
    }
    ldc_status s = ldc::noalloc_setup(p.device, p.msg);
    if (s != LDC_OK) return s;
    base = ldc::noalloc_scratch(p.device);
  }
  const double g = p.opt.spin_g > 0 ? p.opt.spin_g : 2;
  // the kernels take the scratch addresses in place of the plan's buffers for this call
  double *own_mu = p.d_mu, *own_partial = p.d_partial;
  int *own_counter = p.d_counter;
  p.d_mu = base + ldc::kNaState;
  p.d_counter = reinterpret_cast<int *>(base + ldc::kNaCounter);
  p.d_partial = base + ldc::kNaPartial;
  hipLaunchKernelGGL(ldc::noalloc_clear_kernel, dim3(1), dim3(64), 0, p.stream, p.d_counter);
  ldc_status s = ldc::enqueue_density_steps(p, n_electrons, kT, d_D_out);
  if (s == LDC_OK)
    hipLaunchKernelGGL(ldc::noalloc_finish_kernel, dim3(1), dim3(64), 0, p.stream, p.d_mu, g, d_result, own_mu);
  p.d_mu = own_mu;
  p.d_partial = own_partial;
  p.d_counter = own_counter;
  if (s != LDC_OK) return s;
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    p.msg = std::string("HIP error: ") + hipGetErrorString(e);
    return LDC_ERR_DEVICE;
  }
  p.has_density = 1;
  return LDC_OK;
}
