// Internal declarations shared by the host code and the kernel launchers of libldc.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ldc.h"

namespace ldc {

constexpr int kMaxOrb = 16;        // orbitals per atom (compiled limit)
constexpr int kMaxMembers = 1024;  // atoms per cluster (compiled limit)
constexpr int kWG = 256;           // threads per workgroup of the per-cluster kernels
constexpr int kTrack = 2 * kMaxOrb + 2;  // tracked columns in the tridiagonal solver

// Device status word: [0] first error code, [1] failing cluster/atom.
struct DevStatus {
  int code;
  int where;
};

// Per-cluster layout of the tridiagonal-solver records (all offsets in elements).
// n = dimension bound of the cluster (plain-DC dimension), L = number of merge levels.
struct DcLayout {
  // doubles per level: rot_c, rot_s, dK, zt, tau, nrm  -> 6 n
  // ints per level:    perm, kpos, oo, rot_a, rot_b, orig, cnt -> 7 n
  static int levels(int n) {
    int l = 0;
    while ((1 << l) < n) ++l;
    return l;
  }
};

// Stages whose launch is chosen per size bucket (grid of the persistent launch).
enum TunedStage { kTGather = 0, kTPotrf, kTSygst, kTSy2sb, kTSb2st, kTQ2x, kTStedc, kTDensity, kNumTuned };

// A size bucket: a contiguous range of the processing order (clusters sorted by dimension,
// largest first), the largest dimension its clusters can have in the current mode (LDS sizes
// and strides of the bucket's launches follow it), and the launch grid of every tuned stage
// (0: the stage's default).
struct Bucket {
  int begin = 0, count = 0;
  int dim_bound = 0;
  int grid[kNumTuned] = {};
};

// Key of a captured build: the graph is replayed only for the same pointers and parameters.
struct BuildKey {
  const void *H = nullptr, *S = nullptr, *Dprev = nullptr, *Dout = nullptr;
  double lambda_th = 0.0, n_e = 0.0, kT = 0.0;
  int k_min = 0, k_max = 0, has_fixed = 0, prec = 0;
  long long bucket_sig = 0;
  hipStream_t stream = nullptr;
  bool operator==(const BuildKey &o) const {
    return H == o.H && S == o.S && Dprev == o.Dprev && Dout == o.Dout && lambda_th == o.lambda_th &&
           n_e == o.n_e && kT == o.kT && k_min == o.k_min && k_max == o.k_max && has_fixed == o.has_fixed &&
           prec == o.prec && bucket_sig == o.bucket_sig && stream == o.stream;
  }
};

struct Plan {
  int n_atoms = 0, nnzb = 0, n_basis = 0, mmax = 0;
  ldc_options opt{};
  hipStream_t stream = nullptr;
  int n_cu = 0;
  int device = 0;                   // HIP device of the plan (current at creation)
  int workgroups = 0;

  // host copies of the geometry and pattern
  std::vector<int> n_orb, row_ptr, col;
  std::vector<long long> blk_off;
  long long blk_total = 0;                       // elements of one block-sparse matrix
  std::vector<long long> row_elem;               // first element of every block row (n_atoms + 1)

  // regions, in the library's member order: long, short \ F, F \ {i}, i
  std::vector<int> mem_ptr, mem_atom, mem_long;
  std::vector<int> pair_ptr, pair_ab, pair_blk;  // gather list: (a | b << 16), block index
  std::vector<int> fna_ptr, fna_blk;             // P rows: block index of (i, j) per F member
  std::vector<int> p_rows;                       // rows of the P block (sum of M over F_i)
  std::vector<int> dmax;                         // plain-DC dimension (workspace bound)
  std::vector<int> order;                        // processing order, largest first
  int max_members = 0, max_dim = 0;

  // device tables
  int *d_n_orb = nullptr, *d_row_ptr = nullptr, *d_col = nullptr;
  long long *d_blk_off = nullptr, *d_row_elem = nullptr;
  int *d_mem_ptr = nullptr, *d_mem_atom = nullptr, *d_mem_long = nullptr;
  int *d_pair_ptr = nullptr, *d_pair_ab = nullptr, *d_pair_blk = nullptr;
  int *d_fna_ptr = nullptr, *d_fna_blk = nullptr, *d_p_rows = nullptr;
  int *d_dmax = nullptr, *d_order = nullptr;

  // per-cluster workspaces
  long long *d_mat_off = nullptr;   // H slot at off, S slot at off + dmax^2
  long long *d_vec_off = nullptr;   // double vectors
  long long *d_ivec_off = nullptr;  // int vectors
  double *d_mat = nullptr, *d_vec = nullptr;
  int *d_ivec = nullptr;
  int *d_dim = nullptr;             // current reduced dimension per cluster

  // LNO table
  int lno_mode = 0;
  int *d_rank = nullptr;
  double *d_U = nullptr;            // n_atoms x kMaxOrb^2, U_j column-major M_j x k_j
  double *d_lambda = nullptr;       // n_atoms x kMaxOrb^2 scratch (Lambda matrices)
  int *d_fixed = nullptr;           // n_atoms fixed ranks (-1: rule)
  // LNO-contracted pattern blocks (Eq. 26), 6 x blk_total: for v = 0 (U_i^T X_ij),
  // 1 (X_ij U_j), 2 (U_i^T X_ij U_j) and X = H, S, slot 2 v + (X == S); allocated by the
  // first ldc_lno with a previous density, rebuilt by every ldc_solve in LNO mode
  double *d_lno_blk = nullptr;

  // chemical potential state and reductions
  double *d_mu = nullptr;           // [lo, hi, mid, done, n_at_mid, bracket checks...]
  double *d_partial = nullptr;      // per-workgroup partial sums
  int *d_counter = nullptr;
  int *d_queue = nullptr;           // cluster work queue of the per-cluster kernels (2 ints)
  DevStatus *d_status = nullptr;

  // stage timing (HIP events on the plan's stream)
  int profile = 0;
  hipEvent_t ev_begin[LDC_NUM_STAGES] = {}, ev_end[LDC_NUM_STAGES] = {};
  int ev_pending[LDC_NUM_STAGES] = {};
  double stage_ms[LDC_NUM_STAGES] = {};
  int prof_builds = 0;

  // size buckets of the current mode and the one being launched (launchers read their range,
  // dimension bound and grid from it)
  std::vector<Bucket> buckets;
  std::vector<int> dim_bound;       // per cluster: largest dimension in the current mode
  int bucket_mode = -1;             // the bound the buckets were made for (-1: none yet)
  std::string bucket_wkey;          // workload key of the current bounds
  const Bucket *cur = nullptr;
  // tuning: per (stage, bucket) HIP events around the bucket's launch
  int tuning = 0;
  std::vector<hipEvent_t> tune_ev;  // 2 per (stage, bucket)
  std::string tune_source;          // where the current launch choices came from

  // pinned host staging (fixed ranks in, state and status out) and the captured build
  int *h_fixed = nullptr;
  double *h_out = nullptr;          // 32 state doubles, then the status word
  hipEvent_t ev_fixed = nullptr;    // the last copy out of h_fixed
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  BuildKey graph_key;
  int graph_builds = 0, graph_captures = 0;

  const double *last_H = nullptr, *last_S = nullptr;
  int solved = 0;
  int has_density = 0;              // a density was built since the last ldc_solve
  size_t device_bytes = 0;
  std::string msg;
  int err_where = -1;
};

// vector workspace offsets inside a cluster's double region (n = dimension bound)
// Band width of the reduction to band form and the row stride of the band array used by
// the bulge chasing (lower band plus bulge: 2 kBand + 1 diagonals, padded to 80 doubles, five
// 128-byte cache lines, so that every column of the line-aligned array starts on a line).
constexpr int kBand = 32;
constexpr int kBandLd = 80;
static_assert(kBandLd >= 2 * kBand + 1 && kBandLd % 16 == 0, "band array stride");
// Largest reduced cluster dimension (the panel QR holds 8 columns of the panel in LDS and a
// column in 15 registers per lane).
constexpr int kMaxDimTri = 960;

struct VecLayout {
  long long d, e, tau, lam, w, G0, G1, u, y0, y1, vw, vt, kg, dc;
  __host__ __device__ static VecLayout make(int n) {
    VecLayout v;
    long long o = 0;
    v.d = o; o += n;
    v.e = o; o += n;
    v.tau = o; o += n;
    v.lam = o; o += n;
    v.w = o; o += n;
    v.G0 = o; o += (long long)n * kTrack;
    v.G1 = o; o += (long long)n * kTrack;
    v.u = o; o += (long long)(n + 32) * 32;  // compact-WY T factors, one 32 x 32 block per panel
    v.y0 = o; o += (long long)n * kMaxOrb;
    v.y1 = o; o += (long long)n * kMaxOrb;
    // reduction to band form: [V | W] (n x 2 kBand, row-major), -V T (n x kBand, row-major),
    // K and G (kBand x kBand each); the band array of the bulge chasing (n x kBandLd, from the
    // first 128-byte boundary) reuses this space once the band form is complete
    v.vw = o; o += (long long)n * 2 * kBand;
    v.vt = o; o += (long long)n * kBand;
    v.kg = o; o += 2LL * kBand * kBand;
    v.dc = o;
    static_assert(3 * kBand >= kBandLd, "the band array fits the [V | W] and -V T space");
    return v;
  }
  __host__ __device__ static long long total(int n) {
    int l = 0;
    while ((1 << l) < n) ++l;
    return make(n).dc + 6LL * n * (l > 0 ? l : 1);
  }
};

struct IvecLayout {
  __host__ __device__ static long long total(int n) {
    int l = 0;
    while ((1 << l) < n) ++l;
    return 7LL * n * (l > 0 ? l : 1);
  }
};

// host planner
ldc_status build_regions(Plan &p, const double *pos, const double *cell, const int *periodic);

// device part of ldc_density on the plan's current scratch pointers (d_mu, d_counter, d_partial)
ldc_status enqueue_density_steps(Plan &p, double n_electrons, double kT, double *d_D_out);
// scratch of the allocation-free density entry point: address of the file-scope array on a
// device (set up once per device, with the device current), or nullptr
ldc_status noalloc_setup(int device, std::string &msg);
double *noalloc_scratch(int device);

// launch range of the current bucket (the whole processing order when no bucket is set)
inline const int *cur_order(const Plan &p) { return p.cur ? p.d_order + p.cur->begin : p.d_order; }
inline int cur_count(const Plan &p) { return p.cur ? p.cur->count : p.n_atoms; }
inline int cur_dim(const Plan &p) { return p.cur ? p.cur->dim_bound : p.max_dim; }
inline int stage_grid(const Plan &p, int stage, int dflt) {
  const int g = p.cur ? p.cur->grid[stage] : 0;
  return g > 0 ? g : dflt;
}

// kernel launchers (each enqueues on p.stream)
void launch_lambda(Plan &p, const double *d_S, const double *d_D);
void launch_lno_eig(Plan &p, const double *d_S, double lambda_th, int k_min, int k_max);
// LNO-contracted pattern blocks (Eq. 26), once per ldc_solve in LNO mode
void launch_lno_blocks(Plan &p, const double *d_H, const double *d_S);
void launch_gather(Plan &p, const double *d_H, const double *d_S);
void launch_potrf(Plan &p);
void launch_sygst(Plan &p);
void launch_sy2sb(Plan &p);
void launch_sb2st(Plan &p);
void launch_q2x(Plan &p);
void launch_stedc(Plan &p);
// halvings of the chemical-potential bisection per launch (a tree of 2^k - 1 points), and the
// number of launches that covers the 200-halving limit
constexpr int kMuLevels = 4;
constexpr int kMuLaunches = (200 + kMuLevels - 1) / kMuLevels;
void launch_mu_init(Plan &p, double kT);
void launch_mu_step(Plan &p, double n_electrons, double kT, double g);
void launch_mu_fixed(Plan &p, double mu);
// Row modes of launch_density: density rows (sums of D.H and D.S to state[16..17]), energy
// density rows (E.H, E.S to state[18..19]), both at mu = state[MU_MU], kT = state[MU_KT]; or
// windowed density rows over (w_lo, w_hi) with edge width w_kT (W.H, W.S to state[20..21]).
enum { kRowsDensity = 0, kRowsEnergy = 1, kRowsWindow = 2 };
void launch_density(Plan &p, int mode, double *d_D, const double *d_H, const double *d_S, double w_lo = 0.0,
                    double w_hi = 0.0, double w_kT = 1.0);
// sums of the rows' traces with H and S over all clusters into the state slots of the mode
void launch_density_sums(Plan &p, int mode);
// state set-up of a density (n_e, kT, g; mu_fixed >= ... with fixed != 0: no bisection)
void launch_state_init(Plan &p, double n_e, double kT, double g, int fixed, double mu);
// every entry of an int array set to v
void launch_fill_int(Plan &p, int *d, int n, int v);
// toy SCF loop: Mulliken populations, potential on H0, linear mixing (residual to d_res[0])
void launch_mulliken(Plan &p, const double *d_D, const double *d_S, double *d_q, double g);
void launch_potential(Plan &p, const double *d_H0, const double *d_S, const double *d_v, double *d_H);
// q0_i = N_e M_i / sum_j M_j
void launch_reference_populations(Plan &p, double n_electrons, double *d_q0);
void launch_scf_mix(Plan &p, const double *d_q_out, double *d_q_in, const double *d_q0, double U, double alpha,
                    double *d_v, double *d_res);

}  // namespace ldc

struct ldc_plan_s {
  ldc::Plan p;
};
