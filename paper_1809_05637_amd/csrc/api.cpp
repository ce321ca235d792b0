// C ABI of libldc: plan lifecycle and the per-build entry points (ldc_lno, ldc_solve,
// ldc_density).  All device work is enqueued on the plan's stream.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <new>

#include "ldc_internal.h"

using ldc::Plan;

namespace {

// slot of the plan's small state array that receives the SCF mixing residual
constexpr int kScfResidualSlot = 24;

const char *kVersion = "ldc 0.1.0 (gfx950)";

#define HIPCHK(expr)                                                                         \
  do {                                                                                       \
    hipError_t _e = (expr);                                                                  \
    if (_e != hipSuccess) {                                                                  \
      p.msg = std::string("HIP error: ") + hipGetErrorString(_e) + " at " #expr;            \
      return LDC_ERR_DEVICE;                                                                 \
    }                                                                                        \
  } while (0)

template <typename T>
ldc_status dev_alloc(Plan &p, T **ptr, size_t count) {
  *ptr = nullptr;
  if (count == 0) count = 1;
  hipError_t e = hipMalloc((void **)ptr, sizeof(T) * count);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    p.msg = "device allocation of " + std::to_string(sizeof(T) * count) + " bytes failed";
    *ptr = nullptr;
    return LDC_ERR_OOM;
  }
  p.device_bytes += sizeof(T) * count;
  return LDC_OK;
}

template <typename T>
ldc_status upload(Plan &p, T **ptr, const std::vector<T> &v) {
  ldc_status s = dev_alloc(p, ptr, v.size());
  if (s != LDC_OK) return s;
  if (!v.empty()) HIPCHK(hipMemcpy(*ptr, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice));
  return LDC_OK;
}

void free_all(Plan &p) {
  void *ptrs[] = {p.d_n_orb,    p.d_row_ptr,  p.d_col,      p.d_blk_off, p.d_mem_ptr, p.d_mem_atom, p.d_mem_long,
                  p.d_pair_ptr, p.d_pair_ab,  p.d_pair_blk, p.d_fna_ptr, p.d_fna_blk, p.d_p_rows,   p.d_dmax,
                  p.d_order,    p.d_mat_off,  p.d_vec_off,  p.d_ivec_off, p.d_mat,    p.d_vec,      p.d_ivec,
                  p.d_dim,      p.d_rank,     p.d_U,        p.d_lambda,  p.d_fixed,   p.d_mu,       p.d_partial,
                  p.d_counter,  p.d_status,   p.d_lno_blk,  p.d_row_elem};
  for (void *q : ptrs)
    if (q) (void)hipFree(q);
  for (int s = 0; s < LDC_NUM_STAGES; ++s) {
    if (p.ev_begin[s]) (void)hipEventDestroy(p.ev_begin[s]);
    if (p.ev_end[s]) (void)hipEventDestroy(p.ev_end[s]);
  }
}

// Reads and clears the device status word (synchronizes the stream).
ldc_status check_status(Plan &p) {
  HIPCHK(hipStreamSynchronize(p.stream));
  ldc::DevStatus st{0, -1};
  HIPCHK(hipMemcpy(&st, p.d_status, sizeof(st), hipMemcpyDeviceToHost));
  if (st.code != 0) {
    static const char *names[] = {"ok", "bad argument", "overlap matrix not positive definite",
                                  "eigensolver did not converge", "electron count outside the bracket",
                                  "LNO basis rank deficient", "out of memory", "device error", "state",
                                  "limit exceeded"};
    const int code = st.code;
    p.msg = std::string(code >= 0 && code < 10 ? names[code] : "error") + " (cluster/atom " +
            std::to_string(st.where) + ")";
    p.err_where = st.where;
    ldc::DevStatus zero{0, -1};
    HIPCHK(hipMemcpy(p.d_status, &zero, sizeof(zero), hipMemcpyHostToDevice));
    return (ldc_status)code;
  }
  return LDC_OK;
}

const char *kStageNames[LDC_NUM_STAGES] = {"lambda", "lno_eig", "gather", "potrf", "sygst",
                                           "sy2sb", "sb2st", "q2x", "stedc", "mu", "density"};

inline void stage_begin(Plan &p, int s) {
  if (p.profile) (void)hipEventRecord(p.ev_begin[s], p.stream);
}
inline void stage_end(Plan &p, int s) {
  if (p.profile) {
    (void)hipEventRecord(p.ev_end[s], p.stream);
    p.ev_pending[s] = 1;
  }
}
// Adds the elapsed times of completed stages (events must have completed).
void collect_stages(Plan &p) {
  if (!p.profile) return;
  for (int s = 0; s < LDC_NUM_STAGES; ++s) {
    if (!p.ev_pending[s]) continue;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.ev_begin[s], p.ev_end[s]) == hipSuccess) p.stage_ms[s] += ms;
    else (void)hipGetLastError();
    p.ev_pending[s] = 0;
  }
}

}  // namespace

extern "C" {

const char *ldc_stage_name(int stage) {
  return (stage >= 0 && stage < LDC_NUM_STAGES) ? kStageNames[stage] : "unknown";
}

ldc_status ldc_profile(ldc_plan_t plan, int enable) {
  if (!plan) return LDC_ERR_ARG;
  Plan &p = plan->p;
  HIPCHK(hipStreamSynchronize(p.stream));
  if (enable && !p.ev_begin[0]) {
    for (int s = 0; s < LDC_NUM_STAGES; ++s) {
      HIPCHK(hipEventCreate(&p.ev_begin[s]));
      HIPCHK(hipEventCreate(&p.ev_end[s]));
    }
  }
  p.profile = enable ? 1 : 0;
  for (int s = 0; s < LDC_NUM_STAGES; ++s) {
    p.stage_ms[s] = 0.0;
    p.ev_pending[s] = 0;
  }
  p.prof_builds = 0;
  return LDC_OK;
}

ldc_status ldc_stage_times(ldc_plan_t plan, double *ms, int *builds) {
  if (!plan || !ms) return LDC_ERR_ARG;
  Plan &p = plan->p;
  HIPCHK(hipStreamSynchronize(p.stream));
  collect_stages(p);
  for (int s = 0; s < LDC_NUM_STAGES; ++s) ms[s] = p.stage_ms[s];
  if (builds) *builds = p.prof_builds;
  return LDC_OK;
}

ldc_status ldc_cluster_dims(ldc_plan_t plan, int *dims) {
  if (!plan || !dims) return LDC_ERR_ARG;
  Plan &p = plan->p;
  if (!p.solved) return LDC_ERR_STATE;
  HIPCHK(hipStreamSynchronize(p.stream));
  HIPCHK(hipMemcpy(dims, p.d_dim, sizeof(int) * p.n_atoms, hipMemcpyDeviceToHost));
  return LDC_OK;
}

const char *ldc_version(void) { return kVersion; }

ldc_status ldc_plan_create(ldc_plan_t *out, int n_atoms, const double *pos, const double *cell, const int *periodic,
                           const int *n_orb, int nnzb, const int *row_ptr, const int *col, const ldc_options *opt,
                           void *stream) {
  if (!out) return LDC_ERR_ARG;
  *out = nullptr;
  if (n_atoms <= 0 || !pos || !cell || !periodic || !n_orb || nnzb <= 0 || !row_ptr || !col || !opt ||
      !(opt->r_L > 0.0))
    return LDC_ERR_ARG;
  ldc_plan_s *h = new (std::nothrow) ldc_plan_s();
  if (!h) return LDC_ERR_OOM;
  Plan &p = h->p;
  p.n_atoms = n_atoms;
  p.nnzb = nnzb;
  p.opt = *opt;
  p.stream = (hipStream_t)stream;
  p.n_orb.assign(n_orb, n_orb + n_atoms);
  p.row_ptr.assign(row_ptr, row_ptr + n_atoms + 1);
  p.col.assign(col, col + nnzb);
  auto fail = [&](ldc_status s, const std::string &m) {
    free_all(p);
    delete h;
    (void)m;
    return s;
  };
  // validate the pattern
  if (p.row_ptr[0] != 0 || p.row_ptr[n_atoms] != nnzb) return fail(LDC_ERR_ARG, "row_ptr");
  for (int i = 0; i < n_atoms; ++i) {
    if (p.n_orb[i] < 1) return fail(LDC_ERR_ARG, "n_orb");
    if (p.n_orb[i] > ldc::kMaxOrb) return fail(LDC_ERR_LIMIT, "n_orb");
    if (p.row_ptr[i + 1] < p.row_ptr[i]) return fail(LDC_ERR_ARG, "row_ptr");
    bool diag = false;
    for (int b = p.row_ptr[i]; b < p.row_ptr[i + 1]; ++b) {
      if (p.col[b] < 0 || p.col[b] >= n_atoms) return fail(LDC_ERR_ARG, "col range");
      if (b > p.row_ptr[i] && p.col[b] <= p.col[b - 1]) return fail(LDC_ERR_ARG, "col order");
      diag |= (p.col[b] == i);
    }
    if (!diag) return fail(LDC_ERR_ARG, "diagonal block missing");
  }
  for (int i = 0; i < n_atoms; ++i)
    for (int b = p.row_ptr[i]; b < p.row_ptr[i + 1]; ++b) {
      const int j = p.col[b];
      if (!std::binary_search(p.col.begin() + p.row_ptr[j], p.col.begin() + p.row_ptr[j + 1], i))
        return fail(LDC_ERR_ARG, "pattern not symmetric");
    }
  p.blk_off.resize(nnzb);
  long long o = 0;
  p.n_basis = 0;
  p.mmax = 0;
  for (int i = 0; i < n_atoms; ++i) {
    p.n_basis += p.n_orb[i];
    p.mmax = std::max(p.mmax, p.n_orb[i]);
    for (int b = p.row_ptr[i]; b < p.row_ptr[i + 1]; ++b) {
      p.blk_off[b] = o;
      o += (long long)p.n_orb[i] * p.n_orb[p.col[b]];
    }
  }
  p.blk_total = o;
  p.row_elem.resize(n_atoms + 1);
  for (int i = 0; i < n_atoms; ++i) p.row_elem[i] = p.row_ptr[i] < nnzb ? p.blk_off[p.row_ptr[i]] : o;
  p.row_elem[n_atoms] = o;
  ldc_status s = ldc::build_regions(p, pos, cell, periodic);
  if (s != LDC_OK) {
    h->p.msg = p.msg;
    free_all(p);
    delete h;
    return s;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&p.n_cu, hipDeviceAttributeMultiprocessorCount, dev) !=
                                              hipSuccess) {
    (void)hipGetLastError();
    free_all(p);
    delete h;
    return LDC_ERR_DEVICE;
  }
  if (p.max_dim > ldc::kMaxDimTri) {
    free_all(p);
    delete h;
    return LDC_ERR_LIMIT;  // the band reduction holds 8 panel columns in LDS
  }
  p.workgroups = opt->workgroups > 0 ? opt->workgroups : 2 * p.n_cu;
  p.workgroups = std::max(1, std::min(p.workgroups, n_atoms));

  // per-cluster workspace offsets
  std::vector<long long> mat_off(n_atoms), vec_off(n_atoms), ivec_off(n_atoms);
  long long mo = 0, vo = 0, io = 0;
  for (int c = 0; c < n_atoms; ++c) {
    const long long dm = p.dmax[c];
    mat_off[c] = mo;
    mo += 2 * dm * dm;
    mo = (mo + 31) & ~31LL;
    vec_off[c] = vo;
    vo += ldc::VecLayout::total((int)dm);
    vo = (vo + 31) & ~31LL;
    ivec_off[c] = io;
    io += ldc::IvecLayout::total((int)dm);
    io = (io + 63) & ~63LL;
  }
#define TRY(x)                  \
  do {                          \
    ldc_status _s = (x);        \
    if (_s != LDC_OK) {         \
      free_all(p);              \
      delete h;                 \
      return _s;                \
    }                           \
  } while (0)
  TRY(upload(p, &p.d_n_orb, p.n_orb));
  TRY(upload(p, &p.d_row_ptr, p.row_ptr));
  TRY(upload(p, &p.d_col, p.col));
  TRY(upload(p, &p.d_blk_off, p.blk_off));
  TRY(upload(p, &p.d_row_elem, p.row_elem));
  TRY(upload(p, &p.d_mem_ptr, p.mem_ptr));
  TRY(upload(p, &p.d_mem_atom, p.mem_atom));
  TRY(upload(p, &p.d_mem_long, p.mem_long));
  TRY(upload(p, &p.d_pair_ptr, p.pair_ptr));
  TRY(upload(p, &p.d_pair_ab, p.pair_ab));
  TRY(upload(p, &p.d_pair_blk, p.pair_blk));
  TRY(upload(p, &p.d_fna_ptr, p.fna_ptr));
  TRY(upload(p, &p.d_fna_blk, p.fna_blk));
  TRY(upload(p, &p.d_p_rows, p.p_rows));
  TRY(upload(p, &p.d_dmax, p.dmax));
  TRY(upload(p, &p.d_order, p.order));
  TRY(upload(p, &p.d_mat_off, mat_off));
  TRY(upload(p, &p.d_vec_off, vec_off));
  TRY(upload(p, &p.d_ivec_off, ivec_off));
  TRY(dev_alloc(p, &p.d_mat, (size_t)mo));
  TRY(dev_alloc(p, &p.d_vec, (size_t)vo));
  TRY(dev_alloc(p, &p.d_ivec, (size_t)io));
  TRY(dev_alloc(p, &p.d_dim, (size_t)n_atoms));
  TRY(dev_alloc(p, &p.d_rank, (size_t)n_atoms));
  TRY(dev_alloc(p, &p.d_U, (size_t)n_atoms * ldc::kMaxOrb * ldc::kMaxOrb));
  TRY(dev_alloc(p, &p.d_lambda, (size_t)n_atoms * ldc::kMaxOrb * ldc::kMaxOrb));
  TRY(dev_alloc(p, &p.d_fixed, (size_t)n_atoms));
  TRY(dev_alloc(p, &p.d_mu, 32));
  TRY(dev_alloc(p, &p.d_partial, (size_t)(16 * p.workgroups + 2 * n_atoms)));  // mu tree partials, cluster pairs
  TRY(dev_alloc(p, &p.d_counter, 4));
  TRY(dev_alloc(p, &p.d_status, 1));
#undef TRY
  if (hipMemset(p.d_status, 0, sizeof(ldc::DevStatus)) != hipSuccess || hipMemset(p.d_mu, 0, 32 * sizeof(double)) !=
                                                                               hipSuccess ||
      hipMemset(p.d_counter, 0, 4 * sizeof(int)) != hipSuccess) {
    free_all(p);
    delete h;
    return LDC_ERR_DEVICE;
  }
  *out = h;
  return LDC_OK;
}

ldc_status ldc_regions(int n_atoms, const double *pos, const double *cell, const int *periodic, const int *n_orb,
                       int nnzb, const int *row_ptr, const int *col, const ldc_options *opt, int cap, int *member_ptr,
                       int *members, int *is_long) {
  if (n_atoms <= 0 || !pos || !cell || !periodic || !n_orb || nnzb <= 0 || !row_ptr || !col || !opt ||
      !(opt->r_L > 0.0) || !member_ptr)
    return LDC_ERR_ARG;
  Plan p;
  p.n_atoms = n_atoms;
  p.nnzb = nnzb;
  p.opt = *opt;
  p.n_orb.assign(n_orb, n_orb + n_atoms);
  p.row_ptr.assign(row_ptr, row_ptr + n_atoms + 1);
  p.col.assign(col, col + nnzb);
  if (p.row_ptr[0] != 0 || p.row_ptr[n_atoms] != nnzb) return LDC_ERR_ARG;
  ldc_status s = ldc::build_regions(p, pos, cell, periodic);
  if (s != LDC_OK) return s;
  for (int i = 0; i <= n_atoms; ++i) member_ptr[i] = p.mem_ptr[i];
  if ((int)p.mem_atom.size() > cap) return LDC_ERR_LIMIT;
  for (size_t q = 0; q < p.mem_atom.size(); ++q) {
    if (members) members[q] = p.mem_atom[q];
    if (is_long) is_long[q] = p.mem_long[q];
  }
  return LDC_OK;
}

ldc_status ldc_plan_destroy(ldc_plan_t plan) {
  if (!plan) return LDC_ERR_ARG;
  (void)hipStreamSynchronize(plan->p.stream);
  free_all(plan->p);
  delete plan;
  return LDC_OK;
}

ldc_status ldc_plan_set_stream(ldc_plan_t plan, void *stream) {
  if (!plan) return LDC_ERR_ARG;
  plan->p.stream = (hipStream_t)stream;
  return LDC_OK;
}

ldc_status ldc_plan_query(ldc_plan_t plan, ldc_plan_info *info) {
  if (!plan || !info) return LDC_ERR_ARG;
  const Plan &p = plan->p;
  info->n_atoms = p.n_atoms;
  info->n_basis = p.n_basis;
  info->nnzb = p.nnzb;
  info->max_members = p.max_members;
  info->max_dim_pao = p.max_dim;
  info->lno_mode = p.lno_mode;
  info->device_bytes = p.device_bytes;
  return LDC_OK;
}

ldc_status ldc_plan_cluster(ldc_plan_t plan, int atom, int *members, int *is_long, int *n_members, int *n_long) {
  if (!plan) return LDC_ERR_ARG;
  const Plan &p = plan->p;
  if (atom < 0 || atom >= p.n_atoms) return LDC_ERR_ARG;
  const int b = p.mem_ptr[atom], e = p.mem_ptr[atom + 1];
  int nl = 0;
  for (int q = b; q < e; ++q) {
    if (members) members[q - b] = p.mem_atom[q];
    if (is_long) is_long[q - b] = p.mem_long[q];
    nl += p.mem_long[q];
  }
  if (n_members) *n_members = e - b;
  if (n_long) *n_long = nl;
  return LDC_OK;
}

ldc_status ldc_lno(ldc_plan_t plan, const double *d_S, const double *d_Dprev, const ldc_rank_rule *rule,
                   int *ranks_out) {
  if (!plan) return LDC_ERR_ARG;
  Plan &p = plan->p;
  p.solved = 0;
  p.has_density = 0;
  if (!d_Dprev) {
    p.lno_mode = 0;
    if (ranks_out)
      for (int i = 0; i < p.n_atoms; ++i) ranks_out[i] = p.n_orb[i];
    return LDC_OK;
  }
  if (!d_S || !rule) return LDC_ERR_ARG;
  if (!p.d_lno_blk) {
    ldc_status s = dev_alloc(p, &p.d_lno_blk, (size_t)(6 * p.blk_total));
    if (s != LDC_OK) return s;
  }
  std::vector<int> fixed(p.n_atoms, -1);
  if (rule->fixed_rank)
    for (int i = 0; i < p.n_atoms; ++i) fixed[i] = rule->fixed_rank[i];
  HIPCHK(hipMemcpyAsync(p.d_fixed, fixed.data(), sizeof(int) * p.n_atoms, hipMemcpyHostToDevice, p.stream));
  stage_begin(p, 0);
  ldc::launch_lambda(p, d_S, d_Dprev);
  stage_end(p, 0);
  stage_begin(p, 1);
  ldc::launch_lno_eig(p, d_S, rule->lambda_th, rule->k_min, rule->k_max);
  stage_end(p, 1);
  HIPCHK(hipGetLastError());
  // the host copy above must not outlive this call: wait for it
  HIPCHK(hipStreamSynchronize(p.stream));
  p.lno_mode = 1;
  if (ranks_out) {
    ldc_status s = check_status(p);
    if (s != LDC_OK) return s;
    HIPCHK(hipMemcpy(ranks_out, p.d_rank, sizeof(int) * p.n_atoms, hipMemcpyDeviceToHost));
  }
  return LDC_OK;
}

ldc_status ldc_solve(ldc_plan_t plan, const double *d_H, const double *d_S) {
  if (!plan || !d_H || !d_S) return LDC_ERR_ARG;
  Plan &p = plan->p;
  stage_begin(p, 2);
  ldc::launch_gather(p, d_H, d_S);
  stage_end(p, 2);
  stage_begin(p, 3);
  ldc::launch_potrf(p);
  stage_end(p, 3);
  stage_begin(p, 4);
  ldc::launch_sygst(p);
  stage_end(p, 4);
  stage_begin(p, 5);
  ldc::launch_sy2sb(p);
  stage_end(p, 5);
  stage_begin(p, 6);
  ldc::launch_sb2st(p);
  stage_end(p, 6);
  stage_begin(p, 7);
  ldc::launch_q2x(p);
  stage_end(p, 7);
  stage_begin(p, 8);
  ldc::launch_stedc(p);
  stage_end(p, 8);
  HIPCHK(hipGetLastError());
  p.last_H = d_H;
  p.last_S = d_S;
  p.solved = 1;
  return LDC_OK;
}

static ldc_status finish_density(Plan &p, double g, double *mu_out, double *e_band_out, double *n_e_out) {
  ldc_status s = check_status(p);
  if (s != LDC_OK) return s;
  double st[32];
  HIPCHK(hipMemcpy(st, p.d_mu, sizeof(st), hipMemcpyDeviceToHost));
  if (mu_out) *mu_out = st[8];
  if (e_band_out) *e_band_out = g * st[16];
  if (n_e_out) *n_e_out = g * st[17];
  p.has_density = 1;
  return LDC_OK;
}

ldc_status ldc_density(ldc_plan_t plan, double n_electrons, double kT, double *d_D_out, double *mu_out,
                       double *e_band_out, double *n_e_out) {
  if (!plan || !d_D_out || !(kT > 0.0)) return LDC_ERR_ARG;
  Plan &p = plan->p;
  if (!p.solved) {
    p.msg = "ldc_density called before ldc_solve";
    return LDC_ERR_STATE;
  }
  const double g = p.opt.spin_g > 0 ? p.opt.spin_g : 2;
  double st[32] = {0};
  st[5] = n_electrons;
  st[6] = kT;
  st[7] = g;
  HIPCHK(hipMemcpyAsync(p.d_mu, st, sizeof(st), hipMemcpyHostToDevice, p.stream));
  stage_begin(p, 9);
  ldc::launch_mu_init(p, kT);
  int iters = 0;
  while (true) {
    for (int q = 0; q < 64 / ldc::kMuLevels; ++q) ldc::launch_mu_step(p, n_electrons, kT, g);
    iters += 64;
    HIPCHK(hipGetLastError());
    double chk[32];
    HIPCHK(hipMemcpyAsync(chk, p.d_mu, sizeof(chk), hipMemcpyDeviceToHost, p.stream));
    HIPCHK(hipStreamSynchronize(p.stream));
    if (chk[2] != 0.0 || iters >= 256) break;
  }
  stage_end(p, 9);
  stage_begin(p, 10);
  ldc::launch_density(p, ldc::kRowsDensity, d_D_out, p.last_H, p.last_S);
  stage_end(p, 10);
  HIPCHK(hipGetLastError());
  ldc_status s = finish_density(p, g, mu_out, e_band_out, n_e_out);
  if (p.profile) {
    collect_stages(p);
    p.prof_builds += 1;
  }
  return s;
}

ldc_status ldc_density_at(ldc_plan_t plan, double mu, double kT, double *d_D_out, double *e_band_out,
                          double *n_e_out) {
  if (!plan || !d_D_out || !(kT > 0.0)) return LDC_ERR_ARG;
  Plan &p = plan->p;
  if (!p.solved) {
    p.msg = "ldc_density_at called before ldc_solve";
    return LDC_ERR_STATE;
  }
  const double g = p.opt.spin_g > 0 ? p.opt.spin_g : 2;
  double st[32] = {0};
  st[2] = 1.0;
  st[6] = kT;
  st[7] = g;
  st[8] = mu;
  HIPCHK(hipMemcpyAsync(p.d_mu, st, sizeof(st), hipMemcpyHostToDevice, p.stream));
  ldc::launch_density(p, ldc::kRowsDensity, d_D_out, p.last_H, p.last_S);
  HIPCHK(hipGetLastError());
  return finish_density(p, g, nullptr, e_band_out, n_e_out);
}

ldc_status ldc_energy_density(ldc_plan_t plan, double *d_E_out, double *tr_es_out) {
  if (!plan || !d_E_out) return LDC_ERR_ARG;
  Plan &p = plan->p;
  if (!p.solved || !p.has_density) {
    p.msg = "ldc_energy_density called before a density build on the current solve";
    return LDC_ERR_STATE;
  }
  const double g = p.opt.spin_g > 0 ? p.opt.spin_g : 2;
  ldc::launch_density(p, ldc::kRowsEnergy, d_E_out, p.last_H, p.last_S);
  HIPCHK(hipGetLastError());
  if (!tr_es_out) return LDC_OK;
  ldc_status s = check_status(p);
  if (s != LDC_OK) return s;
  double st[32];
  HIPCHK(hipMemcpy(st, p.d_mu, sizeof(st), hipMemcpyDeviceToHost));
  *tr_es_out = g * st[19];
  return LDC_OK;
}

ldc_status ldc_window_density(ldc_plan_t plan, double e_lo, double e_hi, double kT, double *d_W_out,
                              double *tr_ws_out) {
  if (!plan || !d_W_out) return LDC_ERR_ARG;
  if (!(e_lo < e_hi) || !(kT > 0.0)) return LDC_ERR_ARG;
  Plan &p = plan->p;
  if (!p.solved) {
    p.msg = "ldc_window_density called before ldc_solve";
    return LDC_ERR_STATE;
  }
  const double g = p.opt.spin_g > 0 ? p.opt.spin_g : 2;
  ldc::launch_density(p, ldc::kRowsWindow, d_W_out, p.last_H, p.last_S, e_lo, e_hi, kT);
  HIPCHK(hipGetLastError());
  if (!tr_ws_out) return LDC_OK;
  ldc_status s = check_status(p);
  if (s != LDC_OK) return s;
  double st[32];
  HIPCHK(hipMemcpy(st, p.d_mu, sizeof(st), hipMemcpyDeviceToHost));
  *tr_ws_out = g * st[21];
  return LDC_OK;
}

ldc_status ldc_mulliken(ldc_plan_t plan, const double *d_D, const double *d_S, double *d_q) {
  if (!plan || !d_D || !d_S || !d_q) return LDC_ERR_ARG;
  Plan &p = plan->p;
  const double g = p.opt.spin_g > 0 ? p.opt.spin_g : 2;
  ldc::launch_mulliken(p, d_D, d_S, d_q, g);
  HIPCHK(hipGetLastError());
  return LDC_OK;
}

ldc_status ldc_potential(ldc_plan_t plan, const double *d_H0, const double *d_S, const double *d_v, double *d_H) {
  if (!plan || !d_H0 || !d_S || !d_v || !d_H) return LDC_ERR_ARG;
  Plan &p = plan->p;
  ldc::launch_potential(p, d_H0, d_S, d_v, d_H);
  HIPCHK(hipGetLastError());
  return LDC_OK;
}

ldc_status ldc_scf_mix(ldc_plan_t plan, const double *d_q_out, double *d_q_in, const double *d_q0, double U,
                       double alpha, double *d_v, double *residual_out) {
  if (!plan || !d_q_out || !d_q_in || !d_q0 || !d_v) return LDC_ERR_ARG;
  if (!(alpha >= 0.0 && alpha <= 1.0)) return LDC_ERR_ARG;
  Plan &p = plan->p;
  ldc::launch_scf_mix(p, d_q_out, d_q_in, d_q0, U, alpha, d_v, p.d_mu + kScfResidualSlot);
  HIPCHK(hipGetLastError());
  if (!residual_out) return LDC_OK;
  HIPCHK(hipStreamSynchronize(p.stream));
  HIPCHK(hipMemcpy(residual_out, p.d_mu + kScfResidualSlot, sizeof(double), hipMemcpyDeviceToHost));
  return LDC_OK;
}

ldc_status ldc_cluster_spectrum(ldc_plan_t plan, int atom, double *eps, double *w, int *dim) {
  if (!plan) return LDC_ERR_ARG;
  Plan &p = plan->p;
  if (atom < 0 || atom >= p.n_atoms) return LDC_ERR_ARG;
  if (!p.solved) return LDC_ERR_STATE;
  ldc_status s = check_status(p);
  if (s != LDC_OK) return s;
  int n = 0;
  HIPCHK(hipMemcpy(&n, p.d_dim + atom, sizeof(int), hipMemcpyDeviceToHost));
  long long voff = 0;
  HIPCHK(hipMemcpy(&voff, p.d_vec_off + atom, sizeof(long long), hipMemcpyDeviceToHost));
  const ldc::VecLayout vl = ldc::VecLayout::make(p.dmax[atom]);
  if (eps) HIPCHK(hipMemcpy(eps, p.d_vec + voff + vl.lam, sizeof(double) * n, hipMemcpyDeviceToHost));
  if (w) HIPCHK(hipMemcpy(w, p.d_vec + voff + vl.w, sizeof(double) * n, hipMemcpyDeviceToHost));
  if (dim) *dim = n;
  return LDC_OK;
}

const char *ldc_last_error(ldc_plan_t plan, int *cluster_id) {
  if (!plan) {
    if (cluster_id) *cluster_id = -1;
    return "null plan";
  }
  if (cluster_id) *cluster_id = plan->p.err_where;
  return plan->p.msg.c_str();
}

}  // extern "C"
