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
                  p.d_counter,  p.d_status,   p.d_lno_blk,  p.d_row_elem, p.d_queue};
  for (void *q : ptrs)
    if (q) (void)hipFree(q);
  for (int s = 0; s < LDC_NUM_STAGES; ++s) {
    if (p.ev_begin[s]) (void)hipEventDestroy(p.ev_begin[s]);
    if (p.ev_end[s]) (void)hipEventDestroy(p.ev_end[s]);
  }
  for (hipEvent_t e : p.tune_ev)
    if (e) (void)hipEventDestroy(e);
  p.tune_ev.clear();
  if (p.ev_fixed) (void)hipEventDestroy(p.ev_fixed);
  if (p.graph_exec) (void)hipGraphExecDestroy(p.graph_exec);
  if (p.graph) (void)hipGraphDestroy(p.graph);
  if (p.h_fixed) (void)hipHostFree(p.h_fixed);
  if (p.h_out) (void)hipHostFree(p.h_out);
  p.ev_fixed = nullptr;
  p.graph_exec = nullptr;
  p.graph = nullptr;
  p.h_fixed = nullptr;
  p.h_out = nullptr;
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

constexpr int kMaxBuckets = 4;

// Bucket edges: nb contiguous ranges of equal size of the processing order (clusters sorted by
// their plain-DC dimension, largest first); every bucket takes the largest dimension bound of
// its clusters.  Launch grids start at the stages' defaults.
void make_buckets(Plan &p, int nb) {
  nb = std::max(1, std::min(nb, std::min(kMaxBuckets, p.n_atoms)));
  p.buckets.assign(nb, ldc::Bucket{});
  for (int k = 0; k < nb; ++k) {
    ldc::Bucket &b = p.buckets[k];
    b.begin = (int)((long long)p.n_atoms * k / nb);
    const int end = (int)((long long)p.n_atoms * (k + 1) / nb);
    b.count = end - b.begin;
    b.dim_bound = 1;
    for (int q = b.begin; q < end; ++q) b.dim_bound = std::max(b.dim_bound, p.dim_bound[p.order[q]]);
  }
}

// Largest dimension every cluster can have: plain DC (all members with their orbitals), or
// LNO mode under a rank rule (a long member j contributes at most min(M_j, k_max), or
// min(M_j, fixed_j + 1) with a fixed rank: the rule that keeps a complex pair whole may add one).
void compute_dim_bounds(Plan &p, int lno, const ldc_rank_rule *rule) {
  p.dim_bound.assign(p.n_atoms, 0);
  for (int c = 0; c < p.n_atoms; ++c) {
    int d = 0;
    for (int q = p.mem_ptr[c]; q < p.mem_ptr[c + 1]; ++q) {
      const int a = p.mem_atom[q], M = p.n_orb[a];
      int k = M;
      if (lno && p.mem_long[q]) {
        const int fx = (rule && rule->fixed_rank) ? rule->fixed_rank[a] : -1;
        if (fx >= 0) k = std::min(M, fx + 1);
        else k = (rule && rule->k_max >= 0) ? std::min(M, rule->k_max) : M;
        k = std::max(k, 0);
      }
      d += k;
    }
    p.dim_bound[c] = std::max(1, std::min(d, p.dmax[c]));
  }
}

// Signature of the bucket set-up (edges, bounds, grids): part of the key of a captured build.
long long bucket_signature(const Plan &p) {
  unsigned long long h = 1469598103934665603ull;
  auto mix = [&](long long v) {
    h ^= (unsigned long long)v;
    h *= 1099511628211ull;
  };
  for (const ldc::Bucket &b : p.buckets) {
    mix(b.begin);
    mix(b.count);
    mix(b.dim_bound);
    for (int s = 0; s < ldc::kNumTuned; ++s) mix(b.grid[s]);
  }
  return (long long)h;
}

// Workload key of the tuning cache: atoms, mode and a hash of the dimension bounds.
std::string workload_key(const Plan &p, int lno) {
  unsigned long long h = 1469598103934665603ull;
  for (int c = 0; c < p.n_atoms; ++c) {
    h ^= (unsigned long long)p.dim_bound[c];
    h *= 1099511628211ull;
  }
  char buf[96];
  std::snprintf(buf, sizeof buf, "%d:%s:%016llx:p%d", p.n_atoms, lno ? "lno" : "pao", h, p.opt.prec);
  return buf;
}

std::string device_key() {
  int dev = 0, rt = 0;
  hipDeviceProp_t prop{};
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    (void)hipGetLastError();
    return "unknown";
  }
  (void)hipRuntimeGetVersion(&rt);
  // the architecture, the compute-unit count and the runtime: the marketing name is left out (it
  // reads empty under some tools, which would split one device into two keys)
  std::string name = std::string(prop.gcnArchName) + " " + std::to_string(prop.multiProcessorCount) + " CUs hip " +
                     std::to_string(rt);
  for (char &ch : name)
    if (ch == '"' || ch == '\\') ch = ' ';
  return name;
}

// Tuning cache: a JSON file with one entry per line,
//   {"device": "...", "workload": "...", "n_buckets": B, "grids": [[g0, .., g7], ...], "build_ms": T}
// Returns true and sets the buckets when an entry for this device and workload exists.
bool load_tuning(Plan &p, const char *path, const std::string &wkey) {
  if (!path || !*path) return false;
  FILE *f = std::fopen(path, "r");
  if (!f) return false;
  const std::string dkey = device_key();
  char line[4096];
  bool found = false;
  while (!found && std::fgets(line, sizeof line, f)) {
    const std::string ln(line);
    if (ln.find("\"device\": \"" + dkey + "\"") == std::string::npos) continue;
    if (ln.find("\"workload\": \"" + wkey + "\"") == std::string::npos) continue;
    const size_t nbp = ln.find("\"n_buckets\": ");
    const size_t gp = ln.find("\"grids\": [");
    if (nbp == std::string::npos || gp == std::string::npos) continue;
    const int nb = std::atoi(ln.c_str() + nbp + 13);
    if (nb < 1 || nb > kMaxBuckets) continue;
    make_buckets(p, nb);
    const char *q = ln.c_str() + gp + 10;
    bool ok = true;
    for (int b = 0; b < (int)p.buckets.size() && ok; ++b) {
      q = std::strchr(q, '[');
      if (!q) {
        ok = false;
        break;
      }
      ++q;
      for (int s = 0; s < ldc::kNumTuned; ++s) {
        char *e = nullptr;
        const long v = std::strtol(q, &e, 10);
        if (e == q) {
          ok = false;
          break;
        }
        p.buckets[b].grid[s] = (int)std::max(0L, std::min(v, 65536L));
        q = e;
        while (*q == ',' || *q == ' ') ++q;
      }
    }
    found = ok;
  }
  std::fclose(f);
  if (!found) make_buckets(p, 1);
  return found;
}

bool store_tuning(const Plan &p, const char *path, const std::string &wkey, double build_ms) {
  if (!path || !*path) return false;
  const std::string dkey = device_key();
  std::vector<std::string> keep;
  if (FILE *f = std::fopen(path, "r")) {
    char line[4096];
    while (std::fgets(line, sizeof line, f)) {
      std::string ln(line);
      if (ln.rfind("{\"device\"", 0) != 0) continue;
      if (ln.find("\"device\": \"" + dkey + "\"") != std::string::npos &&
          ln.find("\"workload\": \"" + wkey + "\"") != std::string::npos)
        continue;  // replaced below
      while (!ln.empty() && (ln.back() == '\n' || ln.back() == ',' || ln.back() == ' ')) ln.pop_back();
      keep.push_back(ln);
    }
    std::fclose(f);
  }
  std::string e = "{\"device\": \"" + dkey + "\", \"workload\": \"" + wkey +
                  "\", \"n_buckets\": " + std::to_string(p.buckets.size()) + ", \"grids\": [";
  for (size_t b = 0; b < p.buckets.size(); ++b) {
    e += (b ? ", [" : "[");
    for (int s = 0; s < ldc::kNumTuned; ++s) e += (s ? ", " : "") + std::to_string(p.buckets[b].grid[s]);
    e += "]";
  }
  char ms[64];
  std::snprintf(ms, sizeof ms, "%.3f", build_ms);
  e += std::string("], \"build_ms\": ") + ms + "}";
  keep.push_back(e);
  FILE *f = std::fopen(path, "w");
  if (!f) return false;
  std::fprintf(f, "{\"format\": \"ldc-tune-1\", \"entries\": [\n");
  for (size_t i = 0; i < keep.size(); ++i) std::fprintf(f, "%s%s\n", keep[i].c_str(), i + 1 < keep.size() ? "," : "");
  std::fprintf(f, "]}\n");
  std::fclose(f);
  return true;
}

// Buckets for the mode of the next solve: one bucket unless the plan is batched; a batched
// plan takes its launch choices from the tuning cache when it has an entry for this workload.
void prepare_buckets(Plan &p, int lno, const ldc_rank_rule *rule) {
  compute_dim_bounds(p, lno, rule);
  const std::string wkey = workload_key(p, lno);
  if (wkey == p.bucket_wkey && !p.buckets.empty()) return;  // same bounds: same buckets
  p.bucket_wkey = wkey;
  const int nb_keep = p.buckets.empty() ? 1 : (int)p.buckets.size();
  if (p.opt.batched && p.opt.tune_cache && load_tuning(p, p.opt.tune_cache, wkey)) {
    p.tune_source = "cache";
  } else if (p.opt.batched && p.tune_source == "tuned" && p.bucket_mode == lno) {
    // keep the choices of the last ldc_tune for this mode, with the new bounds
    std::vector<ldc::Bucket> old = p.buckets;
    make_buckets(p, nb_keep);
    for (size_t b = 0; b < p.buckets.size() && b < old.size(); ++b)
      for (int s = 0; s < ldc::kNumTuned; ++s) p.buckets[b].grid[s] = old[b].grid[s];
  } else {
    make_buckets(p, 1);
    p.tune_source = "default";
  }
  p.bucket_mode = lno;
}

// Tuning events around the launch of (stage, bucket).
inline void tune_begin(Plan &p, int st, int b) {
  if (p.tuning) (void)hipEventRecord(p.tune_ev[2 * (st * kMaxBuckets + b)], p.stream);
}
inline void tune_end(Plan &p, int st, int b) {
  if (p.tuning) (void)hipEventRecord(p.tune_ev[2 * (st * kMaxBuckets + b) + 1], p.stream);
}

// Runs fn for every bucket of the plan (p.cur set), with the tuning events of stage st.
template <typename F>
void for_buckets(Plan &p, int st, F fn) {
  for (size_t b = 0; b < p.buckets.size(); ++b) {
    p.cur = &p.buckets[b];
    tune_begin(p, st, (int)b);
    fn();
    tune_end(p, st, (int)b);
  }
  p.cur = nullptr;
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
      !(opt->r_L > 0.0) || (opt->prec != LDC_FP64 && opt->prec != LDC_MIXED_FP32))
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
  p.device = dev;
  // the allocation-free entry point's scratch address on this device (once per device); a
  // failure here is reported by that entry point, which retries the set-up
  {
    std::string m;
    (void)ldc::noalloc_setup(dev, m);
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
  TRY(dev_alloc(p, &p.d_queue, 2));
  TRY(dev_alloc(p, &p.d_status, 1));
#undef TRY
  if (hipMemset(p.d_status, 0, sizeof(ldc::DevStatus)) != hipSuccess || hipMemset(p.d_mu, 0, 32 * sizeof(double)) !=
                                                                               hipSuccess ||
      hipMemset(p.d_counter, 0, 4 * sizeof(int)) != hipSuccess || hipMemset(p.d_queue, 0, 2 * sizeof(int)) != hipSuccess ||
      hipHostMalloc((void **)&p.h_fixed, sizeof(int) * (size_t)n_atoms, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void **)&p.h_out, sizeof(double) * 40, hipHostMallocDefault) != hipSuccess ||
      hipEventCreateWithFlags(&p.ev_fixed, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    free_all(p);
    delete h;
    return LDC_ERR_DEVICE;
  }
  compute_dim_bounds(p, 0, nullptr);
  make_buckets(p, 1);
  p.bucket_mode = 0;
  p.tune_source = "default";
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
  info->blk_total = p.blk_total;
  info->n_buckets = (int)p.buckets.size();
  info->tuned = p.tune_source == "cache" ? 2 : (p.tune_source == "tuned" ? 1 : 0);
  info->graph_captures = p.graph_captures;
  info->graph_replays = p.graph_builds;
  return LDC_OK;
}

ldc_status ldc_plan_buckets(ldc_plan_t plan, int *begin, int *count, int *dim_bound, int *grids) {
  if (!plan) return LDC_ERR_ARG;
  const Plan &p = plan->p;
  for (size_t b = 0; b < p.buckets.size(); ++b) {
    if (begin) begin[b] = p.buckets[b].begin;
    if (count) count[b] = p.buckets[b].count;
    if (dim_bound) dim_bound[b] = p.buckets[b].dim_bound;
    if (grids)
      for (int s = 0; s < ldc::kNumTuned; ++s) grids[b * ldc::kNumTuned + s] = p.buckets[b].grid[s];
  }
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

}  // extern "C"

namespace {

ldc_status ensure_lno_blocks(Plan &p) {
  if (p.d_lno_blk) return LDC_OK;
  return dev_alloc(p, &p.d_lno_blk, (size_t)(6 * p.blk_total));
}

// The device part of ldc_lno, stream-ordered, no host synchronization: the fixed ranks go
// through the plan's pinned buffer (or a fill kernel when there are none).
ldc_status enqueue_lno(Plan &p, const double *d_S, const double *d_Dprev, const ldc_rank_rule *rule,
                       bool capturing = false) {
  p.solved = 0;
  p.has_density = 0;
  if (!d_Dprev) {
    p.lno_mode = 0;
    return LDC_OK;
  }
  ldc_status st = ensure_lno_blocks(p);
  if (st != LDC_OK) return st;
  if (rule->fixed_rank) {
    if (capturing) {
      // the captured copy reads the staging buffer, which ldc_build fills before every launch
      HIPCHK(hipMemcpyAsync(p.d_fixed, p.h_fixed, sizeof(int) * p.n_atoms, hipMemcpyHostToDevice, p.stream));
    } else {
      // the previous copy out of the staging buffer must be done before it is overwritten
      HIPCHK(hipEventSynchronize(p.ev_fixed));
      std::memcpy(p.h_fixed, rule->fixed_rank, sizeof(int) * p.n_atoms);
      HIPCHK(hipMemcpyAsync(p.d_fixed, p.h_fixed, sizeof(int) * p.n_atoms, hipMemcpyHostToDevice, p.stream));
      HIPCHK(hipEventRecord(p.ev_fixed, p.stream));
    }
  } else {
    ldc::launch_fill_int(p, p.d_fixed, p.n_atoms, -1);
  }
  stage_begin(p, 0);
  ldc::launch_lambda(p, d_S, d_Dprev);
  stage_end(p, 0);
  stage_begin(p, 1);
  ldc::launch_lno_eig(p, d_S, rule->lambda_th, rule->k_min, rule->k_max);
  stage_end(p, 1);
  HIPCHK(hipGetLastError());
  p.lno_mode = 1;
  return LDC_OK;
}

ldc_status enqueue_solve(Plan &p, const double *d_H, const double *d_S) {
  if (p.lno_mode) ldc::launch_lno_blocks(p, d_H, d_S);
  stage_begin(p, 2);
  for_buckets(p, ldc::kTGather, [&] { ldc::launch_gather(p, d_H, d_S); });
  stage_end(p, 2);
  stage_begin(p, 3);
  for_buckets(p, ldc::kTPotrf, [&] { ldc::launch_potrf(p); });
  stage_end(p, 3);
  stage_begin(p, 4);
  for_buckets(p, ldc::kTSygst, [&] { ldc::launch_sygst(p); });
  stage_end(p, 4);
  stage_begin(p, 5);
  for_buckets(p, ldc::kTSy2sb, [&] { ldc::launch_sy2sb(p); });
  stage_end(p, 5);
  stage_begin(p, 6);
  for_buckets(p, ldc::kTSb2st, [&] { ldc::launch_sb2st(p); });
  stage_end(p, 6);
  stage_begin(p, 7);
  for_buckets(p, ldc::kTQ2x, [&] { ldc::launch_q2x(p); });
  stage_end(p, 7);
  stage_begin(p, 8);
  for_buckets(p, ldc::kTStedc, [&] { ldc::launch_stedc(p); });
  stage_end(p, 8);
  HIPCHK(hipGetLastError());
  p.last_H = d_H;
  p.last_S = d_S;
  p.solved = 1;
  return LDC_OK;
}

// Rows of one mode for every bucket, then their trace sums.
void enqueue_rows(Plan &p, int mode, double *d_out, double w_lo = 0.0, double w_hi = 0.0, double w_kT = 1.0) {
  for_buckets(p, ldc::kTDensity, [&] { ldc::launch_density(p, mode, d_out, p.last_H, p.last_S, w_lo, w_hi, w_kT); });
  ldc::launch_density_sums(p, mode);
}

ldc_status enqueue_density(Plan &p, double n_electrons, double kT, double *d_D_out);

}  // namespace

// The device part of ldc_density (state set-up, bisection, rows and their sums) on the
// plan's current scratch pointers; used by the allocation-free entry point.
ldc_status ldc::enqueue_density_steps(Plan &p, double n_electrons, double kT, double *d_D_out) {
  return enqueue_density(p, n_electrons, kT, d_D_out);
}

namespace {

// The bisection (a fixed number of launches; those after convergence return at once) and the
// density rows.
ldc_status enqueue_density(Plan &p, double n_electrons, double kT, double *d_D_out) {
  const double g = p.opt.spin_g > 0 ? p.opt.spin_g : 2;
  ldc::launch_state_init(p, n_electrons, kT, g, 0, 0.0);
  stage_begin(p, 9);
  ldc::launch_mu_init(p, kT);
  for (int q = 0; q < ldc::kMuLaunches; ++q) ldc::launch_mu_step(p, n_electrons, kT, g);
  stage_end(p, 9);
  stage_begin(p, 10);
  enqueue_rows(p, ldc::kRowsDensity, d_D_out);
  stage_end(p, 10);
  HIPCHK(hipGetLastError());
  return LDC_OK;
}

ldc_status finish_density(Plan &p, double g, double *mu_out, double *e_band_out, double *n_e_out) {
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

}  // namespace

extern "C" {

ldc_status ldc_lno(ldc_plan_t plan, const double *d_S, const double *d_Dprev, const ldc_rank_rule *rule,
                   int *ranks_out) {
  if (!plan) return LDC_ERR_ARG;
  Plan &p = plan->p;
  if (d_Dprev && (!d_S || !rule)) return LDC_ERR_ARG;
  prepare_buckets(p, d_Dprev ? 1 : 0, rule);
  ldc_status s = enqueue_lno(p, d_S, d_Dprev, rule);
  if (s != LDC_OK) return s;
  if (ranks_out) {
    if (!d_Dprev) {
      for (int i = 0; i < p.n_atoms; ++i) ranks_out[i] = p.n_orb[i];
      return LDC_OK;
    }
    s = check_status(p);
    if (s != LDC_OK) return s;
    HIPCHK(hipMemcpy(ranks_out, p.d_rank, sizeof(int) * p.n_atoms, hipMemcpyDeviceToHost));
  }
  return LDC_OK;
}

ldc_status ldc_solve(ldc_plan_t plan, const double *d_H, const double *d_S) {
  if (!plan || !d_H || !d_S) return LDC_ERR_ARG;
  return enqueue_solve(plan->p, d_H, d_S);
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
  ldc_status s = enqueue_density(p, n_electrons, kT, d_D_out);
  if (s != LDC_OK) return s;
  s = finish_density(p, g, mu_out, e_band_out, n_e_out);
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
  ldc::launch_state_init(p, 0.0, kT, g, 1, mu);
  enqueue_rows(p, ldc::kRowsDensity, d_D_out);
  HIPCHK(hipGetLastError());
  return finish_density(p, g, nullptr, e_band_out, n_e_out);
}

}  // extern "C"

namespace {

// Reads the status word and state that a captured build copied to the pinned buffer.
ldc_status finish_graph_build(Plan &p, double g, double *mu_out, double *e_band_out, double *n_e_out) {
  int code = 0, where = -1;
  std::memcpy(&code, p.h_out + 32, sizeof(int));
  std::memcpy(&where, reinterpret_cast<const char *>(p.h_out + 32) + sizeof(int), sizeof(int));
  if (code != 0) {
    static const char *names[] = {"ok", "bad argument", "overlap matrix not positive definite",
                                  "eigensolver did not converge", "electron count outside the bracket",
                                  "LNO basis rank deficient", "out of memory", "device error", "state",
                                  "limit exceeded"};
    p.msg = std::string(code >= 0 && code < 10 ? names[code] : "error") + " (cluster/atom " + std::to_string(where) +
            ")";
    p.err_where = where;
    ldc::DevStatus zero{0, -1};
    HIPCHK(hipMemcpy(p.d_status, &zero, sizeof(zero), hipMemcpyHostToDevice));
    return (ldc_status)code;
  }
  if (mu_out) *mu_out = p.h_out[8];
  if (e_band_out) *e_band_out = g * p.h_out[16];
  if (n_e_out) *n_e_out = g * p.h_out[17];
  p.has_density = 1;
  return LDC_OK;
}

ldc_status eager_build(Plan &p, const double *d_H, const double *d_S, const double *d_Dprev, const ldc_rank_rule *rule,
                       double n_electrons, double kT, double *d_D_out, double *mu_out, double *e_band_out,
                       double *n_e_out) {
  const double g = p.opt.spin_g > 0 ? p.opt.spin_g : 2;
  ldc_status s = enqueue_lno(p, d_S, d_Dprev, rule);
  if (s == LDC_OK) s = enqueue_solve(p, d_H, d_S);
  if (s == LDC_OK) s = enqueue_density(p, n_electrons, kT, d_D_out);
  if (s != LDC_OK) return s;
  s = finish_density(p, g, mu_out, e_band_out, n_e_out);
  if (p.profile) {
    collect_stages(p);
    p.prof_builds += 1;
  }
  return s;
}

}  // namespace

extern "C" {

ldc_status ldc_build(ldc_plan_t plan, const double *d_H, const double *d_S, const double *d_Dprev,
                     const ldc_rank_rule *rule, double n_electrons, double kT, double *d_D_out, double *mu_out,
                     double *e_band_out, double *n_e_out) {
  if (!plan || !d_H || !d_S || !d_D_out || !(kT > 0.0) || (d_Dprev && !rule)) return LDC_ERR_ARG;
  Plan &p = plan->p;
  const double g = p.opt.spin_g > 0 ? p.opt.spin_g : 2;
  prepare_buckets(p, d_Dprev ? 1 : 0, rule);
  // a graph is captured on the plan's own stream; the legacy default stream cannot be captured
  if (!p.opt.use_graph || p.profile || p.tuning || p.stream == nullptr)
    return eager_build(p, d_H, d_S, d_Dprev, rule, n_electrons, kT, d_D_out, mu_out, e_band_out, n_e_out);
  if (d_Dprev) {
    ldc_status s = ensure_lno_blocks(p);
    if (s != LDC_OK) return s;
  }
  // the copy node of a captured build reads the fixed ranks from the staging buffer (the
  // previous build has finished: every ldc_build ends with a synchronization)
  if (d_Dprev && rule->fixed_rank) std::memcpy(p.h_fixed, rule->fixed_rank, sizeof(int) * p.n_atoms);
  ldc::BuildKey key;
  key.H = d_H;
  key.S = d_S;
  key.Dprev = d_Dprev;
  key.Dout = d_D_out;
  if (d_Dprev) {
    key.lambda_th = rule->lambda_th;
    key.k_min = rule->k_min;
    key.k_max = rule->k_max;
    key.has_fixed = rule->fixed_rank ? 1 : 0;
  }
  key.n_e = n_electrons;
  key.kT = kT;
  key.prec = p.opt.prec;
  key.bucket_sig = bucket_signature(p);
  key.stream = p.stream;
  if (!p.graph_exec || !(key == p.graph_key)) {
    if (p.graph_exec) (void)hipGraphExecDestroy(p.graph_exec);
    if (p.graph) (void)hipGraphDestroy(p.graph);
    p.graph_exec = nullptr;
    p.graph = nullptr;
    HIPCHK(hipStreamSynchronize(p.stream));
    HIPCHK(hipStreamBeginCapture(p.stream, hipStreamCaptureModeThreadLocal));
    ldc_status s = enqueue_lno(p, d_S, d_Dprev, rule, true);
    if (s == LDC_OK) s = enqueue_solve(p, d_H, d_S);
    if (s == LDC_OK) s = enqueue_density(p, n_electrons, kT, d_D_out);
    if (s == LDC_OK) {
      // state and status word out to the pinned buffer, inside the graph
      if (hipMemcpyAsync(p.h_out, p.d_mu, sizeof(double) * 32, hipMemcpyDeviceToHost, p.stream) != hipSuccess ||
          hipMemcpyAsync(p.h_out + 32, p.d_status, sizeof(ldc::DevStatus), hipMemcpyDeviceToHost, p.stream) !=
              hipSuccess) {
        p.msg = "copy to the staging buffer could not be captured";
        s = LDC_ERR_DEVICE;
      }
    }
    hipGraph_t gr = nullptr;
    const hipError_t e = hipStreamEndCapture(p.stream, &gr);
    if (s != LDC_OK || e != hipSuccess) {
      if (gr) (void)hipGraphDestroy(gr);
      (void)hipGetLastError();
      if (s == LDC_OK) p.msg = std::string("graph capture failed: ") + hipGetErrorString(e);
      return s != LDC_OK ? s : LDC_ERR_DEVICE;
    }
    hipGraphExec_t ex = nullptr;
    const hipError_t ei = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
    if (ei != hipSuccess) {
      (void)hipGraphDestroy(gr);
      (void)hipGetLastError();
      p.msg = std::string("graph instantiation failed: ") + hipGetErrorString(ei);
      return LDC_ERR_DEVICE;
    }
    p.graph = gr;
    p.graph_exec = ex;
    p.graph_key = key;
    p.graph_captures += 1;
  } else {
    // the host state that the captured sequence set when it was recorded
    p.lno_mode = d_Dprev ? 1 : 0;
    p.last_H = d_H;
    p.last_S = d_S;
    p.solved = 1;
  }
  HIPCHK(hipGraphLaunch(p.graph_exec, p.stream));
  HIPCHK(hipStreamSynchronize(p.stream));
  p.graph_builds += 1;
  return finish_graph_build(p, g, mu_out, e_band_out, n_e_out);
}

ldc_status ldc_tune(ldc_plan_t plan, const double *d_H, const double *d_S, const double *d_Dprev,
                    const ldc_rank_rule *rule, double n_electrons, double kT, double *d_D_out, double *best_ms_out) {
  if (!plan || !d_H || !d_S || !d_D_out || !(kT > 0.0) || (d_Dprev && !rule)) return LDC_ERR_ARG;
  Plan &p = plan->p;
  const int lno = d_Dprev ? 1 : 0;
  if (p.tune_ev.empty()) {
    p.tune_ev.assign(2 * ldc::kNumTuned * kMaxBuckets, nullptr);
    for (hipEvent_t &e : p.tune_ev) HIPCHK(hipEventCreate(&e));
  }
  hipEvent_t t0 = nullptr, t1 = nullptr;
  HIPCHK(hipEventCreate(&t0));
  HIPCHK(hipEventCreate(&t1));
  const int saved_profile = p.profile;
  p.profile = 0;
  compute_dim_bounds(p, lno, rule);
  const std::string wkey = workload_key(p, lno);
  // one build with the launches as set; returns its time (ms) or < 0 on error
  auto run = [&](ldc_status &st) -> double {
    (void)hipEventRecord(t0, p.stream);
    st = enqueue_lno(p, d_S, d_Dprev, rule);
    if (st == LDC_OK) st = enqueue_solve(p, d_H, d_S);
    if (st == LDC_OK) st = enqueue_density(p, n_electrons, kT, d_D_out);
    (void)hipEventRecord(t1, p.stream);
    if (st == LDC_OK) st = check_status(p);
    float ms = -1.f;
    if (st == LDC_OK && hipEventElapsedTime(&ms, t0, t1) != hipSuccess) st = LDC_ERR_DEVICE;
    return ms;
  };
  constexpr int kCand = 4;  // candidate grids: 1..4 workgroups per CU
  ldc_status st = LDC_OK;
  double best_ms = 1e300;
  std::vector<ldc::Bucket> best;
  for (int nb = 1; nb <= kMaxBuckets && st == LDC_OK; ++nb) {
    if (nb > 1 && p.n_atoms / nb < 2 * p.n_cu) break;  // a bucket must still fill the GPU
    make_buckets(p, nb);
    std::vector<float> t((size_t)ldc::kNumTuned * nb * kCand, 1e30f);
    p.tuning = 1;
    for (int ci = 0; ci < kCand && st == LDC_OK; ++ci) {
      for (ldc::Bucket &b : p.buckets)
        for (int s = 0; s < ldc::kNumTuned; ++s) b.grid[s] = (ci + 1) * p.n_cu;
      run(st);
      if (st != LDC_OK) break;
      for (int s = 0; s < ldc::kNumTuned; ++s)
        for (int b = 0; b < nb; ++b) {
          float ms = 0.f;
          if (hipEventElapsedTime(&ms, p.tune_ev[2 * (s * kMaxBuckets + b)], p.tune_ev[2 * (s * kMaxBuckets + b) + 1]) ==
              hipSuccess)
            t[((size_t)s * nb + b) * kCand + ci] = ms;
          else
            (void)hipGetLastError();
        }
    }
    p.tuning = 0;
    if (st != LDC_OK) break;
    for (int s = 0; s < ldc::kNumTuned; ++s)
      for (int b = 0; b < nb; ++b) {
        int bc = 0;
        for (int ci = 1; ci < kCand; ++ci)
          if (t[((size_t)s * nb + b) * kCand + ci] < t[((size_t)s * nb + b) * kCand + bc]) bc = ci;
        p.buckets[b].grid[s] = (bc + 1) * p.n_cu;
      }
    double ms = 1e300;
    for (int rep = 0; rep < 2 && st == LDC_OK; ++rep) ms = std::min(ms, run(st));
    if (st == LDC_OK && ms < best_ms) {
      best_ms = ms;
      best = p.buckets;
    }
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  p.tuning = 0;
  p.profile = saved_profile;
  if (st != LDC_OK) {
    make_buckets(p, 1);
    p.tune_source = "default";
    p.bucket_wkey.clear();
    return st;
  }
  p.buckets = best;
  p.tune_source = "tuned";
  p.bucket_mode = lno;
  p.bucket_wkey = wkey;
  if (p.opt.tune_cache && !store_tuning(p, p.opt.tune_cache, wkey, best_ms)) {
    p.msg = std::string("could not write the tuning cache ") + p.opt.tune_cache;
    return LDC_ERR_ARG;
  }
  if (best_ms_out) *best_ms_out = best_ms;
  return LDC_OK;
}

ldc_status ldc_reference_populations(ldc_plan_t plan, double n_electrons, double *d_q0) {
  if (!plan || !d_q0) return LDC_ERR_ARG;
  Plan &p = plan->p;
  ldc::launch_reference_populations(p, n_electrons, d_q0);
  HIPCHK(hipGetLastError());
  return LDC_OK;
}

ldc_status ldc_energy_density(ldc_plan_t plan, double *d_E_out, double *tr_es_out) {
  if (!plan || !d_E_out) return LDC_ERR_ARG;
  Plan &p = plan->p;
  if (!p.solved || !p.has_density) {
    p.msg = "ldc_energy_density called before a density build on the current solve";
    return LDC_ERR_STATE;
  }
  const double g = p.opt.spin_g > 0 ? p.opt.spin_g : 2;
  enqueue_rows(p, ldc::kRowsEnergy, d_E_out);
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
  enqueue_rows(p, ldc::kRowsWindow, d_W_out, e_lo, e_hi, kT);
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
