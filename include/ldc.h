/*
 * ldc.h -- C ABI of the MI355X (gfx950) DC-LNO density-build library (libldc.so).
 *
 * Method: O(N) divide-conquer with localized natural orbitals (Ozaki, Fukuda & Jiang,
 * arXiv 1809.05637).  For every atom i a truncated cluster (all atoms within r_L) is
 * solved as a small generalized eigenproblem; atoms far from i (the long region) are
 * represented by a few LNOs each; one chemical potential is shared by all clusters and
 * atom i's density-matrix rows come from its own cluster.
 *
 * Matrix layout shared by every entry point (H, S, previous and output density):
 *   variable-size block-sparse rows, one block per atom pair, images folded onto the pair
 *   (Gamma-point supercell).  Row i holds blocks (i, j) for j in the structural overlap
 *   pattern of i, j ascending, the diagonal block included; the pattern is symmetric.
 *   Block (i, j) is an M_i x M_j row-major float64 array; blocks are stored back to back
 *   in row order, so block b starts at the prefix sum of the sizes of blocks 0..b-1.
 *   H and S must be symmetric (H_ji = H_ij^T) and S positive definite.
 *
 * Memory: pointers named d_* are device pointers owned by the caller; the library never
 * frees or writes caller inputs.  All other pointers are host pointers.  The plan owns
 * its device workspaces (cluster matrices, LNO table, spectra, tracked projections).
 *
 * Ordering: every call is enqueued on the plan's HIP stream (set at creation or with
 * ldc_plan_set_stream) in call order.  ldc_lno (without ranks_out) and ldc_solve never wait
 * for the device; entry points that return host values (ranks_out, mu_out, ...) synchronize
 * that stream once, before returning.  Errors raised inside kernels (non-positive Cholesky
 * pivot, unconverged eigensolver, ...) are reported by the next call that synchronizes;
 * ldc_last_error then names the first failing cluster/atom.
 *
 * Errors: functions return ldc_status; nothing is thrown across the ABI.  After an error
 * the plan stays usable for new calls.
 */
#ifndef LDC_H
#define LDC_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ldc_plan_s *ldc_plan_t;

typedef enum {
  LDC_OK = 0,
  LDC_ERR_ARG = 1,          /* invalid argument (null pointer, bad size, bad pattern) */
  LDC_ERR_NOT_SPD = 2,      /* a cluster overlap matrix has a non-positive Cholesky pivot */
  LDC_ERR_EIG_NOCONV = 3,   /* an eigensolver (Lambda or cluster) did not converge */
  LDC_ERR_MU_BRACKET = 4,   /* electron count outside (0, g * sum of weights) */
  LDC_ERR_RANK = 5,         /* an LNO basis is rank deficient or a rank is out of range */
  LDC_ERR_OOM = 6,          /* device memory allocation failed */
  LDC_ERR_DEVICE = 7,       /* a HIP runtime call failed */
  LDC_ERR_STATE = 8,        /* call order violated (e.g. ldc_density before ldc_solve) */
  LDC_ERR_LIMIT = 9         /* a size exceeds a compiled limit (orbitals per atom, members) */
} ldc_status;

/* Plan options.  Zero-initialised fields take the defaults shown, except r_L (required) and
 * kappa (0 is a valid buffer fraction: the short region is then F_i plus the shells needed to
 * reach N_F; pass a negative kappa for the paper's 0.3). */
typedef enum {
  LDC_FP64 = 0,        /* every step in FP64 */
  LDC_MIXED_FP32 = 1   /* precision form: FP32 storage and products where the method allows it
                          (see ldc_build); Cholesky, tridiagonal eigensolve and mu in FP64 */
} ldc_precision;

typedef struct {
  double r_L;          /* cluster radius (same length unit as the positions); required > 0 */
  double kappa;        /* buffer fraction of the short region, Sec. III (iii); < 0 -> 0.3 */
  double dist_tol;     /* relative tolerance for sphere membership; 0 -> 1e-9 */
  double shell_tol;    /* relative tolerance grouping equal distances into shells; 0 -> 1e-8 */
  int spin_g;          /* spin factor g in N_e = g Tr(D S) (Eq. 13); 0 -> 2 */
  int workgroups;      /* persistent workgroups per per-cluster kernel; 0 -> 2 x CUs */
  int prec;            /* ldc_precision; 0 -> LDC_FP64 */
  int batched;         /* 1: size buckets with launch choices from the tuning cache (ldc_tune);
                          0: one launch per stage over all clusters with the default grids */
  int use_graph;       /* 1: ldc_build captures a whole build into a HIP graph on its first call
                          and replays it while pointers and parameters stay the same */
  const char *tune_cache;  /* path of the tuning cache (JSON) read when batched, written by
                              ldc_tune; NULL: none.  The string must outlive the plan. */
} ldc_options;

/* LNO rank rule (Sec. II.B step (iii), Eq. 22): k_j = clamp(#{Re lambda >= lambda_th},
 * k_min, k_max); a cut through a complex-conjugate pair of eigenvalues moves past the pair
 * (or before it when k_max forbids).  fixed_rank (host, n_atoms entries, or NULL): entries
 * >= 0 replace the count for that atom (the pair rule still applies). */
typedef struct {
  double lambda_th;
  int k_min;
  int k_max;               /* < 0: M_j */
  const int *fixed_rank;
} ldc_rank_rule;

typedef struct {
  int n_atoms;
  int n_basis;             /* sum of M_i */
  int nnzb;                /* number of blocks in the pattern */
  int max_members;         /* largest cluster (atoms) */
  int max_dim_pao;         /* largest cluster dimension with PAOs everywhere (plain DC) */
  int lno_mode;            /* 1 after ldc_lno with a previous density, 0 for plain DC */
  size_t device_bytes;     /* device memory held by the plan */
  long long blk_total;     /* doubles in one block-sparse matrix (the length of H, S and D) */
  int n_buckets;           /* size buckets of the current mode */
  int tuned;               /* launch choices: 0 defaults, 1 from ldc_tune, 2 from the cache */
  int graph_captures;      /* builds captured into a HIP graph by ldc_build */
  int graph_replays;       /* ldc_build calls that launched a captured graph */
} ldc_plan_info;

/* Build the per-geometry plan (Sec. III (i)-(iv)): cluster of every atom (all atoms within
 * r_L by minimum-image distance on periodic axes), first neighbours F_i = the pattern row
 * of i, short region = smallest neighbour shell holding >= N_F + kappa N_S atoms (F_i always
 * short), long region = the rest.  Uploads the index tables and allocates the workspaces.
 *   pos: n_atoms x 3 positions; cell: 3 x 3 row-major lattice (only the diagonal is used:
 *   orthorhombic cells); periodic: 3 flags; n_orb: M_i (1..16); row_ptr (n_atoms+1) and
 *   col (nnzb): the block pattern; stream: hipStream_t or NULL for the default stream. */
ldc_status ldc_plan_create(ldc_plan_t *out, int n_atoms, const double *pos, const double *cell,
                           const int *periodic, const int *n_orb, int nnzb, const int *row_ptr,
                           const int *col, const ldc_options *opt, void *stream);
ldc_status ldc_plan_destroy(ldc_plan_t plan);
ldc_status ldc_plan_set_stream(ldc_plan_t plan, void *stream);
ldc_status ldc_plan_query(ldc_plan_t plan, ldc_plan_info *info);

/* The size buckets of the current mode (host arrays of n_buckets entries, any may be NULL):
 * the range [begin, begin + count) of the processing order (clusters by plain-DC dimension,
 * largest first), the largest dimension its clusters can have, and the launch grids of the
 * eight bucketed stages (gather, Cholesky, standard form, band reduction, bulge chasing,
 * second-stage transform, tridiagonal eigensolve, density rows; 0 = default), row-major
 * n_buckets x 8. */
ldc_status ldc_plan_buckets(ldc_plan_t plan, int *begin, int *count, int *dim_bound, int *grids);

/* Host-only planner (no device work, no GPU needed): the members of every atom's cluster,
 * exactly as ldc_plan_create computes them, in the library's member order.
 *   member_ptr: host array of n_atoms + 1 offsets; members, is_long: host arrays of capacity
 *   cap.  Returns LDC_ERR_LIMIT (and the needed size in member_ptr[n_atoms]) if cap is too
 *   small. */
ldc_status ldc_regions(int n_atoms, const double *pos, const double *cell, const int *periodic, const int *n_orb,
                       int nnzb, const int *row_ptr, const int *col, const ldc_options *opt, int cap,
                       int *member_ptr, int *members, int *is_long);

/* Members of atom's cluster in the library's order (long atoms, short atoms outside F_i,
 * F_i without i, then i).  members/is_long: host arrays of capacity >= max_members;
 * n_members, n_long: host scalars.  Any output pointer may be NULL. */
ldc_status ldc_plan_cluster(ldc_plan_t plan, int atom, int *members, int *is_long, int *n_members,
                            int *n_long);

/* (b) LNOs (Sec. II.B (i)-(iii)): Lambda_j = sum_k rho_jk S_kj (Eq. 17), its nonsymmetric
 * eigendecomposition (Eq. 20) via Hessenberg reduction and Francis double-shift QR, the
 * kept span of eigenvalues ranked by real part (Eq. 22, rank rule above), made
 * S_jj-orthonormal.  d_Dprev == NULL selects plain DC (no long region) for the next
 * ldc_solve.  ranks_out (host, n_atoms) may be NULL; when given, the call synchronizes. */
ldc_status ldc_lno(ldc_plan_t plan, const double *d_S, const double *d_Dprev, const ldc_rank_rule *rule,
                   int *ranks_out);

/* (a)+(c)+(d): gather every cluster's H^(i), S^(i) with PAO-PAO, PAO-LNO and LNO-LNO
 * blocks (Eq. 26) and solve H^(i) c = eps S^(i) c (Sec. II.C (ii)-(iii)): Cholesky of S^(i),
 * reduction to standard form, Householder tridiagonalization and divide-and-conquer on the
 * tridiagonal matrix.  Keeps eps^(i), the centre weights w_mu = sum_{alpha in i}
 * c_{i alpha,mu} (S^(i) c_mu)_{i alpha} and what the density rows need inside the plan. */
ldc_status ldc_solve(ldc_plan_t plan, const double *d_H, const double *d_S);

/* (e): common chemical potential by bisection on N(mu) = g sum_i sum_mu f((eps-mu)/kT) w
 * (Sec. II.C (iv)) from [min eps - 40 kT, max eps + 40 kT] until hi - lo <= 4e-16 max(1,|mid|)
 * (at most 200 halvings), then density rows rho_{i alpha, j beta} = sum_mu f c_{i alpha,mu}
 * c_{j beta,mu} for every j in the pattern row of i (Eq. 24 with Eq. 27) written to d_D_out
 * (same layout as S).  e_band = g sum_ij tr(D_ij H_ji) needs the H passed to ldc_solve
 * (still valid on the device); n_e = g Tr(D S).  Synchronizes. */
ldc_status ldc_density(ldc_plan_t plan, double n_electrons, double kT, double *d_D_out, double *mu_out,
                       double *e_band_out, double *n_e_out);

/* One whole density build (Sec. II.C (i)-(v)): ldc_lno from d_Dprev (NULL: plain DC) with
 * the rank rule, ldc_solve and ldc_density, enqueued without host waits and synchronized once
 * at the end (mu, e_band, n_e to the host).  The chemical-potential bisection runs as a fixed
 * number of launches that stop advancing once converged, so the whole sequence is
 * stream-ordered.  With opt.use_graph the sequence is captured into a HIP graph on the first
 * call (on a plan whose stream is not the default stream; on the default stream the build runs
 * eagerly) and replayed by later calls with the same pointers, rank-rule parameters, n_electrons,
 * kT and bucket set-up (the fixed ranks themselves may change between calls); anything else
 * re-captures.  With opt.batched every bucketed stage is launched once per size bucket with
 * the bucket's tuned grid.  Same outputs and errors as ldc_density. */
ldc_status ldc_build(ldc_plan_t plan, const double *d_H, const double *d_S, const double *d_Dprev,
                     const ldc_rank_rule *rule, double n_electrons, double kT, double *d_D_out, double *mu_out,
                     double *e_band_out, double *n_e_out);

/* Autotuner of the batched form: for 1..4 size buckets (equal shares of the processing
 * order, each still holding >= 2 x CUs clusters) it times every bucketed stage per bucket
 * with 1, 2, 3 and 4 workgroups per CU (one whole build per candidate, HIP events around
 * every launch), keeps the fastest grid of each (stage, bucket), times the combination
 * (best of two whole builds), and keeps the bucket count with the fastest build.  The choice
 * stays in the plan for this mode and, when opt.tune_cache is set, is written there keyed by
 * device, HIP runtime version and workload (atom count, mode and the clusters' dimension
 * bounds).  Runs 6 whole builds per bucket count tried with the given inputs (d_D_out is
 * overwritten);
 * best_ms_out (host, may be NULL) receives the tuned build time.  Synchronizes. */
ldc_status ldc_tune(ldc_plan_t plan, const double *d_H, const double *d_S, const double *d_Dprev,
                    const ldc_rank_rule *rule, double n_electrons, double kT, double *d_D_out, double *best_ms_out);

/* For callers that cannot allocate device memory or wait for the device (code under HIP graph
 * capture, tight serving loops): ldc_density without any allocation and without a host
 * synchronization.  The bisection state, the workgroups' ticket counter, their partial sums
 * and the per-cluster row sums live in one file-scope device array of the library (1.3 MB,
 * present on every GPU the library runs on until the process ends) instead of the plan's
 * buffers; mu, E_band and N_e go to d_result (device, 3 doubles, in that order).  The density
 * rows, mu, E_band and N_e equal ldc_density's for the same solve.  Limits: at most 65536
 * atoms and 2048 workgroups per plan, else LDC_ERR_LIMIT with a message.  All calls on one GPU
 * share the array: calls that overlap in time on one GPU (two streams, two threads) race.  The
 * density kernel's cluster work queue is the plan's own (allocated with the plan), so calls on
 * one plan must not overlap either.  Errors inside kernels are reported by the next call that
 * synchronizes. */
ldc_status ldc_density_noalloc(ldc_plan_t plan, double n_electrons, double kT, double *d_D_out, double *d_result);

/* Density rows at a given chemical potential (no bisection); otherwise as ldc_density. */
ldc_status ldc_density_at(ldc_plan_t plan, double mu, double kT, double *d_D_out, double *e_band_out,
                          double *n_e_out);

/* Energy density matrix rows (Eq. 25 with Eq. 27, the energy-weighted integral of the
 * cluster's spectral Green function): e_{i alpha, j beta} = sum_mu f eps c_{i alpha,mu}
 * c_{j beta,mu} for every j in the pattern row of i, written to d_E_out (same layout as S),
 * at the chemical potential and kT of the last ldc_density / ldc_density_at call, from the
 * spectra and tracked projections the plan keeps (no new eigensolve).  tr_es_out (host, may
 * be NULL): g Tr(E S), which equals g sum_i sum_mu f eps w = E_band since F_i lies in the
 * short region; when given, the call synchronizes.  LDC_ERR_STATE if no density was built
 * since the last ldc_solve. */
ldc_status ldc_energy_density(ldc_plan_t plan, double *d_E_out, double *tr_es_out);

/* Energy-window density rows (Sec. II.B: the projector that defines Lambda may select another
 * energy window than the occupied states, e.g. bands near the Fermi level):
 *   W_{i alpha, j beta} = sum_mu w(eps) c_{i alpha,mu} c_{j beta,mu},
 *   w(eps) = f((eps - e_hi)/kT) - f((eps - e_lo)/kT)   (f the Fermi function: a smooth box),
 * for every j in the pattern row of i, written to d_W_out (same layout as S), from the spectra
 * and tracked projections of the last ldc_solve (no chemical potential needed).  Passing d_W_out
 * to ldc_lno as the previous density gives energy-window LNOs.  tr_ws_out (host, may be NULL):
 * g Tr(W S), the window's state count g sum_i sum_mu w(eps) w_mu; when given, the call
 * synchronizes.  LDC_ERR_ARG unless e_lo < e_hi and kT > 0; LDC_ERR_STATE before ldc_solve. */
ldc_status ldc_window_density(ldc_plan_t plan, double e_lo, double e_hi, double kT, double *d_W_out,
                              double *tr_ws_out);

/* Toy self-consistent loop (Sec. II.C step (i): the LNOs are recomputed from the previous SCF
 * step's density at every step, so that they become self-consistent).  A step is
 *   ldc_potential (H from H0 and v)  ->  ldc_lno (from the previous D)  ->  ldc_solve  ->
 *   ldc_density  ->  ldc_mulliken  ->  ldc_scf_mix,
 * with the model Hamiltonian H_ij = H0_ij + (v_i + v_j)/2 S_ij, v_i = U (q_i - q0_i), on the
 * Mulliken populations q_i.  All vectors below are device arrays of n_atoms doubles; the
 * calls are enqueued on the plan's stream.
 *
 * ldc_mulliken: q_i = g sum_{j in the pattern row of i} sum_ab D_ij[a,b] S_ij[a,b] from the
 * density rows d_D (row i of D comes from cluster i; for the full density matrix this is
 * g sum_{a in i} (D S)_aa).  Inputs in the layout of S. */
ldc_status ldc_mulliken(ldc_plan_t plan, const double *d_D, const double *d_S, double *d_q);

/* ldc_reference_populations: the neutral populations q0_i = N_e M_i / sum_j M_j of the toy
 * loop (every atom at the system's filling) into the device array d_q0 (n_atoms). */
ldc_status ldc_reference_populations(ldc_plan_t plan, double n_electrons, double *d_q0);

/* ldc_potential: H_ij = H0_ij + (v_i + v_j)/2 S_ij on every pattern block (a uniform v shifts
 * every cluster eigenvalue by v).  d_H may be d_H0 (in place). */
ldc_status ldc_potential(ldc_plan_t plan, const double *d_H0, const double *d_S, const double *d_v, double *d_H);

/* ldc_scf_mix: linear mixing of the input populations, q_in <- q_in + alpha (q_out - q_in)
 * (d_q_in updated in place, 0 <= alpha <= 1), then d_v = U (q_in - q0) for the next step.
 * residual_out (host, may be NULL): max_i |q_out - q_in| before the mixing; when given, the
 * call synchronizes. */
ldc_status ldc_scf_mix(ldc_plan_t plan, const double *d_q_out, double *d_q_in, const double *d_q0, double U,
                       double alpha, double *d_v, double *residual_out);

/* Copy one cluster's spectrum (eps ascending, weights) to host arrays of capacity
 * >= max_dim_pao; *dim receives its dimension.  Synchronizes. */
ldc_status ldc_cluster_spectrum(ldc_plan_t plan, int atom, double *eps, double *w, int *dim);

/* Reduced dimension of every cluster after the last ldc_solve (host array, n_atoms). */
ldc_status ldc_cluster_dims(ldc_plan_t plan, int *dims);

/* Stage timing with HIP events recorded on the plan's stream around each stage.
 * Stages: 0 Lambda, 1 LNO eigensolve, 2 gather, 3 Cholesky, 4 standard form,
 * 5 reduction to band form, 6 band to tridiagonal, 7 second-stage transform of the
 * tracked columns, 8 tridiagonal eigensolve, 9 chemical potential, 10 density rows.
 * ldc_profile(plan, 1) enables timing and clears the accumulated times; 0 disables it.
 * ldc_stage_times fills ms (LDC_NUM_STAGES entries, summed over builds) and *builds (the
 * number of completed ldc_density calls while enabled).  Synchronizes. */
#define LDC_NUM_STAGES 11
ldc_status ldc_profile(ldc_plan_t plan, int enable);
ldc_status ldc_stage_times(ldc_plan_t plan, double *ms, int *builds);
const char *ldc_stage_name(int stage);

/* Message and failing cluster/atom (-1 if none) of the last error on this plan. */
const char *ldc_last_error(ldc_plan_t plan, int *cluster_id);

/* Library version string. */
const char *ldc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LDC_H */
