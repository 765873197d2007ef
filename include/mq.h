/*
 * mq.h -- C ABI of the batched eddy-current UQ library (libmq.so, HIP, gfx950).
 *
 * Operations (Hahn and Schoeps, "Multi-Level Monte Carlo sampling with
 * Parallel-in-Time Integration for Uncertainty Quantification in Electric
 * Machine Simulation"):
 *   fem_setup       Section II-A, Eqs. (1)-(5): 2-D A-formulation, P1 elements
 *                   (w_i = N_i e_z), M_sigma, K_nu and r(t) on a structured mesh.
 *   mlmc_level_run  Section II-A, Eqs. (6)-(7) (implicit Euler) for every sample
 *                   of one MLMC level, on the level's time grid and on the next
 *                   coarser one with the same input (Section II-B, coupled
 *                   differences), and the mean Joule loss of Eq. (26).
 *   parareal_run    Section II-C, Eq. (12): Parareal for samples of the finest
 *                   level, batched over samples and time slices.
 *   mlmc_estimate   Section II-B, Eq. (9): the MLMC estimator (with level means
 *                   and level variances).
 *
 * Conventions
 *  - Every function returns an int status: MQ_OK (0); a positive warning
 *    (results valid, see the per-instance flags in mq_run_stats); or a negative
 *    error (outputs unspecified).  mq_last_error() returns a message for the
 *    last non-zero status of the calling thread.  No C++ exception crosses the
 *    boundary.
 *  - Array arguments marked "device" are HIP device pointers on the device that
 *    was current at fem_setup / mq_server_create (or host pointers on a handle
 *    set up with mem_kind = MQ_MEM_HOST, see mq_problem_desc); arrays marked
 *    "host" are host pointers.  The caller owns every array; the library owns its handles and
 *    the device memory it allocates, and frees both in the *_destroy calls.
 *  - `stream` arguments are hipStream_t passed as void* (NULL: default stream).
 *    Compute calls run on the problem's stream and return after the stream
 *    has finished (results are ready on return).
 *  - Inputs are validated before any launch; invalid sizes return
 *    MQ_ERR_INVALID_ARG, non-finite xi MQ_ERR_NONFINITE.
 *  - Handles are not thread-safe; a server accepts mq_submit from any thread.
 *  - Times: t_k = k dt from the integer step index, a(t_0) = a_0 (zero unless
 *    mq_set_initial_state gave one), the source is
 *    evaluated at t_{k+1}.  The state is solved in increment form
 *    (M/dt + K) d_k = r(t_{k+1}) - K a_k, a_{k+1} = a_k + d_k, which is
 *    algebraically Eq. (7); Q = (1/T) sum_k d_k^T M d_k / dt (Eq. (26)).
 */
#ifndef MQ_H
#define MQ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  MQ_OK = 0,
  MQ_WARN_NOT_CONVERGED = 1, /* some instance hit an iteration cap (flags in stats) */
  MQ_ERR_INVALID_ARG = -1,
  MQ_ERR_NO_DEVICE = -2,
  MQ_ERR_OUT_OF_MEMORY = -3,
  MQ_ERR_DEVICE = -4,
  MQ_ERR_NONFINITE = -5,
  MQ_ERR_BUSY = -6,
  MQ_ERR_CANCELLED = -7
};

enum { MQ_MAT_LOGNORMAL_SCALAR = 0, MQ_MAT_KL = 1, MQ_MAT_NONLINEAR = 2 };
enum { MQ_PREC_FP64 = 0, MQ_PREC_MIXED = 1 };
enum { MQ_APPLY_A = 0, MQ_APPLY_M = 1, MQ_APPLY_K = 2 };
/* kernel path selection (mq_problem_desc.path) */
/* Execution path: RESIDENT (CG state in registers/LDS, meshes up to 129 x 129),
 * STREAMING (vectors in global memory, any mesh), both one workgroup per
 * instance and many instances per launch; WIDE: one instance at a time over
 * the whole device (grid-wide passes, inner iterations replayed from a captured
 * graph) — for few large instances, where latency matters more than throughput;
 * needs multigrid (n_nodes = 2^k + 1) and a linear material; level runs only. */
enum { MQ_PATH_AUTO = 0, MQ_PATH_RESIDENT = 1, MQ_PATH_STREAMING = 2, MQ_PATH_WIDE = 3 };
/* inner preconditioner (mq_problem_desc.precond): Jacobi is a symmetric
 * diagonal scaling; MULTIGRID is a geometric V(1,1)-cycle with damped-Jacobi
 * smoothing and Galerkin coarse operators (resident path, n_nodes = 2^k + 1) */
enum { MQ_PRECOND_AUTO = 0, MQ_PRECOND_JACOBI = 1, MQ_PRECOND_MULTIGRID = 2 };
/* where the array arguments of a handle's calls live (mq_problem_desc.mem_kind) */
enum { MQ_MEM_DEVICE = 0, MQ_MEM_HOST = 1 };
/* mass matrix (mq_problem_desc.mass): the consistent P1 matrix of Eq. (4), or its
 * row-sum lumped diagonal (a test option: with it a sampled sine mode of the
 * homogeneous square is an eigenvector with a closed-form eigenvalue) */
enum { MQ_MASS_CONSISTENT = 0, MQ_MASS_LUMPED = 1 };

/* Problem description (Section II-A; materials per the workload).
 * Unit square, n_nodes x n_nodes nodes, each cell split along "/" into two P1
 * triangles; A = 0 on the boundary.  Elements whose centroid lies in
 * `conductor` (inclusive) are conducting; elsewhere sigma = 0, nu = nu_air.
 * The source J(t) = J0 sin(2 pi freq t) acts on elements whose centroid x lies
 * in [strip[0], strip[1]].  Conductor materials by kind:
 *  LOGNORMAL_SCALAR: sigma = sigma0 exp(s_sigma xi_0), nu = nu_cond exp(s_nu xi_1)
 *  KL:  ln sigma_e = ln sigma0 + s_kl sum_k sqrt(lam_k) phi_k(c_e) xi_k, nu = nu_cond,
 *       separable exponential covariance exp(-|dx|/corr_len - |dy|/corr_len)
 *       on the conductor rectangle, n_modes largest modes, c_e = centroid.
 *  NONLINEAR: sigma = sigma0, nu(|B|) = k1' exp(k2' |B|^2) + k3',
 *       k_i' = k_i exp(s_k xi_i), solved per step by Picard iteration
 *       (||a^(i+1) - a^(i)|| <= picard_tol ||a^(i+1)||, at most picard_max).
 * Linear solves: preconditioned CG inside iterative refinement; a step
 * is converged when ||b - (M/dt + K) d||_2 <= tol ||b||_2 in FP64.  The inner
 * CG runs in FP64 (MQ_PREC_FP64) or FP32 (MQ_PREC_MIXED) to inner_rtol
 * relative to its own initial residual, at most max_iter iterations per
 * solve and max_sweeps refinement sweeps per step. */
typedef struct mq_problem_desc {
  int32_t n_nodes;
  int32_t material;
  int32_t precision;
  int32_t path;
  double conductor[4]; /* x0, x1, y0, y1 */
  double strip[2];     /* x0, x1 */
  double J0, freq;
  double sigma0, nu_cond, nu_air;
  double s_sigma, s_nu;
  int32_t n_modes, picard_max;
  double corr_len, s_kl;
  double k1, k2, k3, s_k, picard_tol;
  double tol, inner_rtol;
  int32_t max_iter, max_sweeps;
  int32_t precond;   /* MQ_PRECOND_*: AUTO = multigrid where available (n_nodes = 2^k + 1; on the
                        resident path if its LDS holds the hierarchy), else Jacobi;
                        MULTIGRID where it is not available: MQ_ERR_INVALID_ARG */
  int32_t tile;      /* workgroup shape: 0 auto (the built-in default, 1).  Resident path: 1 = 16 rows
                        per thread, 2 = 32 rows per thread in 512-thread workgroups (meshes with
                        64..127 interior nodes per side; others use 1).  Streaming path: 1 = one
                        1024-thread workgroup per compute unit, 2 = two 512-thread workgroups */
  double mg_omega;   /* damped-Jacobi weight of the multigrid smoother (0: 0.8) */
  int32_t mg_levels; /* coarse levels in use (0: all, down to one node) */
  int32_t mg_coarse_sweeps; /* damped-Jacobi sweeps after Z = diag^{-1} R at the coarsest level
                               in use (0..64) */
  int32_t split_steps;  /* resident path, linear material: when a launch holds more instances than
                           the device has slots, short instances may run as dependent pieces of
                           this many steps, queued after the long ones, where a simulation of the
                           work queue says the launch ends sooner (results are bitwise those of
                           the unsplit run).  0: 32; -1: never. */
  int32_t mg_block_min; /* multigrid coarse levels with at least this many interior nodes per side
                           run on the whole workgroup, smaller ones on one wavefront (0: 15) */
  int32_t mem_kind;     /* MQ_MEM_DEVICE (0): array arguments are device pointers.  MQ_MEM_HOST:
                           the arrays of mq_set_initial_state, mlmc_level_run, mlmc_multilevel_run
                           and parareal_run are host pointers, staged through device copies
                           (the call blocks; the rate includes the transfers); the handle's other
                           calls return MQ_ERR_INVALID_ARG.  Servers built on such a description
                           still take device memory only internally (requests carry xi inline). */
  int32_t mass;         /* MQ_MASS_CONSISTENT (0) or MQ_MASS_LUMPED */
} mq_problem_desc;

typedef struct mq_problem mq_problem;

typedef struct mq_problem_info {
  int32_t n_nodes, n_dof, pitch, n_xi;
  int32_t box[4];        /* interior-node box [x0, x1) x [y0, y1) of sample-dependent rows */
  int32_t resident_ok;   /* 1 if the register/LDS-resident path fits this mesh/precision */
  int32_t lds_bytes;     /* LDS per workgroup of the resident path */
  int32_t precond;       /* preconditioner in use (MQ_PRECOND_JACOBI or _MULTIGRID) */
  int32_t mg_levels;     /* coarse levels of the multigrid hierarchy (0 if unused) */
  int32_t n_modes_used;
  double kl_lambda[16];  /* 2-D KL eigenvalues in use (KL material) */
  int32_t tile;          /* workgroup shape in use (1 or 2, see mq_problem_desc.tile) */
  int32_t block;         /* threads per workgroup of the time-stepping kernel */
} mq_problem_info;

/* Per-call statistics (host struct, nullable). */
typedef struct mq_run_stats {
  int64_t n_instances;
  int64_t sample_steps;        /* implicit Euler steps executed (all instances) */
  int64_t inner_iters;         /* CG iterations summed over instances */
  int64_t sweeps;              /* refinement sweeps summed over instances */
  int64_t picard_iters;        /* Picard iterations summed (nonlinear) */
  int32_t max_inner_per_step;  /* largest inner-iteration count of any step */
  int32_t n_not_converged;     /* instances that hit a cap */
  int32_t n_failed;            /* instances with a non-finite residual (or a piece that waited
                                  for its predecessor past the time limit) */
  int32_t path;                /* MQ_PATH_RESIDENT or MQ_PATH_STREAMING */
  int32_t grid, block;         /* launch shape of the time-stepping kernel */
  double kernel_ms;            /* device time of the time-stepping launches */
  double total_ms;             /* wall time of the call */
  double lat_p50_ms, lat_p99_ms, lat_max_ms; /* per-sample latency.  Level and multilevel runs:
                                                from the call's start on the host until the
                                                sample's Q (fine and coupled coarse) is readable
                                                in host memory (each instance writes its Q and a
                                                completion flag to coherent pinned memory, polled
                                                by the calling thread).  Other runs: device-clock
                                                completion after the first instance started, last
                                                launch */
  double phase_ms[8];  /* resident and streaming paths: phases summed over instances (one
                          thread's clock): multigrid fine descent (pre-smoothing), restriction +
                          coarse levels, fine ascent (prolongation + post-smoothing), CG apply +
                          updates + reductions; right-hand side, refinement residuals,
                          increment updates, QoI + state update */
  double busy_ms;      /* sum over instances of their device time (start to end) */
  int64_t n_pieces;    /* launch entries when instances ran as dependent pieces (split_steps),
                          else 0 */
} mq_run_stats;

/* One MLMC level (Section II-B): every sample runs steps_per_period *
 * n_periods implicit Euler steps of dt = 1/(freq steps_per_period) and, if
 * coarse_steps_per_period > 0, the coupled coarse run with the same xi. */
typedef struct mq_level_desc {
  int32_t steps_per_period;
  int32_t coarse_steps_per_period; /* 0 at level 0 (Q_{-1} = 0) */
  int32_t n_periods;
  int32_t reserved;
} mq_level_desc;

/* Parareal (Section II-C): [0, n_periods/freq] split into n_slices slices;
 * fine F = fine_steps_per_slice IE steps per slice, coarse C =
 * coarse_steps_per_slice IE steps per slice.  Iterate until the largest
 * relative interface jump ||F_n - U_n|| / ||F_n|| <= tol or k_max iterations
 * (fixed_k > 0: exactly fixed_k iterations, no tolerance test). */
typedef struct mq_parareal_desc {
  int32_t n_periods, n_slices, fine_steps_per_slice, coarse_steps_per_slice;
  int32_t k_max, fixed_k;
  double tol;
} mq_parareal_desc;

/* The tail-splitting plan that the level runs use on the resident path
 * (host arithmetic only; see mq_problem_desc.split_steps): a launch of n
 * instances of steps[i] steps on `slots` persistent slots, with split_steps
 * as in the descriptor.  *m_out receives the number of launch entries (n when
 * nothing is split); the first min(m, cap) entries are written: entry e runs
 * steps [first[e], first[e] + len[e]) of instance orig[e] and waits for entry
 * dep[e] (-1: none).  makespan (nullable, [2]): the simulated launch length in
 * steps without and with the plan (pieces counted with two extra steps of
 * set-up).  Errors: n < 0, a step count < 1, slots < 1, split_steps < -1. */
int mq_plan_split(int32_t n, const int32_t* steps, int32_t slots, int32_t split_steps, int32_t cap,
                  int32_t* orig, int32_t* first, int32_t* len, int32_t* dep, double* makespan, int32_t* m_out);

const char* mq_last_error(void);
int mq_version(void);

/* Per-instance flag bits (mq_last_flags; mq_run_stats counts them). */
enum {
  MQ_FLAG_NOT_CONVERGED = 1, /* a step ended at max_iter / max_sweeps above tol (results are those of
                                the last sweep) */
  MQ_FLAG_FAILED = 2,        /* a non-finite residual: the instance's results are not valid; the
                                other instances of the call are unaffected */
  MQ_FLAG_PICARD_CAP = 4,    /* a step's Picard iteration stopped at picard_max above picard_tol
                                (counted in n_not_converged) */
  MQ_FLAG_PARAREAL_KMAX = 8  /* Parareal stopped at k_max above tol (Section II-C) */
};

/* Per-instance flags of the calling thread's last mlmc_level_run,
 * mlmc_multilevel_run or parareal_run (any handle), so that a caller given
 * MQ_WARN_NOT_CONVERGED can tell which results to distrust.  Order: level run:
 * the n fine instances by sample, then (coupled level) the n coarse ones;
 * multilevel run: the same per level, levels in order; Parareal: one entry per
 * sample, the OR of its fine and coarse instances plus MQ_FLAG_PARAREAL_KMAX.
 * After any other run call, or a run call that failed before its launch, the
 * list is empty.  flags: host [cap] (nullable when cap = 0); *n_out: host, the
 * list's length (entries beyond cap are not written).  The list belongs to the
 * calling thread.  Errors: MQ_ERR_INVALID_ARG (n_out null, cap < 0, flags null
 * with cap > 0). */
int mq_last_flags(int32_t* flags, int64_t cap, int64_t* n_out);

/* Build the mesh, masks, KL basis, load shape and device tables.
 * d: host; stream: hipStream_t or NULL; *out receives the handle.
 * Errors: MQ_ERR_INVALID_ARG (n_nodes < 3, bad boxes, tolerances), MQ_ERR_NO_DEVICE,
 * MQ_ERR_OUT_OF_MEMORY. */
int fem_setup(const mq_problem_desc* d, void* stream, mq_problem** out);
int mq_problem_destroy(mq_problem* p);
int mq_ndof(const mq_problem* p, int64_t* nd);
int mq_problem_info_get(const mq_problem* p, mq_problem_info* info);

/* Start state a_0 = a(t_0) of Eq. (7) for every later run on this handle:
 * mlmc_level_run, mlmc_multilevel_run, mlmc_adaptive_run and mlmc_combined_run
 * (fine and coupled coarse runs alike), the handle's levels of
 * mlmc_multimesh_run, and U_0 of parareal_run (Eq. (12)); servers are not
 * affected.  a0: device [n_dof] FP64, interior DoF order (j-1)(N-2)+(i-1) (the
 * boundary ring stays A = 0), copied before return; NULL restores a_0 = 0.
 * Errors: MQ_ERR_INVALID_ARG (null handle), MQ_ERR_NONFINITE (NaN or Inf in a0,
 * the previous a_0 is kept), MQ_ERR_OUT_OF_MEMORY. */
int mq_set_initial_state(mq_problem* p, const double* a0);

/* One MLMC level for n_samples samples.
 * xi: device [n_samples][n_xi] FP64.  q_fine: device [n_samples] (Q on the
 * level's grid).  q_coarse: device [n_samples] or NULL; required when
 * lv->coarse_steps_per_period > 0.  final_state: device [n_samples][n_dof] or
 * NULL (fine-run end state, interior DoF order (j-1)(N-2)+(i-1)).  st: host or NULL.
 * Returns MQ_WARN_NOT_CONVERGED if any instance hit a cap. */
int mlmc_level_run(mq_problem* p, const mq_level_desc* lv, int32_t n_samples, const double* xi,
                   double* q_fine, double* q_coarse, double* final_state, mq_run_stats* st);

/* Allocation-free form of mlmc_level_run, for callers that cannot allocate
 * device memory during the call (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation).  Same arguments, results and
 * errors as mlmc_level_run (results bitwise equal); every per-call buffer
 * (sample tables, source tables, instance table, statistics, the persistent
 * kernel's work slots) is carved from a fixed device workspace of
 * MQ_NOALLOC_WORKSPACE_BYTES that the library holds on each device it runs on
 * until the process ends; the call makes no hipMalloc/hipFree or other
 * allocation (its instances are never split into pieces, and kernel_ms is
 * taken with the host clock).  The work slots are as many as fit after the
 * inputs, so a large batch may run on fewer than all compute units.
 * Limits: a run whose inputs plus one work slot exceed the workspace returns
 * MQ_ERR_INVALID_ARG before any launch; the wide path is refused; the handle
 * must take device pointers.  Every call on a device shares that device's
 * workspace, which keeps the last call's contents: calls that overlap on one
 * device (other threads or streams) race and must be serialised by the caller. */
#define MQ_NOALLOC_WORKSPACE_BYTES 268435456 /* 256 MiB */
int mlmc_level_run_noalloc(mq_problem* p, const mq_level_desc* lv, int32_t n_samples, const double* xi,
                           double* q_fine, double* q_coarse, double* final_state, mq_run_stats* st);

/* Several levels in ONE persistent launch (instances of all levels share the
 * device work queue, longest first).  lv, n_samples, xi, q_fine, q_coarse are
 * host arrays of n_levels entries; the pointers inside are device pointers as
 * in mlmc_level_run (q_coarse[l] may be NULL only where lv[l] has no coarse run). */
int mlmc_multilevel_run(mq_problem* p, int32_t n_levels, const mq_level_desc* lv,
                        const int32_t* n_samples, const double* const* xi,
                        double* const* q_fine, double* const* q_coarse, mq_run_stats* st);

/* Spatial and temporal level hierarchy (Section I; Section II-B with levels
 * that refine the mesh as well as the time step): level l runs on the mesh of
 * problems[l] and its coupled coarse run on the mesh of problems[l - 1], with
 * the same input (the KL field is evaluated at each mesh's element centroids).
 * problems: host array of n_levels distinct handles that share material,
 * input dimension and precision; lv, n_samples, xi, q_fine, q_coarse as in
 * mlmc_multilevel_run.  One persistent launch per mesh (its fine runs and the
 * next level's coarse runs), all meshes concurrently on their problems'
 * streams; returns when all are done.  st: kernel_ms is the longest launch. */
int mlmc_multimesh_run(int32_t n_levels, mq_problem* const* problems, const mq_level_desc* lv,
                       const int32_t* n_samples, const double* const* xi, double* const* q_fine,
                       double* const* q_coarse, mq_run_stats* st);

/* Adaptive MLMC (Section II-B, Eq. (11)): the level variances V_l are
 * estimated at run time.  Every level first runs n_pilot samples; each round
 * then runs, in one persistent launch, the additional samples that
 *   N_l = ceil( sqrt(V_l / C_l) * sum_k sqrt(V_k C_k) / (var_fraction * target_rmse^2) )
 * asks for (the minimiser of sum N_l C_l under sum V_l / N_l = var_fraction *
 * target_rmse^2), with C_l the steps of one sample of level l (fine + coarse)
 * and V_l the current unbiased variance of Q_l - Q_{l-1}; N_l never decreases
 * and is capped at n_max[l].  Stops when no level asks for more samples or
 * after max_rounds rounds.
 * xi: host array of device pointers, [n_max[l]][n_xi] each (the inputs of
 * sample k of level l are row k); q_fine, q_coarse: host arrays of device
 * pointers, [n_max[l]] each (q_coarse[0] ignored); sample k's results land in
 * row k.  n_used: host [n_levels] (samples taken); out: host [1 + 2 n_levels] =
 * {E, Y_0..Y_{L-1}, V_0..V_{L-1}} of the final samples.  Returns
 * MQ_WARN_NOT_CONVERGED when a cap (n_max or max_rounds) stopped the
 * allocation short of Eq. (11), or when an instance hit a solver cap. */
typedef struct mq_adaptive_desc {
  double target_rmse;    /* > 0 */
  double var_fraction;   /* share of target_rmse^2 for the estimator variance (0: 0.5) */
  int32_t n_pilot;       /* >= 2 */
  int32_t max_rounds;    /* 0: 10 */
} mq_adaptive_desc;
int mlmc_adaptive_run(mq_problem* p, int32_t n_levels, const mq_level_desc* lv, const int32_t* n_max,
                      const double* const* xi, double* const* q_fine, double* const* q_coarse,
                      const mq_adaptive_desc* ad, int32_t* n_used, double* out, mq_run_stats* st);

/* Parareal for n_samples samples at once (samples x slices batched).
 * xi: device [n_samples][n_xi]; q: device [n_samples] (Q from the final
 * per-slice fine sums); iters: device int32 [n_samples] (K per sample);
 * final_state: device [n_samples][n_dof] or NULL; st: host or NULL.
 * Returns MQ_WARN_NOT_CONVERGED if some sample reached k_max above tol. */
int parareal_run(mq_problem* p, const mq_parareal_desc* pd, int32_t n_samples, const double* xi,
                 double* q, int32_t* iters, double* final_state, mq_run_stats* st);

/* MLMC with Parareal on the finest level (Section II-D): levels 0..L-1 and
 * the coupled coarse runs of level L are batched as in mlmc_multilevel_run,
 * while the fine values of level L come from Parareal (as parareal_run) with
 * the level L-2 discretisation as coarse propagator, all in ONE persistent
 * launch with two work queues: the Parareal entries and the level instances;
 * N_L * M workgroups (at most half) start on the Parareal queue, the others on
 * the levels, and a workgroup whose queue is empty moves to the other one.
 * n_slices = 0 picks M from Eq. (25) with the device's persistent slots as
 * cores: the largest power of two <= max(2, n_c,para) that divides the fine
 * and coarse step counts of level L (a given M must divide both).  q_coarse[L] is bitwise what
 * mlmc_level_run gives for level L; q_fine[L] is the Parareal value and
 * para_iters[N_L] (device) its iteration count K per sample.
 * Errors: fewer than 2 levels, nonlinear material, wide path, invalid slices. */
typedef struct mq_combined_desc {
  int32_t n_slices;                 /* M (0: from Eq. (25), see above) */
  int32_t coarse_steps_per_period;  /* coarse propagator (0: level L-2's steps per period) */
  int32_t k_max;                    /* 0: M */
  int32_t reserved;
  double tol;                       /* largest relative interface jump to stop at */
} mq_combined_desc;

typedef struct mq_combined_stats {
  int32_t n_slices, coarse_steps_per_period, n_cores, n_c_para;
  double ms_levels;    /* device time from the launch's start to the last level instance's end */
  double ms_parareal;  /* device time from the launch's start to the last Parareal entry's end */
  double ms_total;
  int64_t para_fine_steps, para_coarse_steps;  /* sample-steps Parareal executed (all samples) */
  double mean_k;
  int32_t max_k;
  int32_t level_slots;  /* workgroups that start on the level queue: the device's n_cores less
                           N_L * M (at most half) that start on the Parareal queue */
} mq_combined_stats;

int mlmc_combined_run(mq_problem* p, int32_t n_levels, const mq_level_desc* lv, const int32_t* n_samples,
                      const double* const* xi, const mq_combined_desc* cd, double* const* q_fine,
                      double* const* q_coarse, int32_t* para_iters, mq_run_stats* st, mq_combined_stats* cs);

/* Cost model of the combined method (Section II-C Eqs. (13)-(16), Section
 * II-D Eqs. (17)-(25)), host arithmetic only.  C_l: sequential cost of one
 * sample of level l (any unit), N_l: samples; K, M: Parareal iterations and
 * slices on level L with tau_F = C_L and tau_C = C_{L-2}; n_cores: n_c of
 * Eqs. (24)-(25).  Errors: n_levels outside [3, 16], K outside [1, M],
 * C_l <= 0, N_l < 1. */
typedef struct mq_cost_in {
  int32_t n_levels, K, M, n_cores;
  double C[16], N[16];
} mq_cost_in;

typedef struct mq_cost_out {
  double tau_para, effort_para;  /* Eqs. (15), (16) */
  double tau_ref, effort_ref;    /* Eq. (17) */
  double tau_comb, effort_comb;  /* Eqs. (18), (19) */
  double speedup;                /* tau_ref / tau_comb */
  double s_inf;                  /* Eq. (21): sum_l C_l / (sum_{l<L} C_l + C_{L-1}) */
  double eps_inf;                /* Eq. (23): effort_comb / effort_ref */
  double r;                      /* C_L / C_{L-1} */
  int32_t kappa;                 /* Eq. (22) with n = M */
  int32_t n_c_para;              /* Eq. (25) */
  int32_t batches[16];           /* Eq. (24) */
  double s_nc;                   /* speedup on n_cores cores (0 when n_c_para < 1) */
} mq_cost_out;

int mq_cost_model(const mq_cost_in* in, mq_cost_out* out);

/* Eq. (9) in FP64 on the device with a fixed summation order.
 * n_per_level: host [n_levels]; q_fine, q_coarse: host arrays of device
 * pointers (q_coarse[0] ignored, Q_{-1} = 0).  out: device [1 + 2 n_levels] =
 * {E, Y_0..Y_L, V_0..V_L} (V_l with N_l - 1; 0 when N_l = 1).  stream: hipStream_t or NULL. */
int mlmc_estimate(int32_t n_levels, const int32_t* n_per_level, const double* const* q_fine,
                  const double* const* q_coarse, double* out, void* stream);

/* Test hook: y = which(xi) x with which in {A = M/dt + K, M, K} for n samples.
 * xi device [n][n_xi]; x, y device [n][n_dof] FP64 (interior DoF order). */
int mq_debug_apply(mq_problem* p, int32_t which, double dt, int32_t n, const double* xi,
                   const double* x, double* y);

/* ---------------------------------------------------------------- serving
 * Continuous batching of independent sample solves (the time integration of
 * Section II-A for one KL input on its own mesh and time grid; linear
 * materials).  The server has a scheduler thread of its own.  Requests are
 * admitted in arrival order while the device memory they need fits
 * hbm_budget_bytes and fewer than max_inflight are admitted; an admitted
 * request keeps its tables, state and QoI on the device until it completes.
 * Each mesh size has n_streams lanes (a HIP stream each); whenever a lane is
 * idle, the next chunk_steps steps of every admitted request of its mesh size
 * that is not running elsewhere go into one persistent launch on it, so
 * requests that arrive while others run join the next launch and overlap on
 * the device with those already running.  Launches split a request at fixed
 * request-relative steps and resume it exactly, so its result is the same bit
 * for bit whatever else the server runs, and equal to mlmc_level_run of the
 * same input at level 0 (for a request of the wide lane, below: on a problem
 * set up with path MQ_PATH_WIDE).  Device memory (per-mesh work buffers, request slots)
 * is kept for reuse until mq_server_destroy and counts against the budget. */
typedef struct mq_server_desc {
  mq_problem_desc base;      /* material/precision/tolerances; n_nodes ignored; linear */
  int64_t hbm_budget_bytes;  /* > 0 */
  int32_t max_inflight;      /* >= 1 admitted requests at most */
  int32_t n_streams;         /* lanes per mesh size, 0..8 (0: 2) */
  int32_t max_batch;         /* requests in one launch at most (0: 4096) */
  int32_t chunk_steps;       /* steps per request per launch (0: 32) */
  int32_t wide_min_nodes;    /* requests with n_nodes >= this (and n_nodes = 2^k + 1, multigrid
                                allowed by base) run one at a time on the wide path, over the
                                whole device, while fewer than wide_load_limit batched requests
                                are admitted and at most wide_queue of them wait; otherwise they
                                are batched.  0: 513; -1: never.  The wide lane's set-up (one
                                work slot per mesh size) is outside hbm_budget_bytes and its
                                requests outside max_inflight. */
  int32_t wide_queue;        /* wide-lane requests allowed to wait (0: 8) */
  int32_t wide_load_limit;   /* see wide_min_nodes (0: half the device's compute units) */
  int32_t reserved;
} mq_server_desc;

typedef struct mq_request {
  int32_t n_nodes, steps_per_period, n_periods, n_xi;
  double xi[16];
  uint64_t user_id;
} mq_request;

typedef struct mq_result {
  uint64_t ticket, user_id;
  double q;                  /* Eq. (26) mean Joule loss over n_periods / freq */
  int32_t status;            /* MQ_OK, MQ_WARN_NOT_CONVERGED, or an error: MQ_ERR_BUSY when the
                                request alone does not fit the budget, MQ_ERR_NONFINITE when
                                the solve produced NaN/Inf, MQ_ERR_DEVICE / _OUT_OF_MEMORY */
  int32_t inner_iters;       /* inner CG iterations, summed over the request's steps */
  int32_t sweeps;            /* refinement sweeps, summed over the request's steps */
  int32_t path;              /* MQ_PATH_RESIDENT / _STREAMING (batched lane) or MQ_PATH_WIDE */
  int64_t t_submit_ns, t_start_ns, t_done_ns; /* steady-clock ns: mq_submit, first launch,
                                                 QoI copied to the host */
  char message[64];          /* status < 0: what failed (NUL-terminated, truncated) */
} mq_result;

typedef struct mq_server mq_server;
/* Create a server on the current device; stream is unused (the server owns its
 * streams).  Errors: invalid limits or base description, nonlinear material. */
int mq_server_create(const mq_server_desc* sd, void* stream, mq_server** out);
/* Queue a request (host struct, copied); *ticket identifies it in mq_poll.
 * Validated at once (mesh size, steps, n_xi of the material, finite xi);
 * callable from any thread. */
int mq_submit(mq_server* s, const mq_request* rq, uint64_t* ticket);
/* Copy up to cap finished results (host array) to out and set *n_out.
 * Non-blocking; results come in completion order. */
int mq_poll(mq_server* s, mq_result* out, int32_t cap, int32_t* n_out);
/* Number of requests queued or admitted and not yet finished. */
int mq_server_pending(const mq_server* s, int32_t* n);
/* Waits for the launches in flight, drops unfinished requests, frees everything. */
int mq_server_destroy(mq_server* s);

#ifdef __cplusplus
}
#endif
#endif /* MQ_H */
