/*
 * mlmc.h -- C-ABI of the MI355X multilevel Monte Carlo finite-element library.
 *
 * The library estimates E[Q(u)] for the random diffusion problem
 *     -div(kappa(x, omega) grad u) = f  in D,   u = u0 on the boundary
 * (paper Sec. 2.1, eq. model) by the telescoping multilevel estimator
 *     Qtilde_L = sum_{l=0}^{L} mean(Y_l),  Y_0 = Q_0,  Y_l = Q_l - Q_{l-1}
 * (Sec. 2.2, eq. mlmc_average), with D = [0,1]^3, f = 1, u0 = 0, a log-normal
 * kappa given by a Karhunen-Loeve expansion with exponential covariance
 * (Sec. 5.2), Q1 hexahedral meshes with n_l = n0 * 2^l elements per side
 * (Sec. 2.2, s = 2), and one batched finite-element solve per sample and mesh.
 *
 * Conventions shared by every entry point
 *   Status: every call returns an int status (MLMC_OK, MLMC_PENDING or a
 *     negative MLMC_E_* code).  On error, mlmc_last_error(ctx) describes it;
 *     outputs are left unspecified unless stated otherwise.
 *   Memory: the library allocates no device memory.  All device work space
 *     comes from the caller's arena (mlmc_config.arena/arena_bytes), which is
 *     the device-memory budget; pointers documented as "device" are caller
 *     owned device allocations, "host" pointers are caller-owned host memory.
 *   Stream: all device work of a context is issued on mlmc_config.stream
 *     (a hipStream_t; NULL = the null stream).  Step-level calls return once
 *     work is queued; whole-path calls (sample_level, estimate) synchronise.
 *   Threading: a context is used by one host thread at a time.
 *
 * Layouts
 *   Interior node (i, j, k), 1 <= i, j, k <= n-1, of an n^3 mesh; element
 *   e = ex + n*(ey + n*ez), 0 <= ex, ey, ez < n.
 *   "grid layout" vector of a batch of B samples on mesh n: B blocks of
 *     mlmc_grid_stride(n) entries; node (i, j, k) of sample b sits at
 *     b*stride + i + n*j + n*n*k.  Every entry that is not an interior node
 *     (i == 0, j == 0, k == 0, k == n, and the tail padding) must hold 0 and
 *     is never written by the library.
 *   "element layout" coefficient of a batch: B blocks of n^3 entries,
 *     element e of sample b at b*n^3 + e.
 */
#ifndef MLMC_H
#define MLMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  MLMC_OK = 0,
  MLMC_PENDING = 1,       /* mlmc_poll: the request has not finished yet */
  MLMC_E_INVALID = -1,    /* bad argument or configuration */
  MLMC_E_NOMEM = -2,      /* the arena cannot hold the work space of the call */
  MLMC_E_BUDGET = -3,     /* a request does not fit the HBM budget at all */
  MLMC_E_NOCONV = -4,     /* a solve hit max_iter above its tolerance */
  MLMC_E_NONFINITE = -5,  /* a NaN or Inf appeared in a field or residual */
  MLMC_E_DEVICE = -6      /* a HIP runtime call failed */
};

enum { MLMC_QOI_DOMAIN_AVERAGE = 0, MLMC_QOI_SUBCUBE_AVERAGE = 1 };
/* FP64: every step in fp64.  MIXED: fp32 operator, smoother and multigrid
 * inside fp64 iterative refinement (fp64 outer residual with the fp64 kappa,
 * fp64 dot products, recurrences and statistics).  MIXED_BF16KLE: MIXED, and
 * the KLE contraction with bf16 operands and fp32 accumulation on MFMA -- a
 * perturbation of the coefficient field itself (|g - g_fp64| <= ~2^-7 sum_m
 * |sqrt(lambda_m) xi_m phi_m|), reported against the fp64 result. */
enum { MLMC_PREC_FP64 = 0, MLMC_PREC_MIXED = 1, MLMC_PREC_MIXED_BF16KLE = 2 };
enum { MLMC_SOLVER_GMG_PCG = 0, MLMC_SOLVER_JACOBI_PCG = 1 };
/* Forcing term f of eq. model (Sec. 2.1: f may be a random field too).
 * CONSTANT: f = 1.  LOGNORMAL: f = exp(g_f), g_f the truncated KLE with the
 * modes and eigenvalues of the log-diffusion's field but its own coefficients
 * xi_f (Philox counter word 3 = 2, see mlmc_forcing), independent of kappa;
 * one value per element at its centroid, like kappa.  The Dirichlet data stays
 * u = 0. */
enum { MLMC_FORCING_CONSTANT = 0, MLMC_FORCING_LOGNORMAL = 1 };

typedef struct mlmc_config {
  int32_t n0;          /* elements per side of the coarsest MLMC mesh, >= 2, power of 2 */
  int32_t levels;      /* L + 1 >= 1; level l uses n0 << l elements per side */
  double sigma2;       /* variance of the Gaussian log-field, >= 0 */
  double corr_len;     /* correlation length of exp(-|dx|/corr_len), > 0 */
  int32_t n_modes;     /* number M of 3D KL modes (length of xi), 1..4096 */
  uint64_t seed;       /* Philox key word 0 */
  int32_t qoi;         /* MLMC_QOI_*; the subcube QoI needs 4 | n on every mesh */
  double rtol;         /* true relative residual ||b - A x||_2 / ||b||_2 to reach */
  int32_t max_iter;    /* cap on PCG iterations (outer + inner for mixed) */
  int32_t precision;   /* MLMC_PREC_* */
  int32_t solver;      /* MLMC_SOLVER_* */
  int32_t cheb_degree; /* Chebyshev smoothing degree per half V-cycle, 1..8 (0: 2) */
  int32_t max_batch;   /* samples solved together on the finest mesh, >= 1; a coarser level takes
                          as many as cost the same interior DOFs (at most 65536, and what the
                          arena holds) */
  int32_t forcing;     /* MLMC_FORCING_*; LOGNORMAL is not available while serving */
  void* arena;         /* device memory owned by the caller, 256-byte aligned */
  size_t arena_bytes;  /* size of the arena: the HBM budget of the context */
  void* stream;        /* hipStream_t for all device work of the context */
} mlmc_config;

typedef struct mlmc_ctx mlmc_ctx;

typedef struct mlmc_level_stats {
  uint64_t n;          /* samples accumulated (finite Y only) */
  double mean;         /* mean of Y_l */
  double m2;           /* sum of squared deviations from the mean */
  double var;          /* m2 / n, the 1/N sample variance of eq. sample_variance */
  double cost;         /* mean cost per sample used by the allocation (see below) */
  uint64_t nonfinite;  /* samples whose Y was NaN or Inf: counted here, kept out of n, mean, m2 */
} mlmc_level_stats;

typedef struct mlmc_estimate_out {
  double qtilde;       /* sum_l mean(Y_l), eq. mlmc_average */
  double var_qtilde;   /* sum_l var_l / n_l, Sec. 2.2 */
  int32_t levels;      /* number of levels reported below */
  mlmc_level_stats level[16];
  int32_t lanes;       /* lanes of the last sampling round of the last whole-path call */
  double active_ratio; /* A = a / (p t_w) of eq. active_ratio over that call's rounds: lane-seconds spent
                          on tasks / (lanes x wall seconds) */
} mlmc_estimate_out;

/* ------------------------------------------------------------------ setup */

/* Create a context for the configuration; computes the 1D KL eigenpairs and
 * the M-mode 3D selection on the host (Sec. 5.2, KLE with exponential
 * covariance).  *out receives the context, or NULL on error.
 * Errors: MLMC_E_INVALID for a bad field, MLMC_E_DEVICE. */
int mlmc_create(const mlmc_config* cfg, mlmc_ctx** out);

/* Destroy a context; cancels requests still queued.  NULL is ignored. */
void mlmc_destroy(mlmc_ctx* ctx);

/* Text of the last error of the context (or of the last failed create when
 * ctx is NULL).  Valid until the next call on the context. */
const char* mlmc_last_error(const mlmc_ctx* ctx);

/* Entries per sample in the grid layout of an n^3 mesh (>= (n+1) n^2). */
size_t mlmc_grid_stride(int32_t n);

/* The node numbering of the grid layout on mesh n (the interior unknowns of
 * the Q1 space, Sec. 2.1): out (host, mlmc_grid_stride(n) entries) receives,
 * for every position of a sample's grid vector, the interior unknown
 * g = (i-1) + (n-1)((j-1) + (n-1)(k-1)) stored there, or -1 where the layout
 * holds no unknown.  Computed on the device with the layout's index
 * arithmetic, in scratch space of the arena (the cached work space is carved
 * again by the next call that needs it).  For parity tests.
 * Errors: MLMC_E_INVALID (n not a power of two in 2..1024, NULL out, serving),
 * MLMC_E_NOMEM. */
int mlmc_node_map(mlmc_ctx* ctx, int32_t n, int32_t* out);

/* Arena bytes needed by mlmc_sample_level for `batch` samples of `level`
 * under the configuration (without creating a context). */
size_t mlmc_workspace_bytes(const mlmc_config* cfg, int32_t level, int32_t batch);

/* The selected 3D modes: triples[3*m + d] is the 1D mode index of axis d of
 * mode m and lambda[m] = sigma2 * lambda_i lambda_j lambda_k (host arrays of
 * n_modes entries each; either may be NULL). */
int mlmc_modes(const mlmc_ctx* ctx, int32_t* triples, double* lambda);

/* The same selection without a context (host only, no device call): the
 * n_modes modes of the separable exponential-covariance KLE (Sec. 5.2) with
 * correlation length corr_len and variance sigma2, as mlmc_modes writes them,
 * and the 1D frequencies omega of the indices they use (omega_q of 1D mode q,
 * increasing; the first max_omega of them are written, *n_omega receives
 * their number).  Arrays are host memory and may be NULL.
 * Errors: MLMC_E_INVALID (corr_len not positive and finite, sigma2 negative
 * or not finite, n_modes outside 1..4096, omega NULL with max_omega > 0). */
int mlmc_kl_modes(double corr_len, double sigma2, int32_t n_modes, int32_t* triples, double* lambda, double* omega,
                  int32_t max_omega, int32_t* n_omega);

/* ------------------------------------------- step-level entry points (device) */

/* K1 -- xi[s*n_modes + m] (device, fp64, [count][n_modes]) for the samples
 * first .. first+count-1 of `level`: Philox4x64-10 blocks with key (seed, 0)
 * and counter (sample, level, block, 0), uniforms ((w >> 12) + 1/2) 2^-52 and
 * Box-Muller pairs.  The randomness of omega in Sec. 2.1, drawn per sample
 * index as the batches of Sec. 4.2 hand them out. */
int mlmc_draw_xi(mlmc_ctx* ctx, int32_t level, uint64_t first, int64_t count, double* xi);

/* K2 -- kappa (device, element layout, fp64) = exp(sum_m sqrt(lambda_m)
 * phi_m(c_e) xi_m) at the element centroids c_e of the n^3 mesh, for `count`
 * samples whose xi (device, [count][n_modes]) is given.  Log-normal KLE
 * coefficient of Sec. 5.2; the contraction runs on fp64 MFMA (on bf16 MFMA
 * with fp32 accumulation under MLMC_PREC_MIXED_BF16KLE).
 * kappa32 (device, may be NULL) receives the same values rounded to fp32. */
int mlmc_field(mlmc_ctx* ctx, int32_t n, int64_t count, const double* xi,
               double* kappa, float* kappa32);

/* K5 -- y = A(kappa) u for `count` samples on the n^3 mesh: the Q1 stiffness
 * of eq. model with per-element kappa and homogeneous Dirichlet rows and
 * columns eliminated (Sec. 2.1-2.2).  u, y: device, grid layout, fp64;
 * kappa: device, element layout, fp64.  u and y must not overlap.  Runs the
 * stencil engine selected by mlmc_tuning.zvar_fp64 (register window or
 * LDS-tiled planes). */
int mlmc_apply(mlmc_ctx* ctx, int32_t n, int64_t count, const double* kappa,
               const double* u, double* y);

/* mlmc_apply in fp32 (the operator of the mixed-precision inner solve): u, y
 * and kappa are fp32 arrays in the same layouts; the engine is the one
 * mlmc_tuning.zvar_fp32 selects.  Errors as mlmc_apply. */
int mlmc_apply_f32(mlmc_ctx* ctx, int32_t n, int64_t count, const float* kappa,
                   const float* u, float* y);

/* z = c D^-1 b for `count` samples on the n^3 mesh, the first
 * Chebyshev-Jacobi smoothing step from a zero iterate of the V-cycle below,
 * with D_i = (h/3) sum of kappa_e over the 8 elements e around node i, the
 * diagonal of A(kappa) (the smoothers compute it from kappa in the same
 * order).  b, z: device, grid layout, fp64 (z = 0 where the layout holds no
 * unknown); kappa: device, element layout, fp64.  With b = 1 and c = 1 it
 * exports D^-1, for parity tests of the diagonal.  b and z must not overlap.
 * Errors: MLMC_E_INVALID (bad sizes, NULL or overlapping arrays). */
int mlmc_jacobi(mlmc_ctx* ctx, int32_t n, int64_t count, const double* kappa, const double* b, double c,
                double* z);

/* One multigrid V-cycle z = B(kappa) r of the preconditioner used by the
 * GMG-PCG solve (rediscretised coarse operators with the 8-child mean of
 * kappa, trilinear transfers, Chebyshev-Jacobi smoothing of the context's
 * degree on the interval [0.4375, 1.75] of the spectrum of D^-1 A, exact
 * solve on the 2^3 mesh; the multigrid choices of Sec. 2.3's solver, which
 * the paper leaves to a library).  r, z: device, grid layout, fp64; kappa:
 * device, element layout, fp64.  The kernels are the ones the tuning selects
 * (stencil engine, fusions, coarse single-kernel V-cycle from vsmall_fp64). */
int mlmc_vcycle(mlmc_ctx* ctx, int32_t n, int64_t count, const double* kappa,
                const double* r, double* z);

/* mlmc_vcycle in fp32, the preconditioner of the mixed-precision inner solve:
 * r, z, kappa fp32, with the tuning's fp32 stencil engine, fusions and
 * vsmall_fp32.  The arena holds its work space (Errors: MLMC_E_NOMEM). */
int mlmc_vcycle_f32(mlmc_ctx* ctx, int32_t n, int64_t count, const float* kappa,
                    const float* r, float* z);

/* Solve A(kappa) u = b for f = 1 (b_i = h^3, whatever the configured
 * forcing) for `count` samples with the configured solver and precision, starting from u = 0, to the configured
 * true relative residual.  u: device, grid layout, fp64 (output);
 * iters (host, may be NULL) receives the PCG iteration count per sample.
 * Returns MLMC_E_NOCONV if some sample did not converge (u holds the last
 * iterate). */
int mlmc_solve(mlmc_ctx* ctx, int32_t n, int64_t count, const double* kappa,
               double* u, int32_t* iters);

/* K13 -- q[s] = Q(u_s) (device, fp64, [count]) for the configured QoI:
 * domain average h^3 sum_i u_i, or the mean of u_h over [1/4, 3/4]^3 as the
 * exact integral of the trilinear interpolant (Sec. 2.1, "an integral of u
 * on a sub-region").  u: device, grid layout. */
int mlmc_qoi(mlmc_ctx* ctx, int32_t n, int64_t count, const double* u, double* q);

/* mlmc_qoi for callers that cannot allocate (code under graph capture, tight
 * serving loops, harnesses that forbid allocation): the same QoI with the
 * same kernels and bits, but the per-sample partial sums go to a static
 * 16 MiB device array of the library (each GPU holds its own copy until the
 * process ends) instead of the arena, so the call allocates nothing, carves
 * nothing and leaves the context's cached work space alone.  u, q as in
 * mlmc_qoi.  Limit: count x ceil(vectors / 2048) partial sums must fit the
 * scratch (about 33000 samples of 64^3, 2 million of 8^3); a larger count is
 * refused with MLMC_E_INVALID.  Calls that overlap on one GPU (several
 * streams or threads at once) share the array and race; calls in order on one
 * stream do not (every partial sum is written before it is read). */
int mlmc_qoi_noalloc(mlmc_ctx* ctx, int32_t n, int64_t count, const double* u, double* q);

/* The random forcing of samples first .. first+count-1 of `level` on mesh n
 * (device arrays, sample-major): xi_f of sample i is drawn like xi
 * (mlmc_draw_xi) but from the Philox blocks with counter (i, level, j, 2);
 * f (count x n^3, fp64) receives exp(g_f) at the element centroids, g_f =
 * sum_m sqrt(lambda_m) phi_m xi_f,m (the KLE of mlmc_field); b (count x
 * mlmc_grid_stride(n), fp64, grid layout) the load vector of that
 * elementwise-constant f: b_i = (h^3 / 8) sum of f over the 8 elements around
 * interior node i (each element integrates a Q1 hat function to h^3 / 8), 0 at
 * boundary positions.  Errors: MLMC_E_INVALID for bad arguments, MLMC_E_NOMEM
 * when the arena after the KL tables cannot hold the draw. */
int mlmc_forcing(mlmc_ctx* ctx, int32_t n, int32_t level, uint64_t first, int64_t count, double* f, double* b);

/* -------------------------------------------------- whole path (host out) */

/* Draw, field, solve and QoI for the samples first .. first+count-1 of
 * `level`; a level l > 0 sample solves the n_l and n_{l-1} meshes on the same
 * xi and returns Y = Q_l - Q_{l-1} (Sec. 2.2), level 0 returns Y = Q_0.
 * y, q_fine, q_coarse (q_coarse = 0 at level 0) are host arrays of `count`
 * doubles; iters (host, may be NULL) gets the fine-mesh iteration counts.
 * The samples are also folded into the level's running statistics on the
 * device in sample order (Welford within blocks of 64 consecutive samples,
 * blocks merged by the Chan et al. formula in order; NaN / Inf values of Y
 * are counted apart and not folded in).
 * Work is split into batches (eq. batch, read for the lanes of the tuning:
 * see mlmc_last_plan) of at most the lane capacity: max_batch samples on the
 * finest configured mesh, proportionally more on coarser levels (same DOFs
 * per batch, at most 65536 samples); the fine and coarse solves of each batch
 * are separate tasks, assigned finest mesh first to the least-loaded of the
 * lanes (Alg. incremental_greedy), which run concurrently on their own
 * streams.  Lanes that the arena cannot hold are dropped (one lane at least;
 * its batches are halved down to max_batch if needed).  A sample's result
 * does not depend on its batch or lane.
 * Errors: MLMC_E_NOMEM if the arena cannot hold one batch; MLMC_E_NOCONV or
 * MLMC_E_NONFINITE after all samples ran (outputs filled; a solve whose
 * residual turns NaN / Inf stops at once). */
int mlmc_sample_level(mlmc_ctx* ctx, int32_t level, uint64_t first, uint64_t count,
                      double* y, double* q_fine, double* q_coarse, int32_t* iters);

typedef struct mlmc_estimate_opts {
  double eps;             /* target RMSE (absolute) of the estimator, > 0 (unused with n_fixed) */
  int32_t n_pilot;        /* pilot samples per level before allocating, >= 2 */
  int32_t cost_model;     /* 0: measured GPU seconds per sample; 1: interior DOFs of the pair */
  double extra_fraction;  /* N_l is multiplied by (1 + extra_fraction), >= 0 (Sec. 2.3) */
  int32_t max_rounds;     /* allocation rounds: re-estimate V_l after each top-up, >= 1 */
  const uint64_t* n_fixed;/* host, `levels` entries, or NULL: plain MLMC with these N_l (Sec. 2.2, eq.
                             mlmc_average): every level sampled up to n_fixed[l] in one round, no pilot and
                             no allocation */
} mlmc_estimate_opts;

/* Multilevel estimate to a target RMSE on the context's fixed level set
 * (L = levels - 1): draw n_pilot samples per level (continuing each level's
 * sample indices after those already accumulated), estimate V(Y_l) by the
 * 1/N sample variance (eq. sample_variance) and the cost C_l, take
 *   N_l = ceil(2 eps^-2 sqrt(V_l / C_l) sum_i sqrt(V_i C_i) (1 + extra))
 * (eq. mlmc_num_samples), N_l >= n_pilot, and top every level up to N_l;
 * repeat with the updated variances for max_rounds rounds or until no level
 * needs more samples.  n_per_level (host, `levels` entries, may be NULL)
 * receives the final N_l; out receives the estimator.  The statistical error
 * sum_l V_l / N_l then targets eps^2 / 2 (the bias half of eq. mlmc_error is
 * not estimated).  Each round samples every level that needs samples
 * together, as one set of tasks over the lanes (see mlmc_sample_level).
 * Errors: as mlmc_sample_level; MLMC_E_NOCONV / MLMC_E_NONFINITE are returned
 * after the loop ends normally, with n_per_level and out filled (non-finite
 * samples are kept out of the statistics, unconverged ones are in them). */
int mlmc_estimate(mlmc_ctx* ctx, const mlmc_estimate_opts* opts, uint64_t* n_per_level,
                  mlmc_estimate_out* out);

typedef struct mlmc_adaptive_opts {
  double eps;             /* target RMSE (absolute) of the estimator, eq. mlmc_error, > 0 */
  int32_t l0;             /* finest level of the first round, 1 <= l0 < levels */
  int32_t n_pilot;        /* samples of a level in its first round, >= 2 */
  int32_t cost_model;     /* 0: measured GPU seconds per sample (unsampled levels scaled by their
                             DOFs); 1: interior DOFs of the pair */
  int32_t max_rounds;     /* sampling rounds after the first, >= 0 */
  double extra_fraction;  /* N_l is multiplied by (1 + extra_fraction), >= 0 */
  double alpha0;          /* decay rate of |mean(Y_l)| while one difference level exists (0: 2) */
  double beta0;           /* decay rate of V(Y_l) likewise (0: 4) */
} mlmc_adaptive_opts;

typedef struct mlmc_adaptive_info {
  int32_t L;              /* finest level in use at the end */
  int32_t rounds;         /* sampling rounds done */
  double alpha, beta;     /* last fitted rates of |mean(Y_l)| ~ c s^-alpha l and V(Y_l) ~ c s^-beta l */
  double bias;            /* estimated |E(Q - Q_L)| = c s^-alpha L / (s^alpha - 1) */
  double err;             /* sqrt(bias^2 + sum_l V_l / N_l), eq. mlmc_error */
} mlmc_adaptive_info;

/* Adaptive MLMC (Sec. 2.3 and the adaptive loop of Alg. dyn_par_sched, read
 * as a do-while loop): start with levels 0..l0; each round samples every level
 * in use up to its target (continuing its sample indices), fits
 * |mean(Y_l)| ~ c s^(-alpha l) and V(Y_l) ~ cV s^(-beta l) over l = 1..L
 * (least squares in log_s, alpha clamped to [0.5, 4], beta to [0.5, 8];
 * alpha0 / beta0 through a single level), estimates the bias of Qtilde_L as
 * the tail c s^(-alpha L) / (s^alpha - 1) and e^2 = bias^2 + sum V_l / N_l
 * (eq. mlmc_error), and stops when e <= eps.  Otherwise L grows to
 * ceil(log_s(sqrt(2) c / ((s^alpha - 1) eps)) / alpha) (eq. mlmc_num_levels,
 * capped by the configured levels) and every level's target to
 * eq. mlmc_num_samples (V of new levels from the fit, at least n_pilot);
 * targets never decrease.  s = 2.  n_per_level (host, `levels` entries, may be
 * NULL) receives the samples per level (0 beyond L), info the final L, rates
 * and error, out the estimator.  Errors: MLMC_E_INVALID for bad options, else
 * as mlmc_sample_level. */
int mlmc_estimate_adaptive(mlmc_ctx* ctx, const mlmc_adaptive_opts* opts, uint64_t* n_per_level,
                           mlmc_adaptive_info* info, mlmc_estimate_out* out);

/* ---------------------------------------------- pause-model scheduler stress */

typedef struct mlmc_pause_opts {
  int32_t n_levels;         /* levels 0 .. n_levels-1, 1 <= n_levels <= 16 */
  const int64_t* counts;    /* samples of each level (host, >= 0 each, at most 2^24 in all) */
  const int32_t* widths;    /* workgroup slots a task of the level holds, 1 .. capacity */
  double mu_us;             /* mean duration of one sample, microseconds, > 0 */
  double sigma_us;          /* standard deviation, 0 <= sigma_us <= mu_us / sqrt(3) */
  int32_t capacity;         /* P: workgroup slots of the device, 1 .. 8192 */
  int32_t batch;            /* samples per task (batch sampling), >= 1; 1 = one sample per task */
  double min_step_us;       /* shortest step, >= 0 */
} mlmc_pause_opts;

typedef struct mlmc_pause_out {
  int64_t tasks;            /* tasks run (a task: up to `batch` samples of one level) */
  int64_t steps;            /* scheduling steps (one device launch each) */
  double clock_mhz;         /* rate of the device clock the durations are counted in */
  double wall_s;            /* host time from the first launch to the end of the last step */
  double active_slot_s;     /* a: sum over tasks of width x duration (slot-seconds) */
  double ratio;             /* A = a / (P wall_s), eq. active_ratio */
  double ideal_ratio;       /* A of the same schedule with no time between steps */
  double measured_slot_s;   /* slot-seconds the workgroups spent waiting, device clock */
} mlmc_pause_out;

/* Pause-model stress of the scheduler (Sec. 5.1, "A benchmarking example"):
 * the model of a sample only waits, for a time drawn from
 * U(mu - sqrt(3) sigma, mu + sqrt(3) sigma) (sigma read as a standard
 * deviation), so a run measures the scheduling alone through the active ratio
 * A(p) = a(p) / (p t_w(p)) of eq. active_ratio, p being the capacity in
 * workgroup slots.  A task of level l (batch consecutive samples, or fewer at
 * the end) holds widths[l] slots for the sum of its samples' durations, the
 * device counterpart of a partition of q_l cores.  Durations: sample i of
 * level l takes d = a + w u, a = mu - sqrt(3) sigma, w = 2 sqrt(3) sigma, u the
 * uniform of word 0 of the Philox4x64-10 block with key (seed, 0) and counter
 * (i, l, 0, 1) (the xi draw of mlmc_draw_xi uses counter word 3 = 0), drawn
 * on the device, then counted in device clock ticks as floor(d f + 1/2), f
 * the clock rate in MHz.  Schedule (host loop, one launch per step): tasks are
 * queued finest level first, in sample order (the finest-first rule of
 * Alg. incremental_greedy); at each step boundary every queued task that fits
 * the free slots is admitted, in queue order; the step lasts
 * max(min_step, least remaining time of a running task) and every running
 * workgroup waits min(its task's remaining time, step); tasks whose time is
 * used up finish.  ticks (host, sum of counts entries, may be NULL) receives
 * each sample's duration in ticks, level-major; done_step (same size, may be
 * NULL) the step at whose end the sample's task finished (0-based).
 * Errors: MLMC_E_INVALID for bad options, MLMC_E_NOMEM when the arena after
 * the KL tables cannot hold the draws, MLMC_E_DEVICE. */
int mlmc_pause_model(mlmc_ctx* ctx, const mlmc_pause_opts* opts, int64_t* ticks, int64_t* done_step,
                     mlmc_pause_out* out);

/* ------------------------------------------------------------- tuning */

/* Execution choices that change speed, not the discrete solution each solve
 * converges to (iteration counts and last bits may change). */
typedef struct mlmc_tuning {
  int32_t zvar_fp32;      /* stencil kernel variant bits for fp32: 0 register window, 1 with the next
                             plane prefetched, 2 LDS-tiled planes, 4 LDS-tiled planes also for the
                             step that applies the coarse-grid correction (default 6) */
  int32_t zvar_fp64;      /* same for fp64 (default 2) */
  int32_t vsmall_fp32;    /* mesh from which the coarse V-cycle runs as one LDS kernel (0: off) */
  int32_t vsmall_fp64;    /* same for fp64 (at most 8) */
  int32_t cheb_degree;    /* Chebyshev smoothing degree per half V-cycle, 1..8 */
  int32_t max_batch;      /* samples per batched solve */
  int32_t graph_batch;    /* captured PCG iterations replayed per convergence check (0: no graphs) */
  int32_t fuse;           /* MLMC_FUSE_* bits: kernel fusions and packing in use (default: all but RUPDATE) */
  int32_t field;          /* fp64 KLE evaluation: 1 the dense MFMA tile GEMM; 0 (default) or 2 separable
                             (per x-row of elements, H = xi sqrt(lambda) phi_y phi_z summed over the
                             modes of each x-factor, then g = H phi_x), or the GEMM when one sample's
                             coefficients and the mesh's x-table do not fit a workgroup's LDS; the
                             bf16 precision always uses its MFMA GEMM */
  int32_t lanes;          /* lanes of a sampling round, 1..8 (default 4): concurrent streams, each solving
                             its tasks one after another (1: every batch in turn on the context stream) */
  double seconds;         /* mlmc_autotune: measured seconds per sample of the chosen setting */
} mlmc_tuning;

/* Fusion bits of mlmc_tuning.fuse. */
enum {
  MLMC_FUSE_PROLONG = 1,  /* coarse-grid correction applied inside the first post-smoothing step */
  MLMC_FUSE_UPDATE = 2,   /* PCG x/r update fused with the first smoothing step of the next V-cycle */
  MLMC_FUSE_REFINE = 4,   /* mixed precision: correction, fp64 residual and its demotion in one pass */
  MLMC_FUSE_RESTRICT = 8, /* V-cycle residual restricted to the coarse mesh without being stored */
  MLMC_FUSE_PRESMOOTH = 16, /* Chebyshev degree 1 with the LDS engine (zvar bit 2) and PROLONG and
                              RESTRICT on: the zero-start pre-smoothing step c D^-1 b of each V-cycle
                              level is formed inside the residual and the correction steps, never
                              stored (supersedes UPDATE on those levels) */
  MLMC_FUSE_DIRECTION = 32, /* LDS engine: the PCG direction p = z + beta p is formed inside the operator
                              apply q = A p, which also applies the previous step's x += alpha p (two
                              direction buffers); the last x update of a solve runs after it */
  MLMC_FUSE_RUPDATE = 64   /* with DIRECTION and PRESMOOTH: the PCG update r -= alpha q is formed inside
                              the next iteration's first V-cycle kernel (residual restriction), which
                              writes r to the other of two residual buffers and tests convergence */,
  MLMC_FUSE_SOLVE = 128,   /* mixed precision with GMG on a 4^3 or 8^3 mesh: the whole solve of a sample
                              (fp64 refinement, fp32 PCG, V-cycle) in one workgroup with every vector in
                              LDS, one launch per batch; needs vsmall_fp32 >= the mesh */
  MLMC_FUSE_PACK = 256     /* sampling rounds: the solves of two levels on the same mesh (level l's own
                              and level l+1's coarse one) share one batched solve when together they fit
                              the lane capacity of that mesh */
};

int mlmc_get_tuning(const mlmc_ctx* ctx, mlmc_tuning* out);
/* Errors: MLMC_E_INVALID for a value out of range. */
int mlmc_set_tuning(mlmc_ctx* ctx, const mlmc_tuning* t);

/* Autotuner: time whole batched solves of `batch` samples of `level` (draw,
 * field, solve, QoI; statistics are not touched) while changing one choice
 * at a time (coordinate descent over Chebyshev degree, stencil variant,
 * coarse-kernel threshold, graph batching and batch size), keep the setting
 * with the least time per sample, apply it to the context and return it in
 * *best (may be NULL).  The arena must hold a batch of `batch` samples. */
int mlmc_autotune(mlmc_ctx* ctx, int32_t level, int32_t batch, mlmc_tuning* best);

/* Running statistics of every level and the estimator of eq. mlmc_average
 * with the statistical error sum_l V(Y_l)/N_l (Sec. 2.2). */
int mlmc_get_estimate(const mlmc_ctx* ctx, mlmc_estimate_out* out);

/* Clear the running statistics of every level. */
int mlmc_reset_stats(mlmc_ctx* ctx);

/* K14 -- fold y (device, fp64, `count` values in sample order) into the
 * running statistics of `level` exactly as the whole-path calls do (Welford
 * within blocks of 64 consecutive pushes, blocks merged in order by the Chan
 * et al. formula, eq. sample_variance and eq. mlmc_average; NaN / Inf values
 * counted apart); the result does not depend on how the values are split
 * over calls.  Returns MLMC_E_NONFINITE if some value was not finite (the
 * others are folded in).  For step-level use and tests. */
int mlmc_fold_stats(mlmc_ctx* ctx, int32_t level, const double* y, uint64_t count);

/* One part of a task of a sampling round (see mlmc_sample_level). */
typedef struct mlmc_plan_task {
  int32_t level;       /* MLMC level whose draws the part solves */
  int32_t n;           /* mesh: n0 << level (the level's own), or half of it (the coarse solve of the pair) */
  uint64_t first;      /* first sample index */
  int32_t count;       /* samples */
  int32_t lane;        /* lane its task ran on */
  int32_t task;        /* index of its task (one batched solve) in assignment order */
} mlmc_plan_task;

/* The parts of the tasks of the last sampling round, tasks in assignment
 * order (finest mesh first, each to the least-loaded lane), parts in their
 * order within the task; *n receives their number (the first max of them are
 * written to out, host).  For tests of the scheduling. */
int mlmc_last_plan(const mlmc_ctx* ctx, mlmc_plan_task* out, int32_t max, int32_t* n);

/* ---------------------------------------------------------------- serving */

typedef struct mlmc_sample_result {
  uint64_t ticket;
  int32_t status;       /* MLMC_OK, MLMC_E_NOCONV or MLMC_E_NONFINITE */
  int32_t level;
  uint64_t sample;
  double y;             /* Q_l - Q_{l-1} (Q_0 at level 0) */
  double q_fine, q_coarse;
  int32_t iters;        /* fp32 inner PCG iterations of the fine solve */
  double latency_s;     /* completion - submission, host monotonic clock */
  double queue_s;       /* admission into a slot - submission */
} mlmc_sample_result;

typedef struct mlmc_serve_stats_out {
  uint64_t completed;   /* requests finished since the server started */
  double sample_dofs;   /* interior unknowns of the finished solves */
  double busy_seconds;  /* last completion - first submission */
  int32_t queued;       /* solves waiting for a slot */
  int32_t running;      /* solves in slots */
  int32_t slots[16];    /* pool capacity per mesh n0 << m */
  int32_t occupied[16];
  double slot_busy_s[16]; /* per mesh: sum over solver steps of occupied slots x step seconds */
  double slot_bytes[16];  /* per mesh: arena bytes of one slot (its share of the HBM budget) */
  double uptime_s;        /* seconds since serving started; with the two above, the active ratio
                             A = a / (p t_w) of eq. active_ratio over a window is
                             sum_m d(slot_busy_s[m]) slot_bytes[m] / (sum_m slots[m] slot_bytes[m] d(uptime_s)) */
  uint64_t lends;         /* times an idle pool's region took a guest pool of another mesh */
  uint64_t reclaims;      /* times a pool took its region back from a guest */
} mlmc_serve_stats_out;

/* Start serving: the arena after the KL tables is split into one resident
 * pool per mesh n0 << m with slots_per_mesh[m] slots (NULL: an equal share of
 * the budget per mesh, at most 4096 slots each).  Every slot holds one solve's
 * kappa, fp32 multigrid hierarchy and solver vectors until it finishes.  A
 * host thread and a stream per pool advance all occupied slots one solver
 * step at a time and admit queued solves into free slots between steps
 * (continuous batching).  The solver is the mixed-precision GMG-PCG.  While
 * serving, the batch entry points (sample_level, solve, vcycle, qoi,
 * estimate, autotune) return MLMC_E_INVALID.  Each mesh owns a region of the
 * arena (its pool; with the equal split its whole share).  When a mesh has
 * more queued solves than free slots while another mesh's pool is idle and its
 * region holds a pool of the first mesh's slot count, that region takes a
 * guest pool serving the first mesh's queue (its slots compute exactly as the
 * mesh's own); the region's owner takes it back, after the guest's running
 * solves finish, as soon as it has work of its own.  Errors: MLMC_E_NOMEM
 * when the arena cannot hold the requested pools. */
int mlmc_serve_start(mlmc_ctx* ctx, const int32_t* slots_per_mesh);

/* Stop serving; requests not finished are dropped.  Idempotent. */
int mlmc_serve_stop(mlmc_ctx* ctx);

/* Queue one MLMC sample (the paper's unit of work, a DoSample duty of Sec.
 * 4.2, for one sample index): the n_l solve and, for level > 0, the n_{l-1}
 * solve on the same xi (Sec. 2.2).  *ticket identifies it for mlmc_poll.
 * Thread-safe.  Errors: MLMC_E_BUDGET if a needed mesh has no slots. */
int mlmc_submit(mlmc_ctx* ctx, int32_t level, uint64_t sample_id, uint64_t* ticket);

/* MLMC_PENDING while the request runs; MLMC_OK with *out filled (the ticket
 * is then consumed); MLMC_E_INVALID for an unknown ticket.  Thread-safe. */
int mlmc_poll(mlmc_ctx* ctx, uint64_t ticket, mlmc_sample_result* out);

/* Queue `count` samples at once (levels[i], samples[i]); tickets (host,
 * `count` entries) receive their tickets.  Thread-safe.  On an error no
 * request of the call is queued. */
int mlmc_submit_batch(mlmc_ctx* ctx, int32_t count, const int32_t* levels, const uint64_t* samples,
                      uint64_t* tickets);

/* Wait up to timeout_s seconds for finished requests and move up to `max`
 * of them, in completion order, into out (host array); *n receives the
 * number returned (0 on timeout).  Returned tickets are consumed.
 * Thread-safe. */
int mlmc_drain(mlmc_ctx* ctx, mlmc_sample_result* out, int32_t max, int32_t* n, double timeout_s);

/* Counters of the running server.  Thread-safe. */
int mlmc_serve_stats(mlmc_ctx* ctx, mlmc_serve_stats_out* out);

/* ----------------------------------------------------------- diagnostics */

/* Enable (1) or disable (0) per-kernel event timing on the context stream
 * (clears the counters), and read the launch count, total event-timed
 * milliseconds and total algorithmic bytes (bytes a kernel must move at
 * minimum: every distinct vector read or written once, for the samples still
 * active when the kernel was launched) of kernel `kernel_id`
 * (MLMC_K_*) in `precision` (0: fp64 instance, 1: fp32 instance) since
 * timing was enabled. */
enum {
  MLMC_K_XI = 0, MLMC_K_FIELD, MLMC_K_APPLY, MLMC_K_CHEB_ZERO, MLMC_K_CHEB, MLMC_K_CHEB_XO,
  MLMC_K_RESIDUAL, MLMC_K_RESTRICT, MLMC_K_PROLONG, MLMC_K_COARSEST, MLMC_K_COARSEN,
  MLMC_K_PCG_APPLY, MLMC_K_PCG_UPDATE, MLMC_K_PCG_DOT, MLMC_K_PCG_DIRECTION,
  MLMC_K_TRUE_RESIDUAL, MLMC_K_REDUCE, MLMC_K_QOI, MLMC_K_MISC, MLMC_K_CHEB_PROLONG,
  MLMC_K_PCG_UPDATE_ZERO, MLMC_K_RESIDUAL_RESTRICT, MLMC_K_SOLVE_SMALL, MLMC_K_COUNT
};
int mlmc_set_profiling(mlmc_ctx* ctx, int32_t on);
int mlmc_kernel_time(mlmc_ctx* ctx, int32_t kernel_id, int32_t precision, int64_t* launches,
                     double* total_ms, double* bytes);

#ifdef __cplusplus
}
#endif
#endif /* MLMC_H */
