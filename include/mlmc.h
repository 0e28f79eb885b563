/*
 * mlmc.h -- C ABI of the MI355X (gfx950) library for the batched per-level
 * sample solve of the inexact (mixed-precision) multilevel Monte Carlo
 * method for -div(a grad u) = f on (0,1)^2, u = 0 on the boundary, with a
 * lognormal coefficient a = exp(Z).
 *
 * Discrete problem (the model PDE of Sec. 5.1 with the quantity of interest
 * Q = integral of u over D; vertex-centred 5-point finite volumes):
 *   level l has n_l = n0 * m^l cells per side, h_l = 1/n_l; the unknowns are
 *   the (n_l - 1)^2 interior nodes, ordered P = (iy-1)(n_l-1) + (ix-1);
 *   the coefficient is nodal, a_p = exp(Z_p), Z = xi . Phi_l^T with Phi_l the
 *   field basis (mlmc_config.field) on the (n_l+1)^2 nodes; the
 *   edge coefficient is the harmonic mean of its end nodes (or the P1
 *   element rule, mlmc_config.disc); b = h^2 f;
 *   Q = h^2 * sum_P u_P.
 *
 * Conventions for every entry point:
 *   - All *_dev pointers are device pointers owned by the caller, contiguous
 *     and row-major, aligned to their element size (8 bytes for double,
 *     4 for int32; the workspace: 256 bytes); a misaligned pointer is
 *     rejected with MLMC_EINVAL.
 *     The library never frees caller memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Work is enqueued asynchronously on it unless stated otherwise.
 *   - Return codes: MLMC_OK (0); MLMC_ENOCONV (1): the call completed but at
 *     least one sample did not reach its target (see its status bits);
 *     MLMC_PAUSED (2): a resumable estimate stopped at its round limit;
 *     negative codes mean the call failed and outputs are undefined.  The
 *     text of the last error of a context is returned by mlmc_last_error.
 *   - One context per host thread; calls on one context are not re-entrant.
 */
#ifndef MLMC_H
#define MLMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MLMC_OK 0
#define MLMC_ENOCONV 1
#define MLMC_PAUSED 2   /* mlmc_estimate_resumable stopped after max_rounds: resume from its state */
#define MLMC_EINVAL (-1)  /* bad argument: null/misaligned pointer, level out of range, NaN */
#define MLMC_ENOMEM (-2)  /* workspace smaller than mlmc_workspace_bytes */
#define MLMC_EHIP (-3)    /* HIP runtime error (text via mlmc_last_error) */
#define MLMC_ENOTIMPL (-4) /* option not available for these arguments (e.g. a dtype on this grid) */

/* Per-sample status bits (uint8). */
#define MLMC_ST_CONVERGED 1u  /* relative residual < target */
#define MLMC_ST_PROMOTED 2u   /* re-factorised in a higher precision */
#define MLMC_ST_NONFINITE 4u  /* a non-finite value was met */
#define MLMC_ST_IMAX 8u       /* iteration limit reached without convergence */

typedef struct mlmc_ctx mlmc_ctx;

/* Precision u_f of the factor (Algorithm 2.1, Sec. 2.3; formats of Sec. 2.1).
 * MLMC_F64 and MLMC_F32 factorise in their own precision.  MLMC_F16 and
 * MLMC_BF16 store the factor in 16 bits; from the 32-cell grid up (the MFMA
 * kernels) the factorisation multiplies its 16 x 16 block operands rounded
 * to that format with FP32 accumulation, on the 16-cell and smaller grids
 * it forms the factor in FP32 and rounds the stored copy.  MLMC_FP8 stores
 * the factor in FP8 E4M3 (the quarter precision q43 of Sec. 2.1, unit
 * roundoff 2^-4), formed in FP32; it is available on grids with fewer than
 * 16 cells per side only (a coarsest level such as the paper's h_0 = 1/4),
 * elsewhere the calls return MLMC_ENOTIMPL.  The correction solves run in
 * FP32 arithmetic on the stored factor for every type but MLMC_F64. */
typedef enum { MLMC_F64 = 0, MLMC_F32 = 1, MLMC_BF16 = 2, MLMC_F16 = 3, MLMC_FP8 = 4 } mlmc_dtype;

/* Linear solver of one sample:
 *   MLMC_DIRECT    FP64 factorisation and solve, no refinement loop.
 *   MLMC_DIRECT_IR factorisation in factor_dtype, then Algorithm 2.1:
 *                  FP64 residual, correction solve with the stored factor
 *                  (FP32 arithmetic), FP64 update, stop when
 *                  ||b - A x||_2 / ||b||_2 < eps (strict), at most
 *                  ir_max_iter corrections (Sec. 2.3).
 *   MLMC_MINRES    Jacobi-scaled MINRES in FP64 (Sec. 2.2), run until its
 *                  recurrence estimate of the scaled relative residual is
 *                  below 0.9 eps; the sample has converged when the true
 *                  unscaled FP64 relative residual ||b - A x||/||b|| < eps,
 *                  otherwise MINRES restarts from that residual (at most 8
 *                  restarts, minres_max_iter iterations in all).
 *   MLMC_MINRES_IR MINRES as the inner solver of iterative refinement
 *                  (Sec. 2.3 with a Krylov correction solve): each inner
 *                  MINRES stores its vectors in FP32 and reduces the scaled
 *                  correction residual by max(eps / (2 rel), 1e-5); FP64
 *                  residual and update, the same stop test, at most
 *                  ir_max_iter refinements and minres_max_iter inner
 *                  iterations in all.  factor_dtype is ignored by both.
 *   MLMC_MGCG      conjugate gradients in FP64 preconditioned by one
 *                  geometric multigrid V-cycle in FP32 (red-black
 *                  Gauss-Seidel smoothing, edge coefficients coarsened by
 *                  series averaging, grids down to 2 cells), a solver whose
 *                  cost grows like the number of unknowns (gamma = 2 of the
 *                  cost model of Sec. 4.4); stops on the true FP64 relative
 *                  residual < eps, at most minres_max_iter iterations.
 *                  factor_dtype is ignored. */
typedef enum { MLMC_DIRECT = 0, MLMC_DIRECT_IR = 1, MLMC_MINRES = 2, MLMC_MINRES_IR = 3,
               MLMC_MGCG = 4 } mlmc_solver;

typedef struct {
    int32_t n0;              /* cells per side on level 0 (power of two, >= 4) */
    int32_t m;               /* refinement factor; only 2 is supported */
    int32_t L_max;           /* finest level; n0 * 2^L_max <= 256 */
    int32_t K;               /* number of KL modes, 1..512 */
    double sigma2;           /* variance of Z */
    double corr_len;         /* correlation length lambda of exp(-|x-y|/lambda) */
    double f;                /* constant right-hand side */
    double k_p;              /* accuracy constant of Sec. 4.3 (0.05) */
    double alpha, beta, gamma; /* MLMC rates: bias O(h^alpha), variance O(h^beta)
                                * (2, 4 for this problem), cost per grid
                                * (n-1)^gamma in the estimator's cost model
                                * (4: the factorisation's flops) */
    int32_t ir_max_iter;     /* Algorithm 2.1 i_max (10) */
    int32_t minres_max_iter; /* MINRES iteration cap (e.g. 5000) */
    uint64_t seed;           /* seed of the counter-based xi generator */
    int32_t field;           /* log-coefficient Z = xi . Phi^T (xi ~ N(0,1)):
                              * 0: separable exponential-covariance KL expansion
                              *    (sigma2, corr_len; K modes by decreasing eigenvalue);
                              * 1: the trigonometric expansion of Sec. 5.1,
                              *    Z = sum_{j=1..K} xi_j sigma j^(-field_q) sin(2 pi j x1) cos(2 pi j x2)
                              *    (the paper's s = K, q = field_q, omega_j = sigma xi_j ~ N(0, sigma2)) */
    double field_q;          /* decay exponent q of field 1 (unused by field 0) */
    int32_t disc;            /* edge coefficients of the 5-point operator:
                              * 0: vertex-centred finite volumes, the harmonic mean of
                              *    the edge's end nodes;
                              * 1: P1 finite elements (Sec. 3; the discretisation of the
                              *    paper's experiments, Sec. 5.1) on the right triangles of
                              *    the cells cut along (x, y)-(x+h, y+h), the coefficient
                              *    interpolated linearly: edge (x,y)-(x+h,y) gets
                              *    (2a(x,y) + 2a(x+h,y) + a(x+h,y+h) + a(x,y-h)) / 6 and edge
                              *    (x,y)-(x,y+h) gets (2a(x,y) + 2a(x,y+h) + a(x+h,y+h) + a(x-h,y)) / 6;
                              *    b = h^2 f and Q = h^2 sum u are the same for both. */
    double std_eps;          /* standard MLMC (mlmc_estimate with mixed = 0) with an
                              * iterative solver solves every system to this relative
                              * residual (0: 1e-6, the paper's MINRES setting, Sec. 5.1) */
} mlmc_config;

typedef struct {
    mlmc_dtype factor_dtype; /* u_f; ignored by MLMC_DIRECT (always FP64) */
    mlmc_solver solver;
    double eps_fine;         /* target relative residual of the level-l solve */
    double eps_coarse;       /* target of the coarse partner (level l-1) */
    int32_t promote;         /* 1: re-solve non-converged samples in the next precision */
} mlmc_level_opts;

typedef struct {
    int64_t n;                       /* samples in this call */
    double sum_y, sum_y2;            /* sums of Y_l and Y_l^2 (FP64, fixed order) */
    double sum_qf, sum_qc;           /* sums of Q_l and Q_{l-1} */
    int64_t n_promoted, n_noconv;    /* samples re-solved / not converged */
    double mean_iters;               /* mean corrections (IR) or iterations (MINRES), fine grid */
    double gpu_ms;                   /* device time of the call (event-timed) */
    double mean_iters_coarse;        /* the same for the coarse partner (0 at level 0) */
} mlmc_level_stats;

typedef struct {
    double estimate;   /* Q-hat = sum_l Y-hat_l (eq. of the MLMC estimator, Sec. 4.1) */
    double var_est;    /* sum_l s_l^2 / N_l */
    int32_t L;         /* finest level used */
    int32_t converged; /* bias and variance tests both met */
    int64_t N[16];     /* samples per level */
    double Yhat[16], s2[16], C[16], eps[16];
    double wall_s;     /* host wall time of the call */
    double gpu_ms;     /* sum of device times of the level calls */
    int64_t n_promoted[16]; /* samples per level re-solved with an FP64 factor */
    int64_t n_noconv[16];   /* samples per level that missed their target (any
                             * non-zero entry ends the call with MLMC_ENOCONV) */
} mlmc_result;

/* Create a context: solves the KL eigen-equation on the host, builds Phi_l
 * for every level 0..L_max in FP64 and uploads it (the only host->device
 * traffic of the set-up).  No sample work.  Returns MLMC_EINVAL for an
 * unsupported configuration. */
int mlmc_create(const mlmc_config *cfg, mlmc_ctx **out);
int mlmc_destroy(mlmc_ctx *ctx);
const char *mlmc_last_error(const mlmc_ctx *ctx);

/* Cells per side of level `level`, or -1. */
int32_t mlmc_level_cells(const mlmc_ctx *ctx, int32_t level);

/* delta_0..delta_L of the accuracy rule of Sec. 4.3 (the equation that
 * chooses the precisions) with the configured rates, the bias exponent of
 * delta 1 and its variance exponent 2 (the error lemma of Sec. 4.5):
 * delta_l = (k_p h_l^beta)^(1/2) for l < L,
 * delta_L = min((k_p h_L^beta)^(1/2), k_p h_L^alpha); with alpha = 2,
 * beta = 4 this is Sec. 4.5's sqrt(k_p) h_l^2 and k_p h_L^2.  Into
 * eps_out[0..L] (host memory). */
int mlmc_accuracy_targets(const mlmc_ctx *ctx, int32_t L, double *eps_out);

/* Copy Phi_level, stored transposed as [K][(n+1)^2] FP64 (node
 * p = iy*(n+1)+ix), into the caller's device buffer phit_dev (async on
 * stream).  Phi[p,k] = sigma sqrt(mu_i mu_j) phi_i(x_p) phi_j(y_p) for the
 * k-th selected mode (i, j) in the order of decreasing mu_i mu_j, ties by
 * (i, j). */
int mlmc_get_kl_basis(const mlmc_ctx *ctx, int32_t level, double *phit_dev, void *stream);

/* Bytes of device workspace that mlmc_sample_level (level >= 0), or
 * mlmc_solve / mlmc_grad on grid `level`, need for n_samples samples with
 * these options.  The same workspace serves a following mlmc_grad. */
size_t mlmc_workspace_bytes(const mlmc_ctx *ctx, int32_t level, int64_t n_samples,
                            const mlmc_level_opts *opts);

/* xi[n x K] (FP64) for samples first_sample .. first_sample+n-1 of `level`,
 * from the counter-based generator: SplitMix64 output i for seed s is
 * mix(s + (i+1) 0x9E3779B97F4A7C15); coefficient k of sample j uses pair
 * p = k/2 and outputs i_w = ((((level<<32)|j)<<8|p)<<1)|w, w = 0,1;
 * u1 = ((o0>>11)+1) 2^-53, u2 = (o1>>11) 2^-53, r = sqrt(-2 ln u1),
 * xi_2p = r cos(2 pi u2), xi_2p+1 = r sin(2 pi u2).  Requires K <= 512,
 * sample index < 2^32. */
int mlmc_fill_xi(const mlmc_ctx *ctx, int32_t level, int64_t first_sample, int64_t n,
                 double *xi_dev, void *stream);

/* Replace the seed of the counter-based generator (mlmc_fill_xi and the xi
 * that mlmc_estimate draws), e.g. for independent repetitions of Algorithm
 * 4.1 on one context; nothing else changes. */
int mlmc_set_seed(mlmc_ctx *ctx, uint64_t seed);

/* Batched solve of n samples on the grid of level `level` (no pairing):
 * field GEMM, assembly, factorisation, solve to opts->eps_fine with
 * opts->solver, and Q.  Outputs: q_dev[n]; u_dev[n x (n_l-1)^2] (optional,
 * FP64 solution); status_dev[n] (optional); iters_dev[n] (optional).
 * The workspace keeps the factor, scaling, coefficient and solution for a
 * following mlmc_grad on the same samples.  The call synchronises the
 * stream before it returns (it reads the non-converged count back to return
 * MLMC_ENOCONV). */
int mlmc_solve(mlmc_ctx *ctx, int32_t level, int64_t n, const double *xi_dev,
               const mlmc_level_opts *opts, void *ws_dev, size_t ws_bytes, double *q_dev,
               double *u_dev, uint8_t *status_dev, int32_t *iters_dev, void *stream);

/* One MLMC level (eq. of the MLMC estimator and Algorithm 4.1, Secs. 4.1
 * and 4.3): for each xi row s, Q_l(s) on grid l solved to eps_fine and, for
 * l >= 1, Q_{l-1}(s) on grid l-1 from the same xi row solved to eps_coarse;
 * Y_l = Q_l - Q_{l-1} (Y_0 = Q_0).  q_coarse_dev may be NULL for l = 0.
 * status_dev (optional) holds the fine status in bits 0-3 and the coarse
 * status in bits 4-7.  If stats_host is not NULL the call synchronises the
 * stream and fills it (level sums in FP64, fixed summation order). */
int mlmc_sample_level(mlmc_ctx *ctx, int32_t level, int64_t n, const double *xi_dev,
                      const mlmc_level_opts *opts, void *ws_dev, size_t ws_bytes,
                      double *q_fine_dev, double *q_coarse_dev, double *y_dev,
                      uint8_t *status_dev, mlmc_level_stats *stats_host, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * mlmc_sample_level with the workspace taken from a fixed scratch array that
 * the library holds on every device it runs on (MLMC_NOALLOC_SCRATCH_BYTES,
 * kept until the process ends; its device address is taken once per device
 * at mlmc_create).  The caller still passes xi and the outputs, with the
 * meaning, layout and synchronisation of mlmc_sample_level.  The call
 * allocates nothing (no hipMalloc/hipFree; kernel timing records of
 * mlmc_profile are not taken during it).  MLMC_ENOMEM when
 * mlmc_workspace_bytes(ctx, level, n, opts) exceeds the scratch size.
 * Every call on a device, from any context, shares that device's array and
 * finds the previous call's contents there (the kernels initialise what they
 * read); calls that overlap on one device, on different streams or from
 * different threads, race and must be serialised by the caller. */
#define MLMC_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int mlmc_sample_level_noalloc(mlmc_ctx *ctx, int32_t level, int64_t n, const double *xi_dev,
                              const mlmc_level_opts *opts, double *q_fine_dev, double *q_coarse_dev,
                              double *y_dev, uint8_t *status_dev, mlmc_level_stats *stats_host,
                              void *stream);

/* Several MLMC levels in one call: level levels[i] with n[i] samples and
 * xi_dev[i] ([n[i] x K]) under opts[i].  Every level's fine and coarse grids
 * run concurrently on streams forked from `stream` and joined back to it,
 * so uneven work (many small coarse samples, few large fine ones) shares the
 * GPU.  With use_graph == 0 the grids are spread over four streams of the
 * context, one per hardware queue of the process: the most expensive grid
 * alone on the first, the others longest first onto the least loaded.  With
 * use_graph != 0 every level gets two streams (fine, coarse), and the whole
 * fork/join is captured once into a HIP graph and replayed while the
 * arguments (pointers, sizes, options) stay the same.  Both give the same
 * results.  The workspace is mlmc_levels_workspace_bytes() bytes; y_dev (may be
 * NULL, or an array of n_levels device pointers, entries may be NULL) gets
 * Y_l; stats_host (may be NULL, else n_levels entries) makes the call
 * synchronise and report the level sums (gpu_ms: the whole call). */
size_t mlmc_levels_workspace_bytes(const mlmc_ctx *ctx, int32_t n_levels, const int32_t *levels,
                                   const int64_t *n, const mlmc_level_opts *opts);
int mlmc_sample_levels(mlmc_ctx *ctx, int32_t n_levels, const int32_t *levels, const int64_t *n,
                       const double *const *xi_dev, const mlmc_level_opts *opts, void *ws_dev,
                       size_t ws_bytes, double *const *y_dev, mlmc_level_stats *stats_host,
                       int32_t use_graph, void *stream);

/* Autotuner: on the given level and samples (xi_dev [n x K], the workspace
 * of mlmc_sample_level) times every candidate configuration of each of the
 * level's grids as the whole solve of that grid (factorisation and
 * refinement) and keeps the fastest in the context for the factor dtype of
 * opts and that grid, for every later call.  Candidates: the refinement
 * kernel's waves per block-row pair (1 or 2, grids with n >= 64) and, for
 * the FP16/BF16 factors on grids with n >= 32, the factorisation's block
 * products in the storage format (faster, a less accurate factor) or in
 * FP32.  chosen[0] (fine grid) and chosen[1] (coarse grid) receive
 * waves | (fp32_products << 4) (0 = a single configuration).
 * Synchronises the stream. */
int mlmc_autotune(mlmc_ctx *ctx, int32_t level, int64_t n, const double *xi_dev,
                  const mlmc_level_opts *opts, void *ws_dev, size_t ws_bytes, int32_t *chosen,
                  void *stream);

/* Algorithm 4.1 (adaptive MPML, Sec. 4.3) driven on the GPU: L starts at 1,
 * N_0 = N_1 = n_init; each round recomputes delta_l (Sec. 4.5), tops every
 * level up to N_l with fresh counter-based xi, updates
 * N_l = ceil(sqrt(V_l/C_l) (2/TOL^2) sum_k sqrt(V_k C_k)) with V_l = s_l^2
 * and the deterministic cost C_l = (n_l-1)^gamma + (n_{l-1}-1)^gamma, adds a level
 * while |Y-hat_L| > (m^alpha - 1)/sqrt(2) TOL, and stops when that test and
 * sum_l s_l^2/N_l <= TOL^2/2 hold and no level needs more samples.
 * dtype_per_level[0..L_max] selects u_f per level (ignored by the
 * solvers without a factor).  mixed = 0 runs standard MLMC (Algorithm 4.1
 * without its precision step): with MLMC_DIRECT or MLMC_DIRECT_IR every
 * solve is the FP64 direct solve; with an iterative solver every solve runs
 * that solver to the fixed tolerance cfg.std_eps.  Each level
 * streams its chunks on one of the context's queue streams; one
 * synchronisation per round, and within a round the host waits for the
 * finest level alone: when its samples make the level test add a level, that
 * level's first n_init samples start in the same round (the decisions, N_l
 * and results are those of starting them in the next round).  Device memory: a per-level chunk workspace
 * (8 GiB per level, up to 32 GiB for a level whose first n_init samples then
 * fit one chunk), allocated on the first call and kept by the context for
 * later calls (grown when a call needs more, freed by mlmc_destroy).
 * Every Y_l must reach its accuracy (Algorithm 4.1): a round in which any
 * sample misses its target after promotion, or whose level sums are not
 * finite, ends the call with MLMC_ENOCONV; out then holds the state after
 * that round (converged = 0, n_noconv per level). */
int mlmc_estimate(mlmc_ctx *ctx, double tol, int32_t n_init, const mlmc_dtype *dtype_per_level,
                  mlmc_solver solver, int32_t mixed, mlmc_result *out, void *stream);

/* Estimator state at a round boundary of Algorithm 4.1 (checkpoint and
 * resume): everything the later rounds depend on.  Level l's next sample
 * index is done[l], so a run resumed from a state draws the same samples,
 * adds their sums in the same order and ends with the same result as an
 * uninterrupted run. */
typedef struct {
    int32_t L;                 /* finest level so far (1..L_max) */
    int32_t rounds;            /* rounds completed */
    int64_t N[16];             /* target samples of level l (l <= L) */
    int64_t done[16];          /* samples taken on level l: its next sample index */
    double s1[16], s2[16];     /* sums of Y_l and Y_l^2, in chunk order */
    int64_t n_promoted[16];    /* samples re-solved in FP64 so far */
    int64_t n_noconv[16];      /* samples that missed their target so far */
    double gpu_ms;             /* device time so far */
    double tol;                /* the call's parameters, checked on resume */
    int32_t n_init, mixed, solver;
    int32_t dtype[16];         /* dtype_per_level (0 when NULL) */
    uint64_t seed;             /* the context's generator seed */
} mlmc_estimate_state;

/* mlmc_estimate with a checkpoint.  resume = NULL starts afresh; otherwise
 * the rounds continue from that state, whose parameters and seed must be
 * this call's and this context's (MLMC_EINVAL otherwise).  max_rounds > 0
 * stops after that many rounds of this call: the call then returns
 * MLMC_PAUSED if the estimator had not finished.  state_out (may be NULL)
 * receives the state after the last completed round; out holds the
 * estimate over the levels so far (a level added in the last round counts
 * with the samples it has).  Otherwise as mlmc_estimate, which equals this
 * call with resume = NULL, max_rounds = 0 and state_out = NULL. */
int mlmc_estimate_resumable(mlmc_ctx *ctx, double tol, int32_t n_init, const mlmc_dtype *dtype_per_level,
                            mlmc_solver solver, int32_t mixed, const mlmc_estimate_state *resume,
                            int32_t max_rounds, mlmc_estimate_state *state_out, mlmc_result *out,
                            void *stream);

/* Adjoint gradient dQ/dxi on grid `level` for the n samples of the
 * preceding mlmc_solve on the same workspace with the same opts (solver
 * MLMC_DIRECT or MLMC_DIRECT_IR; the stored factor and solution are reused):
 * solves A lambda = h^2 1 (the gradient of Q = h^2 sum u in u) with the
 * stored factor and FP64 refinement to the relative residual eps_adjoint
 * (non-converging samples are re-solved with an FP64 factor), forms
 *   dQ/dZ_e = -sum_{edges (e,o)} (lambda_e - lambda_o)(u_e - u_o)
 *             2 a_o^2 a_e / (a_e + a_o)^2      (u, lambda = 0 on the boundary)
 * and grad_xi[s,k] = grad_q[s] * sum_e dQ/dZ_e Phi[e,k]  ([n x K] FP64).
 * grad_q_dev[n] may be NULL (taken as 1).  xi_dev must be the forward's xi.
 * Not part of the paper: the exact derivative of the discrete Q. */
int mlmc_grad(mlmc_ctx *ctx, int32_t level, int64_t n, const double *xi_dev,
              const double *grad_q_dev, const mlmc_level_opts *opts, double eps_adjoint,
              void *ws_dev, size_t ws_bytes, double *grad_xi_dev, void *stream);

/* Multilevel Markov chain Monte Carlo with the same per-level solves (the
 * extension of the concluding remark of Sec. 4: the accuracy rule is a
 * statement about the quantity of interest, not about the sampler).
 * Bayesian set-up: prior xi ~ N(0, I_K) (the field of the context), data
 * d_j = u(x_j) + N(0, noise_sd^2) at n_obs observation nodes, log-likelihood
 * of level l  -sum_j (d_j - u_l(x_j))^2 / (2 noise_sd^2).  E_{pi_L}[Q] is
 * estimated by the telescoping sum E_{pi_0}[Q_0] + sum_l E[Y_l]:
 *   level 0: `chains` independent preconditioned Crank-Nicolson chains
 *   (xi' = sqrt(1 - b^2) xi + b w), Y_0 = Q_0 of the state;
 *   level l >= 1: `chains` chains on the level-l posterior whose proposal is
 *   the current state of a pCN chain on the level-(l-1) posterior, advanced
 *   `subsample` steps per fine step, accepted with
 *   min(1, L_l(xi') L_{l-1}(xi) / (L_l(xi) L_{l-1}(xi'))), and
 *   Y_l = Q_l(fine state) - Q_{l-1}(coarse state) (Dodwell et al.'s
 *   multilevel MCMC with an independence proposal from the coarse chain).
 * All chains of a level step together: every step is one batched solve of
 * `chains` samples with opts[l] (eps_fine on grid l, eps_coarse on grid
 * l-1).  Chains start at xi = 0; the first burn_in steps are not recorded.
 * Random numbers: the context's counter-based generator (mlmc_fill_xi) on
 * reserved level indices 4096 + 8 l + k (k = 0 fine proposals, 1 coarse
 * proposals, 2 fine acceptance, 3 coarse acceptance) at sample index
 * step * chains + chain (coarse: (step * subsample + s) * chains + chain);
 * a step's acceptance uniform is Phi(z) of the first normal.  Observation
 * nodes must be interior nodes of the level-0 grid.  Allocates its device
 * buffers for the call; synchronises the stream. */
typedef struct {
    int32_t L;                 /* finest level, 0..L_max */
    int32_t chains;            /* chains per level (1..65536), the batch of every solve */
    int32_t steps[16];         /* recorded steps per chain on level l */
    int32_t burn_in;           /* steps per chain discarded at the start of every level */
    int32_t subsample;         /* coarse pCN steps per fine step (levels >= 1) */
    double pcn_beta;           /* pCN step size b, 0 < b <= 1 */
    double noise_sd;           /* observation noise standard deviation */
    int32_t n_obs;             /* observation nodes, 1..64 */
    double obs_x[64], obs_y[64];  /* node coordinates (multiples of 1/n0, inside (0,1)) */
    double obs_value[64];      /* observed values d_j */
    mlmc_level_opts opts[16];  /* solver of level l's fine and coarse grids */
    uint64_t seed;             /* generator seed of the chains' random numbers */
} mlmc_mcmc_config;

typedef struct {
    double estimate;           /* sum_l Yhat[l] */
    double Yhat[16];           /* mean of Y_l over chains and recorded steps */
    double var_mean[16];       /* variance of Yhat[l] from the spread of the chain means */
    double accept[16];         /* acceptance rate of level l's chains */
    double accept_coarse[16];  /* of its coarse pCN chains (levels >= 1) */
    int64_t solves;            /* batched solves issued */
    double wall_s;
} mlmc_mcmc_result;

int mlmc_mcmc(mlmc_ctx *ctx, const mlmc_mcmc_config *cfg, mlmc_mcmc_result *out, void *stream);

/* Multi-index Monte Carlo with the same per-grid solves (the second sampler
 * of the concluding remark of Sec. 4, Haji-Ali, Nobile and Tempone's
 * estimator): E[Q] is estimated by the sum over an index set of the sample
 * means of the mixed differences
 *   D_a = Q_(l,k) - Q_(l-1,k) - Q_(l,k-1) + Q_(l-1,k-1),   a = (l, k),
 * terms with l - 1 < 0 or k - 1 < 0 left out.  Index l is the grid (n0 2^l
 * cells per side); index k truncates the context's field to its first
 * K_k = min(K, K0 2^k) modes (the modes are ordered by decreasing variance):
 * Q_(l,k)(xi) = Q_l(xi with every coefficient from mode K_k on set to 0).
 * Index i has N[i] independent samples, drawn with the context's generator
 * (mlmc_fill_xi) on the reserved level index 8192 + i, sample index
 * 0 .. N[i]-1; the (up to) four solves of a sample share its xi and run with
 * opts[i]: eps_fine on grid l, eps_coarse on grid l - 1, the same factor
 * dtype and solver on both.  The indices are spread over the context's
 * queue streams (most expensive first onto the least loaded), each stream
 * running its indices' samples in chunks that fit a 4 GiB solve workspace
 * of its own.  Per index the result holds the sample mean and variance of
 * D_a (per-chunk fixed-order sums, added in chunk order), and the samples
 * any of whose solves were promoted to FP64 or did not converge; the call
 * returns MLMC_ENOCONV when any did not.
 * Indices must be distinct, 1 <= K0 <= K, N[i] >= 2.  Allocates its device
 * buffers for the call; synchronises the stream. */
typedef struct {
    int32_t n_idx;             /* indices in the set, 1..64 */
    int32_t idx_l[64];         /* grid index l of index i, 0..L_max */
    int32_t idx_k[64];         /* truncation index k of index i, 0..15 */
    int64_t N[64];             /* samples of index i (>= 2) */
    int32_t K0;                /* modes kept at truncation index 0 */
    mlmc_level_opts opts[64];  /* solver of index i's grids */
    uint64_t seed;             /* generator seed of the indices' xi */
} mlmc_mimc_config;

typedef struct {
    double estimate;           /* sum_i mean[i] */
    double var_estimate;       /* sum_i var[i] / N[i] */
    double mean[64];           /* sample mean of D_a over index i's samples */
    double var[64];            /* sample variance of D_a (N - 1 normalisation) */
    int64_t n_promoted[64];    /* samples with a solve promoted to FP64 */
    int64_t n_noconv[64];      /* samples with a solve that did not converge */
    int64_t solves;            /* batched solves issued */
    double wall_s;
} mlmc_mimc_result;

int mlmc_mimc(mlmc_ctx *ctx, const mlmc_mimc_config *cfg, mlmc_mimc_result *out, void *stream);

/* Kernel timing for measurement.  While enabled, the library brackets each
 * launch of the field, assembly, factor, solve and residual kernels with HIP
 * events on the caller's stream and records (kernel kind, grid n, samples).
 * mlmc_profile_read synchronises, and for kind (0 field, 1 assembly (none on
 * the n = 16 grid, whose factorisation forms the scaled operator itself and
 * counts under 2, except for MINRES), 2 factor, 3 refinement (initial solve + Algorithm 2.1 loop), 4 residual,
 * 5 MINRES, 6 FP64 re-factorisation of promoted samples, 7 FP64 refinement
 * of promoted samples; 6 and 7 launch over the promotion slots and exit at
 * once for slots beyond the device-side count) and grid n returns the
 * summed device time,
 * the number of launches and the summed samples over all recorded launches,
 * then keeps the records (reset with mlmc_profile(ctx, 1) again). */
int mlmc_profile(mlmc_ctx *ctx, int32_t enable);
int mlmc_profile_read(mlmc_ctx *ctx, int32_t kind, int32_t n, double *total_ms, int64_t *launches,
                      int64_t *samples);

#ifdef __cplusplus
}
#endif
#endif /* MLMC_H */
