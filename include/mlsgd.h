/*
 * mlsgd.h -- C ABI of libmlsgd: one MLMC gradient estimate of the
 * entropic-risk objective for 3-D elliptic optimal control under a random
 * diffusion coefficient, on one AMD Instinct MI355X (gfx950).
 *
 * Method: Baumgarten, Guth, Schneiderhan, Vanzan, "Multilevel Stochastic
 * Gradient Descent for Risk-Averse PDE-Constrained Optimization".
 *
 * Common conventions
 *   - Grids: level i has n_i vertices per axis on the unit cube, h_i =
 *     1/(n_i - 1); levels are nested, n_{i+1} = 2 n_i - 1.  A field on a grid
 *     is an array of n^3 doubles, vertex (ix, iy, iz) at index
 *     (ix*n + iy)*n + iz (z fastest).  The Dirichlet boundary is 0: boundary
 *     entries of inputs are ignored and boundary entries of outputs are 0.
 *   - Operator (Sec. 5 model problem, finite-difference form):
 *       (A y)_v = h^-2 sum over the 6 faces (v,w) of a_f (y_v - y_w),
 *       a_f = 2 a_v a_w / (a_v + a_w), a = exp(log a) at the vertices,
 *       log a(x) = sum_{k in {1..K}^3} sqrt(sigma2 lam_k) xi_k prod_d cos(pi k_d x_d),
 *       lam_k = (1 + |k|^2)^(-5/2); term j = ((k1-1)K + (k2-1))K + (k3-1).
 *   - Draws: xi_j ~ N(0,1) from Philox4x64-10 with key (seed, 0) and counter
 *     (block, sample, level, tag), Box-Muller on the word pairs (w0,w1) and
 *     (w2,w3) of each block, u = ((w >> 11) + 1/2) 2^-53.  The fine and the
 *     coarse solve of level i share the level-i draw (Sec. 2.2).
 *   - Control transfer: the right-hand side on grid i is R^(finest -> i)(f + u)
 *     with full weighting R; adjoints move up by trilinear prolongation.
 *   - Inner products: <a, b>_h = h^3 sum over interior vertices.  Gradients
 *     are L^2_h Riesz representers on the finest grid.
 *
 * Memory: every array argument marked "device" is a device pointer owned by
 * the caller, contiguous, read or written asynchronously on the context's
 * stream.  Host arguments are read before the call returns.  Stats structs
 * are host memory, filled after an internal synchronisation of the stream.
 *
 * Errors: every entry point returns an mlsgd status code; on failure
 * mlsgd_last_error(ctx) holds a message.  One context per stream; a context
 * is not thread-safe.
 */
#ifndef MLSGD_H
#define MLSGD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MLSGD_OK 0
#define MLSGD_EINVAL (-1)    /* invalid argument (non-nested grids, M < 1, ...) */
#define MLSGD_ENOCONV (-2)   /* a solve missed rtol; outputs are still written */
#define MLSGD_ENONFINITE (-3)/* NaN or Inf in an input or a result */
#define MLSGD_EHIP (-4)      /* HIP runtime error; see mlsgd_last_error */
#define MLSGD_EOOM (-5)      /* device allocation failed */

#define MLSGD_MAX_LEVELS 8
#define MLSGD_MAX_K 5

/* precision of the solves */
#define MLSGD_FP64 0          /* FP64 everywhere */
#define MLSGD_MIXED_FP32 1    /* FP32 V-cycles inside FP64 refinement */
#define MLSGD_MIXED_BF16 2    /* as MIXED_FP32, the smoother's 1/a cache in bfloat16 */

/* outer solver */
#define MLSGD_SOLVER_CG 0     /* unpreconditioned conjugate gradients */
#define MLSGD_SOLVER_MGPCG 1  /* multigrid-preconditioned CG */

typedef struct mlsgd_problem {
  int32_t n_levels;                    /* number of levels, 1..MLSGD_MAX_LEVELS */
  int32_t grid_n[MLSGD_MAX_LEVELS];    /* vertices per axis, nested, n_0 >= 3 */
  uint64_t seed;                       /* Philox key word 0 */
  int32_t kl_K;                        /* KL terms per axis, 1..MLSGD_MAX_K */
  double kl_sigma2;                    /* KL variance scale sigma^2 >= 0 */
  double theta;                        /* entropic risk parameter >= 0 */
  double alpha;                        /* Tikhonov weight (the paper's lambda) >= 0 */
  int32_t precision;                   /* MLSGD_FP64 | MLSGD_MIXED_* */
  int32_t solver;                      /* MLSGD_SOLVER_* */
  double rtol;                         /* true relative residual target per solve */
  int32_t max_iters;                   /* outer iterations per solve */
  double u_lo, u_hi;                   /* box of U_ad; u_lo > u_hi means no box */
  const double* f;                     /* device, finest grid, nullable (= 0) */
  const double* y_d;                   /* device, finest grid target */
  int32_t kl_law;                      /* MLSGD_LAW_*: law of the KL draws */
  double kl_rho;                       /* correlation length of MLSGD_LAW_EXPONENTIAL, > 0 */
} mlsgd_problem;

/* Laws of the KL expansion log a = sum c_k phi_k with c = sqrt(sigma2 lam) xi.
 * ALGEBRAIC: xi ~ N(0, 1), lam_k = (1 + |k|^2)^(-5/2),
 *   phi_k = cos(k1 pi x) cos(k2 pi y) cos(k3 pi z), draw t = ((k1-1)K + (k2-1))K + (k3-1).
 * EXPONENTIAL (Sec. 5): xi ~ U(-4, 4), lam_jkl = exp(-pi (j + k + l) rho),
 *   phi_jkl = cos(j pi y) cos(k pi z) cos(l pi x), draw t = ((j-1)K + (k-1))K + (l-1).
 * Both draw from Philox4x64-10 (key (seed, 0), counter (block, sample,
 * level, 0)), four 53-bit uniforms u = ((w >> 11) + 1/2) 2^-53 per block:
 * normals by Box-Muller on the pairs (u0, u1), (u2, u3); uniforms -4 + 8 u. */
#define MLSGD_LAW_ALGEBRAIC 0
#define MLSGD_LAW_EXPONENTIAL 1

typedef struct mlsgd_solve_stats {
  int32_t iterations;      /* outer iterations of the slowest solve */
  int32_t nonconverged;    /* solves whose true residual exceeds rtol */
  double max_relres;       /* largest final true relative residual */
} mlsgd_solve_stats;

typedef struct mlsgd_grad_stats {
  double s;                /* max misfit over every solve of the estimate */
  double EY_shifted;       /* E^ML[Y] e^{-theta s} */
  double J;                /* MLMC entropic objective + alpha/2 |u|_h^2 */
  int32_t truncated;       /* 1 if E^ML[Y] < 1 (truncation max{1,.} fired) */
  int32_t iters_state;     /* slowest state solve */
  int32_t iters_adjoint;   /* slowest adjoint solve */
  int32_t nonconverged;
  double max_relres;
  /* per level, in units e^{theta s} (dY, dX) or e^{2 theta s} (m2) */
  double mean_dY[MLSGD_MAX_LEVELS];
  double norm2_mean_dX[MLSGD_MAX_LEVELS];  /* |E_i[dX]|_h^2 on grid i */
  double m2_dX[MLSGD_MAX_LEVELS];          /* sum_m |dX_m - E_i[dX]|_h^2 */
  double m2_dY[MLSGD_MAX_LEVELS];          /* sum_m (dY_m - E_i[dY])^2 */
  double mean_phi_f[MLSGD_MAX_LEVELS];     /* mean fine-grid misfit */
  double grad_norm;        /* |grad|_h */
  double norm2_EX;         /* |E^ML[X]|_h^2 in units e^{2 theta s} */
  double ms_solve;         /* device time of the solves, ms */
  double ms_total;         /* device time of the whole estimate, ms */
  /* per level: measured work per sample, interior unknowns x Krylov
   * iterations summed over the level's state and adjoint solves on the fine
   * and the coarse grid, divided by M; the adaptive controller's cost */
  double work_per_sample[MLSGD_MAX_LEVELS];
} mlsgd_grad_stats;

typedef struct mlsgd_step_stats {
  mlsgd_grad_stats grad;
  int64_t M_next[MLSGD_MAX_LEVELS];  /* sample counts for the next step */
  int64_t offset[MLSGD_MAX_LEVELS];  /* running per-level sample offsets after the step */
  double err_sam, err_num, eps;      /* adaptive-controller estimates (adapt != 0) */
  double tau;                        /* step size taken */
} mlsgd_step_stats;

typedef struct mlsgd_ctx mlsgd_ctx;

/* Create a context.  pb is copied; f and y_d are copied to library memory,
 * so the caller may free them afterwards.  stream: a hipStream_t (or 0 for
 * the null stream) on which all work of the context is enqueued.  Sec. 2 and
 * Sec. 5 define the problem data.  Errors: MLSGD_EINVAL for a malformed
 * problem (non-nested grids, K out of range, theta < 0, null y_d),
 * MLSGD_EOOM, MLSGD_EHIP. */
int mlsgd_create(mlsgd_ctx** out, const mlsgd_problem* pb, void* stream);

/* Free the context and the library memory it holds. */
int mlsgd_destroy(mlsgd_ctx* ctx);

/* Per-context message of the last failure ("" when none). */
const char* mlsgd_last_error(const mlsgd_ctx* ctx);

/* Draw xi for samples first .. first+count-1 of `level` (the random input of
 * one sample, Sec. 2.2 "draw xi^(m,l)"), in draw order under the context's
 * law (MLSGD_LAW_*): xi_out is device memory of count * K^3 doubles,
 * sample-major.  Errors: MLSGD_EINVAL for level out of
 * range, count < 0, first < 0 or a null xi_out with count > 0. */
int mlsgd_sample_fields(mlsgd_ctx* ctx, int level, int64_t first, int64_t count,
                        double* xi_out);

/* Raw Philox4x64-10 words of blocks 0..nblocks-1 for (seed, level, sample,
 * tag), written to out (device, 4*nblocks uint64).  Context-free; enqueued
 * on `stream`.  For bit-exact checks of the draw bookkeeping. */
int mlsgd_philox_words(uint64_t seed, int level, int64_t sample, int tag,
                       int nblocks, uint64_t* out, void* stream);

/* Batched state and adjoint solves for samples first .. first+count-1 of
 * `level` (Sec. 2.2 shorthand: X_l^(m), Y_l^(m) and their coarse partners):
 * coarse = 0 solves on grid n_level, coarse = 1 on grid n_{level-1} with the
 * level-`level` draw.  State: A y = R(f + u); misfit Phi = 1/2 |y - y_d|_h^2;
 * adjoint: A p = y - y_d.  u_fine: device, finest grid.  y_out, p_out:
 * device count*n^3 (nullable: not written; p_out = NULL also skips the
 * adjoint solves); phi_out: device count doubles (nullable).  st: host,
 * nullable.  Returns MLSGD_ENOCONV when a solve misses rtol. */
int mlsgd_solve_state_adjoint(mlsgd_ctx* ctx, int level, int coarse,
                              int64_t first, int64_t count,
                              const double* u_fine, double* y_out,
                              double* p_out, double* phi_out,
                              mlsgd_solve_stats* st);

/* Allocation-free form of mlsgd_solve_state_adjoint, for callers that
 * cannot allocate device memory during the call: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, semantics, outputs and errors as mlsgd_solve_state_adjoint,
 * and the same kernels; the solver rows, Krylov vectors, coefficient caches
 * and partial sums of the call live in a fixed device array of 64 MiB
 * (67108864 bytes) that the library holds on every GPU it runs on until the
 * process ends, instead of a per-batch-shape arena.  The call performs no
 * hipMalloc, hipFree or other device allocation (the context's own buffers
 * come from mlsgd_create).  It clears the part of the array it uses before
 * every call, so no call sees the previous call's contents.  All calls on one
 * GPU share the array: calls that overlap in time on one GPU (two contexts,
 * two streams, two threads) race and must be serialised by the caller.
 * scratch_bytes: host, nullable; receives the bytes the batch needs (also
 * when the call fails for size).  Errors: as mlsgd_solve_state_adjoint;
 * MLSGD_EINVAL also when the batch needs more than the 64 MiB array (about
 * 86 bytes per vertex of the solved grid in FP64: two 65^3 samples fit, three
 * do not, and no 129^3 sample does), when kernel timing is on, or when the
 * context's device is not current; such a call returns before any work is
 * enqueued. */
int mlsgd_solve_state_adjoint_noalloc(mlsgd_ctx* ctx, int level, int coarse,
                                      int64_t first, int64_t count,
                                      const double* u_fine, double* y_out,
                                      double* p_out, double* phi_out,
                                      mlsgd_solve_stats* st,
                                      int64_t* scratch_bytes);

/* Batched state solves of independent problems whose grids differ in size
 * (a batch of single-sample solves of the state equation, Sec. 2.1, on
 * grids of caller-chosen size, beside the MLMC levels).
 * Problem j uses grid n_list[j] (host array), the KL draw of sample first + j
 * of `level` (any level index >= 0; it only keys the draw), the right-hand
 * side f_value on the interior and the context's solver, precision, rtol
 * and max_iters.  Each n must be odd, 5 <= n <= 1025, and coarsen by halving
 * the cells to at most 9 vertices per axis (n - 1 = 2^a b with odd b <= 8);
 * a coarsest grid above 3^3 is solved with the dense inverse of its
 * operator.  y_out: device, nullable; problem j's n_j^3 solution (boundary
 * 0) starts at offset sum_{i<j} n_i^3.  st: host, nullable (largest
 * iteration count, count of misses, largest true relative residual).
 * Errors: MLSGD_EINVAL for count < 1, a null n_list, first < 0, level < 0 or
 * a grid outside the rule; MLSGD_ENOCONV when a solve misses rtol (y_out is
 * still written). */
int mlsgd_solve_sizes(mlsgd_ctx* ctx, int count, const int* n_list, int level, int64_t first,
                      double f_value, double* y_out, mlsgd_solve_stats* st);

/* The exact coarsest-grid solve of mlsgd_solve_sizes' hierarchies that stop
 * above 3^3, exposed for checking: the inverse of the rediscretised operator
 * (the Sec. 5 model problem's finite-difference form, see the top of this
 * header) on an n^3 grid (4 <= n <= 9, N = (n-2)^3 interior unknowns) for the
 * KL draws of samples first .. first+count-1 of `level`, computed as on the
 * solve path: a blocked Cholesky factorisation on the FP64 matrix cores,
 * then L^-1 and A^-1 = L^-T L^-1.  out: device, count * N * N doubles,
 * problem-major, row-major over the interior unknowns in the vertex order
 * (x slowest, z fastest).  Allocates and frees its own work buffers.
 * Errors: MLSGD_EINVAL for n outside 4..9, count outside 1..4096, a negative
 * level or first, or a null out. */
int mlsgd_dense_coarse_inverse(mlsgd_ctx* ctx, int n, int level, int64_t first, int count,
                               double* out);

/* One MLMC gradient estimate (Sec. 2.2, the estimator with truncated
 * denominator; Algorithm 1, GradientEstimate):
 *   grad = E^ML[X] / max{1, E^ML[Y]} + alpha u   on the finest grid,
 *   E^ML[X] = sum_i P^(i -> finest) (1/M_i) sum_m (w_f p_f - w_c P p_c),
 *   E^ML[Y] = sum_i (1/M_i) sum_m (w_f - w_c), w = e^{theta Phi}.
 * Levels 0..L-1 (L <= n_levels); level 0 has no coarse part.  M: host, L
 * sample counts >= 1; first: host, L per-level sample offsets (nullable =
 * 0); grad_out: device, finest grid; st: host, nullable. */
int mlsgd_mlmc_gradient(mlsgd_ctx* ctx, const double* u_fine, int L,
                        const int64_t* M, const int64_t* first,
                        double* grad_out, mlsgd_grad_stats* st);

/* The MLMC entropic objective J = theta^-1 log max{1, E^ML[Y]} + alpha/2
 * |u|_h^2 (theta = 0: MLMC mean of Phi), state solves only (Sec. 2.1 entropic
 * risk, Sec. 2.2 estimator).  J_out: host double. */
int mlsgd_mlmc_objective(mlsgd_ctx* ctx, const double* u_fine, int L,
                         const int64_t* M, const int64_t* first,
                         double* J_out, mlsgd_grad_stats* st);

/* Set the level count and per-level sample counts used by mlsgd_step and
 * reset the running per-level sample offsets to `offsets` (host, nullable =
 * 0).  M: host, L counts >= 1 (>= 2 when the adaptive controller runs). */
int mlsgd_set_batch(mlsgd_ctx* ctx, int L, const int64_t* M,
                    const int64_t* offsets);

/* One projected SGD step u <- Pi(u - tau_k grad) (Sec. 2.2, Algorithm 1,
 * MLSGD) with fresh samples: the gradient uses the current batch and running
 * offsets, which then advance by M.  adapt is a set of flags:
 * MLSGD_ADAPT_BATCH runs the adaptive controller (Sec. 4.1: power sums,
 * optimal batch size with the estimate's measured work per sample as the
 * cost of a level, bias estimate, level growth) to choose the next batch;
 * MLSGD_ADAPT_STEP takes the adaptive step size of Sec. 5
 * (eq. adaptive-step-size: tau_k = (|g_k|^2 - err_sam) / (Lhat |g_k|^2),
 * Lhat = |g_k - g_{k-1}| / (tau_{k-1} |g_{k-1}|), clamped at 0), with tau as
 * the step of the first step after mlsgd_set_batch and as the fallback when
 * Lhat is undefined.  Without MLSGD_ADAPT_STEP tau is the step.  Either flag
 * needs M >= 2 on every level.  u_inout: device, finest grid.  st: host,
 * nullable (st->tau: the step taken). */
#define MLSGD_ADAPT_BATCH 1
#define MLSGD_ADAPT_STEP 2
int mlsgd_step(mlsgd_ctx* ctx, double* u_inout, double tau, int adapt,
               mlsgd_step_stats* st);

/* Solver tuning of a context (smoother, cycle and tile parameters).  The
 * defaults come from measurement on MI355X; mlsgd_set_tuning replaces them,
 * e.g. with the choice of the package's autotuner, and drops the cached
 * layouts (the next call rebuilds them).  Any tuning reaches the same
 * estimate to solver tolerance; only the speed differs. */
#define MLSGD_SMOOTHER_RBGS 0       /* red-black Gauss-Seidel, two passes per sweep */
#define MLSGD_SMOOTHER_RBGS_FUSED 1 /* red-black Gauss-Seidel, one fused pass per sweep */
#define MLSGD_SMOOTHER_CHEBYSHEV 2  /* Chebyshev steps of D^-1 A on [2 cheb_lo, 2] */

typedef struct mlsgd_tuning {
  int32_t smoother;   /* MLSGD_SMOOTHER_* */
  int32_t sweeps;     /* smoothing sweeps (Chebyshev degree) before and after the coarse correction */
  double omega;       /* red-black relaxation weight, (0, 2) */
  double cheb_lo;     /* lower end of the Chebyshev interval as a fraction of 2, (0, 1) */
  int32_t tile_y;     /* y extent of the stencil tiles on grids with > 32 interior points: 4, 8, 16 */
  int32_t xchunk;     /* x planes marched by one workgroup, 8..1024 */
  int32_t cache;      /* 1: coefficient regenerated once per call into a cache; 0: in every sweep */
} mlsgd_tuning;

int mlsgd_get_tuning(const mlsgd_ctx* ctx, mlsgd_tuning* out);
int mlsgd_set_tuning(mlsgd_ctx* ctx, const mlsgd_tuning* tuning);

/* Graph mode (enable = 1): mlsgd_mlmc_gradient, mlsgd_mlmc_objective and
 * mlsgd_step run each batch shape (L, M, gradient or objective) as one
 * replayed HIP graph instead of a host-driven sequence of launches.  The
 * first call of a shape runs as usual and records the iteration counts of
 * its solves; the shape is then captured once with those counts plus a
 * margin (converged problems idle through the extra iterations), followed by
 * the true-residual check and one short restart block.  Later calls upload
 * their draws and u, replay the graph and copy the gradient out; a replay
 * whose solves miss rtol is recomputed by the host-driven path and the shape
 * is captured again with a larger margin, so results always meet rtol.  The
 * graph runs on the context's stream; capture uses a stream of its own.
 * enable = 0 drops the captured graphs.  Not used while mlsgd_kernel_timing
 * is on.  Errors: MLSGD_EINVAL for enable outside {0, 1}. */
int mlsgd_set_graph(mlsgd_ctx* ctx, int enable);

/* Event timing of a kernel of the solves on grid size n (their dominant
 * kernels), for roofline figures.  Each launch of the selected kernel on that
 * grid is bracketed by HIP events on the context's stream: the plain
 * smoothing step (enable = 1), the fused two-step post-smoothing pass
 * (enable = 2), the fused pre-smoothing pass with its residual (enable = 3)
 * or the Krylov matvec (enable = 4); the fused passes run on grids with
 * 64-wide tiles of height 8 or 16 and a cached coefficient.  The call
 * first returns the totals accumulated so far (host outputs, nullable:
 * summed milliseconds, launch count, algorithmic bytes = interior points x
 * bytes the kernel must move, the coefficient counted at 0 bytes since the
 * method regenerates it from the draws; a kernel that reads a per-call
 * coefficient cache moves that cache on top), then, if enable >= 0, resets
 * them and switches timing on
 * (enable = 1, 2, 3 or 4, for grid n) or off (enable = 0); enable < 0
 * only reads.  Errors: MLSGD_EINVAL for enable > 4. */
int mlsgd_kernel_timing(mlsgd_ctx* ctx, int enable, int n, double* ms_total,
                        int64_t* launches, double* bytes);

#ifdef __cplusplus
}
#endif
#endif
