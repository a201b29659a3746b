/*
 * mlsgd_oracle.h -- plain, slow, FP64 CPU oracle for the MLMC entropic-risk
 * gradient of "Multilevel Stochastic Gradient Descent for Risk-Averse
 * PDE-Constrained Optimization" (Baumgarten, Guth, Schneiderhan, Vanzan).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library
 * and its Python binding) includes, links or calls this code.  It shares no
 * code, header, table or constant generator with the HIP path.
 *
 * Conventions (the readings of the paper this oracle takes):
 *   - grid: n vertices per axis on the unit cube, h = 1/(n-1); arrays hold all
 *     n^3 vertices, index v = (ix*n + iy)*n + iz (z fastest); the Dirichlet
 *     boundary is held at 0 and boundary entries of inputs are ignored.
 *   - operator (Sec. 5 model problem, finite-difference reading):
 *       (A y)_v = h^-2 * sum_{faces f=(v,w)} a_f (y_v - y_w),
 *       a_f = 2 a_v a_w / (a_v + a_w),  a = exp(log a) at vertices.
 *   - coefficient: log a(x) = sum_{k in {1..K}^3} c_k prod_d cos(pi k_d x_d),
 *       c_k = sigma * sqrt(lam_k) * xi_k,  lam_k = (1+|k|^2)^(-5/2),
 *       term index j = ((k1-1)K + (k2-1))K + (k3-1), k1 <-> x, k3 <-> z.
 *   - xi_j ~ N(0,1) from Philox4x64-10 (Salmon et al., SC'11), key
 *       (seed, 0), counter (block, sample, level, tag); each block's four
 *       words w give u = ((w >> 11) + 0.5) 2^-53 and two Box-Muller pairs.
 *   - control transfer: full weighting R = P^T / 8 between nested grids,
 *       adjoint transfer: trilinear prolongation P.
 */
#ifndef MLSGD_ORACLE_H
#define MLSGD_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OR_MAX_LEVELS 8

/* solver methods */
#define OR_SOLVE_AUTO 0   /* dense Cholesky for n <= 9, MG-PCG otherwise */
#define OR_SOLVE_CG 1
#define OR_SOLVE_MGPCG 2
#define OR_SOLVE_DENSE 3

typedef struct or_problem {
  int L;                    /* number of levels */
  int n[OR_MAX_LEVELS];     /* vertices per axis, nested: n[i] = 2 n[i-1] - 1 */
  uint64_t seed;
  int K;                    /* KL terms per axis */
  double sigma2;            /* KL variance scale */
  double theta;             /* entropic risk parameter, >= 0 */
  double alpha;             /* Tikhonov weight (the paper's lambda) */
  int method;               /* OR_SOLVE_* */
  double rtol;              /* true relative residual target */
  int maxit;
  int nthreads;             /* OpenMP threads for the (level, sample) loop */
  int common_xi;            /* test switch: key every level's draws as level 0 */
  int law;                  /* OR_LAW_*: law of the KL draws */
  double rho;               /* correlation length of OR_LAW_EXPONENTIAL */
} or_problem;

/* KL laws.  ALGEBRAIC: xi ~ N(0,1), lam = (1 + |k|^2)^(-5/2), phi_k =
 * cos(k1 pi x) cos(k2 pi y) cos(k3 pi z).  EXPONENTIAL (Sec. 5): xi ~
 * U(-4,4), lam_jkl = exp(-pi (j+k+l) rho), phi_jkl = cos(j pi y) cos(k pi z)
 * cos(l pi x).  Coefficients are returned at the index of the product
 * cos(k1 pi x) cos(k2 pi y) cos(k3 pi z), ((k1-1) K + (k2-1)) K + (k3-1). */
#define OR_LAW_ALGEBRAIC 0
#define OR_LAW_EXPONENTIAL 1

typedef struct or_stats {
  double s;                          /* max Phi over the estimate (shift) */
  double EY_shifted;                 /* sum_i mean dY_i in units e^{theta s} */
  double J;                          /* MLMC entropic objective + alpha/2 |u|^2 */
  int truncated;                     /* 1 if E^ML[Y] < 1 (truncation fired) */
  double max_relres;                 /* worst true relative residual */
  int max_iters;                     /* worst iteration count */
  /* per level, shifted units (multiply by e^{theta s} / e^{2 theta s}) */
  double mean_dY[OR_MAX_LEVELS];
  double norm2_mean_dX[OR_MAX_LEVELS]; /* || E_i[dX] ||^2_h on grid i */
  double m2_dX[OR_MAX_LEVELS];         /* sum_m || dX_m - E_i[dX] ||^2_h */
  double m2_dY[OR_MAX_LEVELS];         /* sum_m | dY_m - E_i[dY] |^2 */
  double mean_phi_f[OR_MAX_LEVELS];    /* mean misfit on the fine grid */
  double norm2_EX;                     /* |E^ML[X]|_h^2, shifted units */
} or_stats;

void or_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
void or_philox_words(uint64_t seed, int level, int64_t sample, int tag,
                     int nblocks, uint64_t* out);
void or_normals(uint64_t seed, int level, int64_t sample, int tag, int count,
                double* out);
void or_kl_coeffs(uint64_t seed, int level, int64_t sample, int K,
                  double sigma2, double* c);
void or_draws(uint64_t seed, int level, int64_t sample, int K, int law, double* xi);
void or_kl_coeffs_law(uint64_t seed, int level, int64_t sample, int K, double sigma2,
                      int law, double rho, double* c);
void or_log_coeff(int n, int K, const double* c, double* loga);
void or_apply(int n, int K, const double* c, const double* y, double* out);
void or_assemble_dense(int n, int K, const double* c, double* Adense);
int or_solve(int n, int K, const double* c, const double* b, double* x,
             int method, double rtol, int maxit, double* relres_out);
void or_restrict(int nf, const double* fine, double* coarse);
void or_prolong(int nc, const double* coarse, double* fine);
double or_misfit(int n, const double* y, const double* yd);
int or_mlmc_gradient(const or_problem* pb, const double* f, const double* u,
                     const double* yd, const int64_t* M, const int64_t* first,
                     double* grad, or_stats* st);
int or_mlmc_objective(const or_problem* pb, const double* f, const double* u,
                      const double* yd, const int64_t* M, const int64_t* first,
                      double* J_out, or_stats* st);

#ifdef __cplusplus
}
#endif
#endif
