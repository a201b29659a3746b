/*
 * mlsgd_oracle.c -- plain, slow, obviously correct FP64 CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY: used by tests/, the package's smoke check and
 * the CPU-baseline leg of the benchmark.  It shares no code with the HIP
 * path.  Everything is FP64; loops are written in the order the definitions
 * are stated, with no blocking or fusion.
 *
 * Paper: Baumgarten, Guth, Schneiderhan, Vanzan, "Multilevel Stochastic
 * Gradient Descent for Risk-Averse PDE-Constrained Optimization".
 *   Sec. 2       problem (cost J = R(Phi(y)) + lambda/2 |u|^2, state eq.)
 *   Sec. 2.1     entropic risk R_theta and the exact gradient E[X]/E[Y] + lambda u
 *   Sec. 2.2     MLMC gradient estimator, X_l, Y_l, shared xi^(m,l) on the
 *                fine and coarse grid of level l, dX, dY, X_0 = Y_0 = 0,
 *                truncation max{1, E^ML[Y]}, projected step
 *   Sec. 4.1     second-order power sums (level statistics)
 *   Sec. 5       model problem: (0,1)^3, U = H = L^2, exp(KL) coefficient
 * Readings where the paper is silent are listed in mlsgd_oracle.h.
 */
#include "mlsgd_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PI 3.14159265358979323846

/* ------------------------------------------------------------------ */
/* Philox4x64-10, as published by Salmon, Moraes, Dror and Shaw,       */
/* "Parallel random numbers: as easy as 1, 2, 3" (SC'11): ten rounds   */
/* of two 64x64->128 multiplications, key bumped by the Weyl constants */
/* between rounds.                                                     */
/* ------------------------------------------------------------------ */
void or_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
  uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += W0;
      k1 += W1;
    }
    unsigned __int128 p0 = (unsigned __int128)M0 * x0;
    unsigned __int128 p1 = (unsigned __int128)M1 * x2;
    uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
    uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    uint64_t y0 = hi1 ^ x1 ^ k0;
    uint64_t y1 = lo1;
    uint64_t y2 = hi0 ^ x3 ^ k1;
    uint64_t y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Raw words of blocks 0..nblocks-1 for the draw keyed by (seed, level,
 * sample, tag): key = (seed, 0), counter = (block, sample, level, tag).
 * Every sample of every level owns its own counter range (Sec. 2.2: the
 * xi^(m,l) are independent across m and l). */
void or_philox_words(uint64_t seed, int level, int64_t sample, int tag,
                     int nblocks, uint64_t* out) {
  uint64_t key[2] = {seed, 0};
  for (int b = 0; b < nblocks; ++b) {
    uint64_t ctr[4] = {(uint64_t)b, (uint64_t)sample, (uint64_t)level, (uint64_t)tag};
    or_philox4x64_10(ctr, key, out + 4 * b);
  }
}

/* Standard normals by Box-Muller on pairs (w0,w1), (w2,w3) of each block. */
void or_normals(uint64_t seed, int level, int64_t sample, int tag, int count,
                double* out) {
  int nblocks = (count + 3) / 4;
  uint64_t w[4];
  for (int b = 0; b < nblocks; ++b) {
    uint64_t key[2] = {seed, 0};
    uint64_t ctr[4] = {(uint64_t)b, (uint64_t)sample, (uint64_t)level, (uint64_t)tag};
    or_philox4x64_10(ctr, key, w);
    double u[4];
    for (int q = 0; q < 4; ++q) u[q] = ((double)(w[q] >> 11) + 0.5) * 0x1.0p-53;
    double z[4];
    for (int pr = 0; pr < 2; ++pr) {
      double r = sqrt(-2.0 * log(u[2 * pr]));
      double t = 2.0 * OR_PI * u[2 * pr + 1];
      z[2 * pr] = r * cos(t);
      z[2 * pr + 1] = r * sin(t);
    }
    for (int q = 0; q < 4; ++q)
      if (4 * b + q < count) out[4 * b + q] = z[q];
  }
}

/* The K^3 draws of one sample in draw order: normals for the algebraic law,
 * xi = -4 + 8 u on the 53-bit uniforms u of the same Philox words for the
 * exponential law (Sec. 5: xi_jkl ~ U(-4, 4)). */
void or_draws(uint64_t seed, int level, int64_t sample, int K, int law, double* xi) {
  int nt = K * K * K;
  if (law == OR_LAW_ALGEBRAIC) {
    or_normals(seed, level, sample, 0, nt, xi);
    return;
  }
  int nblocks = (nt + 3) / 4;
  for (int b = 0; b < nblocks; ++b) {
    uint64_t key[2] = {seed, 0};
    uint64_t ctr[4] = {(uint64_t)b, (uint64_t)sample, (uint64_t)level, 0};
    uint64_t w[4];
    or_philox4x64_10(ctr, key, w);
    for (int q = 0; q < 4; ++q) {
      double u = ((double)(w[q] >> 11) + 0.5) * 0x1.0p-53;
      if (4 * b + q < nt) xi[4 * b + q] = -4.0 + 8.0 * u;
    }
  }
}

/* KL coefficients under either law (Sec. 5 for the exponential one: the
 * term (j, k, l) multiplies cos(j pi x_2) cos(k pi x_3) cos(l pi x_1), so in
 * the x-major product index it sits at (k1, k2, k3) = (l, j, k)). */
void or_kl_coeffs_law(uint64_t seed, int level, int64_t sample, int K, double sigma2,
                      int law, double rho, double* c) {
  if (law == OR_LAW_ALGEBRAIC) {
    or_kl_coeffs(seed, level, sample, K, sigma2, c);
    return;
  }
  int nt = K * K * K;
  double* xi = (double*)malloc(sizeof(double) * (size_t)nt);
  or_draws(seed, level, sample, K, law, xi);
  double sigma = sqrt(sigma2);
  for (int j = 1; j <= K; ++j)
    for (int k = 1; k <= K; ++k)
      for (int l = 1; l <= K; ++l) {
        int t = ((j - 1) * K + (k - 1)) * K + (l - 1);
        int e = ((l - 1) * K + (j - 1)) * K + (k - 1);
        double lam = exp(-OR_PI * (double)(j + k + l) * rho);
        c[e] = sigma * sqrt(lam) * xi[t];
      }
  free(xi);
}

/* KL coefficients c_j = sigma sqrt(lam_k) xi_j, lam_k = (1 + |k|^2)^(-5/2),
 * for the coefficient law of the experiments (Sec. 5, with the decay and
 * normal law of the synthetic workloads). */
void or_kl_coeffs(uint64_t seed, int level, int64_t sample, int K,
                  double sigma2, double* c) {
  int nt = K * K * K;
  double* xi = (double*)malloc(sizeof(double) * (size_t)nt);
  or_normals(seed, level, sample, 0, nt, xi);
  double sigma = sqrt(sigma2);
  for (int k1 = 1; k1 <= K; ++k1)
    for (int k2 = 1; k2 <= K; ++k2)
      for (int k3 = 1; k3 <= K; ++k3) {
        int j = ((k1 - 1) * K + (k2 - 1)) * K + (k3 - 1);
        double kk = (double)(k1 * k1 + k2 * k2 + k3 * k3);
        double lam = pow(1.0 + kk, -2.5);
        c[j] = sigma * sqrt(lam) * xi[j];
      }
  free(xi);
}

/* log a at every vertex: the KL sum written out term by term. */
void or_log_coeff(int n, int K, const double* c, double* loga) {
  double h = 1.0 / (double)(n - 1);
  double* cs = (double*)malloc(sizeof(double) * (size_t)(K * n));
  for (int k = 1; k <= K; ++k)
    for (int i = 0; i < n; ++i) cs[(k - 1) * n + i] = cos(OR_PI * k * (i * h));
  for (int ix = 0; ix < n; ++ix)
    for (int iy = 0; iy < n; ++iy)
      for (int iz = 0; iz < n; ++iz) {
        double s = 0.0;
        for (int k1 = 1; k1 <= K; ++k1)
          for (int k2 = 1; k2 <= K; ++k2)
            for (int k3 = 1; k3 <= K; ++k3) {
              int j = ((k1 - 1) * K + (k2 - 1)) * K + (k3 - 1);
              s += c[j] * cs[(k1 - 1) * n + ix] * cs[(k2 - 1) * n + iy] *
                   cs[(k3 - 1) * n + iz];
            }
        loga[((size_t)ix * n + iy) * n + iz] = s;
      }
  free(cs);
}

static double* vertex_coeff(int n, int K, const double* c) {
  size_t N = (size_t)n * n * n;
  double* a = (double*)malloc(sizeof(double) * N);
  or_log_coeff(n, K, c, a);
  for (size_t v = 0; v < N; ++v) a[v] = exp(a[v]);
  return a;
}

static int is_interior(int n, int ix, int iy, int iz) {
  return ix > 0 && iy > 0 && iz > 0 && ix < n - 1 && iy < n - 1 && iz < n - 1;
}

static double face(double av, double aw) { return 2.0 * av * aw / (av + aw); }

/* (A y)_v for interior v with vertex coefficients a; y outside the interior
 * counts as 0 (Dirichlet); out is 0 on the boundary. */
static void op_apply(int n, const double* a, const double* y, double* out) {
  double ih2 = (double)(n - 1) * (double)(n - 1);
  static const int off[6][3] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0},
                                {0, 1, 0},  {0, 0, -1}, {0, 0, 1}};
  for (int ix = 0; ix < n; ++ix)
    for (int iy = 0; iy < n; ++iy)
      for (int iz = 0; iz < n; ++iz) {
        size_t v = ((size_t)ix * n + iy) * n + iz;
        if (!is_interior(n, ix, iy, iz)) {
          out[v] = 0.0;
          continue;
        }
        double s = 0.0;
        for (int f = 0; f < 6; ++f) {
          int jx = ix + off[f][0], jy = iy + off[f][1], jz = iz + off[f][2];
          size_t w = ((size_t)jx * n + jy) * n + jz;
          double yw = is_interior(n, jx, jy, jz) ? y[w] : 0.0;
          s += face(a[v], a[w]) * (y[v] - yw);
        }
        out[v] = ih2 * s;
      }
}

void or_apply(int n, int K, const double* c, const double* y, double* out) {
  double* a = vertex_coeff(n, K, c);
  op_apply(n, a, y, out);
  free(a);
}

static size_t interior_index(int n, int ix, int iy, int iz) {
  int m = n - 2;
  return ((size_t)(ix - 1) * m + (iy - 1)) * m + (iz - 1);
}

static void assemble_from_a(int n, const double* a, double* A) {
  int m = n - 2;
  size_t N = (size_t)m * m * m;
  double ih2 = (double)(n - 1) * (double)(n - 1);
  static const int off[6][3] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0},
                                {0, 1, 0},  {0, 0, -1}, {0, 0, 1}};
  memset(A, 0, sizeof(double) * N * N);
  for (int ix = 1; ix < n - 1; ++ix)
    for (int iy = 1; iy < n - 1; ++iy)
      for (int iz = 1; iz < n - 1; ++iz) {
        size_t v = ((size_t)ix * n + iy) * n + iz;
        size_t r = interior_index(n, ix, iy, iz);
        for (int f = 0; f < 6; ++f) {
          int jx = ix + off[f][0], jy = iy + off[f][1], jz = iz + off[f][2];
          size_t w = ((size_t)jx * n + jy) * n + jz;
          double af = ih2 * face(a[v], a[w]);
          A[r * N + r] += af;
          if (is_interior(n, jx, jy, jz)) A[r * N + interior_index(n, jx, jy, jz)] -= af;
        }
      }
}

/* Dense matrix of A on the interior unknowns (row-major, (n-2)^3 squared). */
void or_assemble_dense(int n, int K, const double* c, double* A) {
  double* a = vertex_coeff(n, K, c);
  assemble_from_a(n, a, A);
  free(a);
}

/* ---------------------------- vectors ------------------------------ */
static double dot_int(int n, const double* x, const double* y) {
  double s = 0.0;
  for (int ix = 1; ix < n - 1; ++ix)
    for (int iy = 1; iy < n - 1; ++iy)
      for (int iz = 1; iz < n - 1; ++iz) {
        size_t v = ((size_t)ix * n + iy) * n + iz;
        s += x[v] * y[v];
      }
  return s;
}

static void mask_boundary(int n, double* x) {
  for (int ix = 0; ix < n; ++ix)
    for (int iy = 0; iy < n; ++iy)
      for (int iz = 0; iz < n; ++iz)
        if (!is_interior(n, ix, iy, iz)) x[((size_t)ix * n + iy) * n + iz] = 0.0;
}

/* ------------------------- grid transfers -------------------------- */
/* Full weighting: coarse interior j gets sum over d in {-1,0,1}^3 of
 * prod_axis w(d) * fine[2j+d], with w(0) = 1/2, w(+-1) = 1/4; this equals
 * P^T / 8 on interior vectors. */
void or_restrict(int nf, const double* fine, double* coarse) {
  int nc = (nf - 1) / 2 + 1;
  double w[3] = {0.25, 0.5, 0.25};
  for (int jx = 0; jx < nc; ++jx)
    for (int jy = 0; jy < nc; ++jy)
      for (int jz = 0; jz < nc; ++jz) {
        size_t vc = ((size_t)jx * nc + jy) * nc + jz;
        if (!is_interior(nc, jx, jy, jz)) {
          coarse[vc] = 0.0;
          continue;
        }
        double s = 0.0;
        for (int dx = -1; dx <= 1; ++dx)
          for (int dy = -1; dy <= 1; ++dy)
            for (int dz = -1; dz <= 1; ++dz) {
              int ix = 2 * jx + dx, iy = 2 * jy + dy, iz = 2 * jz + dz;
              double fv = is_interior(nf, ix, iy, iz) ? fine[((size_t)ix * nf + iy) * nf + iz] : 0.0;
              s += w[dx + 1] * w[dy + 1] * w[dz + 1] * fv;
            }
        coarse[vc] = s;
      }
}

/* Trilinear prolongation from the coarse grid (boundary 0) to the fine grid. */
void or_prolong(int nc, const double* coarse, double* fine) {
  int nf = 2 * (nc - 1) + 1;
  for (int ix = 0; ix < nf; ++ix)
    for (int iy = 0; iy < nf; ++iy)
      for (int iz = 0; iz < nf; ++iz) {
        size_t vf = ((size_t)ix * nf + iy) * nf + iz;
        if (!is_interior(nf, ix, iy, iz)) {
          fine[vf] = 0.0;
          continue;
        }
        int i[3] = {ix, iy, iz};
        int lo[3], hi[3];
        double wl[3], wh[3];
        for (int d = 0; d < 3; ++d) {
          if (i[d] % 2 == 0) {
            lo[d] = hi[d] = i[d] / 2;
            wl[d] = 1.0;
            wh[d] = 0.0;
          } else {
            lo[d] = (i[d] - 1) / 2;
            hi[d] = (i[d] + 1) / 2;
            wl[d] = 0.5;
            wh[d] = 0.5;
          }
        }
        double s = 0.0;
        for (int a = 0; a < 2; ++a)
          for (int b = 0; b < 2; ++b)
            for (int cc = 0; cc < 2; ++cc) {
              int jx = a ? hi[0] : lo[0], jy = b ? hi[1] : lo[1], jz = cc ? hi[2] : lo[2];
              double wt = (a ? wh[0] : wl[0]) * (b ? wh[1] : wl[1]) * (cc ? wh[2] : wl[2]);
              if (wt == 0.0) continue;
              double cv = is_interior(nc, jx, jy, jz) ? coarse[((size_t)jx * nc + jy) * nc + jz] : 0.0;
              s += wt * cv;
            }
        fine[vf] = s;
      }
}

/* ----------------------------- solvers ----------------------------- */
/* In-place Cholesky A = L L^T of a dense SPD matrix (lower triangle). */
static int cholesky(size_t N, double* A) {
  for (size_t j = 0; j < N; ++j) {
    double d = A[j * N + j];
    for (size_t k = 0; k < j; ++k) d -= A[j * N + k] * A[j * N + k];
    if (!(d > 0.0)) return -1;
    d = sqrt(d);
    A[j * N + j] = d;
    for (size_t i = j + 1; i < N; ++i) {
      double s = A[i * N + j];
      for (size_t k = 0; k < j; ++k) s -= A[i * N + k] * A[j * N + k];
      A[i * N + j] = s / d;
    }
  }
  return 0;
}

static void cholesky_solve(size_t N, const double* Lf, const double* b, double* x) {
  for (size_t i = 0; i < N; ++i) {
    double s = b[i];
    for (size_t k = 0; k < i; ++k) s -= Lf[i * N + k] * x[k];
    x[i] = s / Lf[i * N + i];
  }
  for (size_t ii = N; ii-- > 0;) {
    double s = x[ii];
    for (size_t k = ii + 1; k < N; ++k) s -= Lf[k * N + ii] * x[k];
    x[ii] = s / Lf[ii * N + ii];
  }
}

/* Geometric hierarchy for the oracle's own MG-PCG: vertex coefficients are
 * evaluated on every grid (rediscretisation), smoothing is symmetric
 * lexicographic Gauss-Seidel, transfers are full weighting / trilinear and the
 * coarsest grid is solved by dense Cholesky. */
typedef struct {
  int nlev;
  int n[16];
  double* a[16];
  double* x[16];
  double* b[16];
  double* r[16];
  double* Lc;   /* Cholesky factor on the coarsest grid */
  size_t Nc;
} mg_t;

static void mg_build(mg_t* mg, int n, int K, const double* c) {
  memset(mg, 0, sizeof(*mg));
  int lev = 0;
  int m = n;
  for (;;) {
    mg->n[lev] = m;
    size_t N = (size_t)m * m * m;
    mg->a[lev] = vertex_coeff(m, K, c);
    mg->x[lev] = (double*)calloc(N, sizeof(double));
    mg->b[lev] = (double*)calloc(N, sizeof(double));
    mg->r[lev] = (double*)calloc(N, sizeof(double));
    ++lev;
    if (m <= 3 || (m - 1) % 2 != 0) break;
    m = (m - 1) / 2 + 1;
  }
  mg->nlev = lev;
  int nc = mg->n[lev - 1];
  size_t Nc = (size_t)(nc - 2) * (nc - 2) * (nc - 2);
  mg->Nc = Nc;
  mg->Lc = (double*)malloc(sizeof(double) * Nc * Nc);
  assemble_from_a(nc, mg->a[lev - 1], mg->Lc);
  cholesky(Nc, mg->Lc);
}

static void mg_free(mg_t* mg) {
  for (int l = 0; l < mg->nlev; ++l) {
    free(mg->a[l]);
    free(mg->x[l]);
    free(mg->b[l]);
    free(mg->r[l]);
  }
  free(mg->Lc);
}

static void gauss_seidel(int n, const double* a, const double* b, double* x, int forward) {
  double ih2 = (double)(n - 1) * (double)(n - 1);
  static const int off[6][3] = {{-1, 0, 0}, {1, 0, 0}, {0, -1, 0},
                                {0, 1, 0},  {0, 0, -1}, {0, 0, 1}};
  int m = n - 2;
  for (int t = 0; t < m * m * m; ++t) {
    int u = forward ? t : m * m * m - 1 - t;
    int ix = 1 + u / (m * m), iy = 1 + (u / m) % m, iz = 1 + u % m;
    size_t v = ((size_t)ix * n + iy) * n + iz;
    double diag = 0.0, s = b[v];
    for (int f = 0; f < 6; ++f) {
      int jx = ix + off[f][0], jy = iy + off[f][1], jz = iz + off[f][2];
      size_t w = ((size_t)jx * n + jy) * n + jz;
      double af = ih2 * face(a[v], a[w]);
      diag += af;
      if (is_interior(n, jx, jy, jz)) s += af * x[w];
    }
    x[v] = s / diag;
  }
}

static void coarse_solve(mg_t* mg, int l) {
  int n = mg->n[l];
  size_t Nc = mg->Nc;
  double* bb = (double*)calloc(Nc, sizeof(double));
  double* xx = (double*)malloc(sizeof(double) * Nc);
  for (int ix = 1; ix < n - 1; ++ix)
    for (int iy = 1; iy < n - 1; ++iy)
      for (int iz = 1; iz < n - 1; ++iz)
        bb[interior_index(n, ix, iy, iz)] = mg->b[l][((size_t)ix * n + iy) * n + iz];
  cholesky_solve(Nc, mg->Lc, bb, xx);
  memset(mg->x[l], 0, sizeof(double) * (size_t)n * n * n);
  for (int ix = 1; ix < n - 1; ++ix)
    for (int iy = 1; iy < n - 1; ++iy)
      for (int iz = 1; iz < n - 1; ++iz)
        mg->x[l][((size_t)ix * n + iy) * n + iz] = xx[interior_index(n, ix, iy, iz)];
  free(bb);
  free(xx);
}

/* One symmetric V(1,1) cycle on level l: x[l] <- V(b[l]) from a zero guess. */
static void vcycle(mg_t* mg, int l) {
  int n = mg->n[l];
  size_t N = (size_t)n * n * n;
  if (l == mg->nlev - 1) {
    coarse_solve(mg, l);
    return;
  }
  memset(mg->x[l], 0, sizeof(double) * N);
  gauss_seidel(n, mg->a[l], mg->b[l], mg->x[l], 1);
  op_apply(n, mg->a[l], mg->x[l], mg->r[l]);
  for (size_t v = 0; v < N; ++v) mg->r[l][v] = mg->b[l][v] - mg->r[l][v];
  mask_boundary(n, mg->r[l]);
  or_restrict(n, mg->r[l], mg->b[l + 1]);
  vcycle(mg, l + 1);
  or_prolong(mg->n[l + 1], mg->x[l + 1], mg->r[l]);
  for (size_t v = 0; v < N; ++v) mg->x[l][v] += mg->r[l][v];
  gauss_seidel(n, mg->a[l], mg->b[l], mg->x[l], 0);
}

static double true_relres(int n, const double* a, const double* b, const double* x,
                          double* tmp) {
  op_apply(n, a, x, tmp);
  size_t N = (size_t)n * n * n;
  double rr = 0.0;
  for (int ix = 1; ix < n - 1; ++ix)
    for (int iy = 1; iy < n - 1; ++iy)
      for (int iz = 1; iz < n - 1; ++iz) {
        size_t v = ((size_t)ix * n + iy) * n + iz;
        double d = b[v] - tmp[v];
        rr += d * d;
      }
  (void)N;
  double bb = dot_int(n, b, b);
  if (bb == 0.0) return sqrt(rr);
  return sqrt(rr / bb);
}

/* (Preconditioned) conjugate gradients from x = 0 (or the current x on a
 * restart) until the true relative residual is <= rtol; restarts from the
 * true residual up to three times when the recursive residual has drifted. */
static int pcg(int n, const double* a, mg_t* mg, const double* b, double* x,
               double rtol, int maxit, double* relres_out) {
  size_t N = (size_t)n * n * n;
  double* r = (double*)calloc(N, sizeof(double));
  double* z = (double*)calloc(N, sizeof(double));
  double* p = (double*)calloc(N, sizeof(double));
  double* q = (double*)calloc(N, sizeof(double));
  double bnorm = sqrt(dot_int(n, b, b));
  int it = 0;
  double rel = 0.0;
  memset(x, 0, sizeof(double) * N);
  if (bnorm == 0.0) {
    *relres_out = 0.0;
    free(r); free(z); free(p); free(q);
    return 0;
  }
  for (int restart = 0; restart < 4; ++restart) {
    op_apply(n, a, x, q);
    for (size_t v = 0; v < N; ++v) r[v] = b[v] - q[v];
    mask_boundary(n, r);
    if (mg) {
      memcpy(mg->b[0], r, sizeof(double) * N);
      vcycle(mg, 0);
      memcpy(z, mg->x[0], sizeof(double) * N);
    } else {
      memcpy(z, r, sizeof(double) * N);
    }
    memcpy(p, z, sizeof(double) * N);
    double rz = dot_int(n, r, z);
    while (it < maxit) {
      op_apply(n, a, p, q);
      double alpha = rz / dot_int(n, p, q);
      for (size_t v = 0; v < N; ++v) {
        x[v] += alpha * p[v];
        r[v] -= alpha * q[v];
      }
      ++it;
      if (sqrt(dot_int(n, r, r)) <= rtol * bnorm) break;
      if (mg) {
        memcpy(mg->b[0], r, sizeof(double) * N);
        vcycle(mg, 0);
        memcpy(z, mg->x[0], sizeof(double) * N);
      } else {
        memcpy(z, r, sizeof(double) * N);
      }
      double rz_new = dot_int(n, r, z);
      double beta = rz_new / rz;
      rz = rz_new;
      for (size_t v = 0; v < N; ++v) p[v] = z[v] + beta * p[v];
    }
    rel = true_relres(n, a, b, x, q);
    if (rel <= rtol || it >= maxit) break;
  }
  *relres_out = rel;
  free(r); free(z); free(p); free(q);
  return it;
}

static int solve_with_a(int n, int K, const double* c, const double* a,
                        const double* b, double* x, int method, double rtol,
                        int maxit, double* relres_out) {
  size_t N = (size_t)n * n * n;
  if (method == OR_SOLVE_AUTO) method = (n <= 9) ? OR_SOLVE_DENSE : OR_SOLVE_MGPCG;
  if (method == OR_SOLVE_DENSE) {
    int m = n - 2;
    size_t Ni = (size_t)m * m * m;
    double* A = (double*)malloc(sizeof(double) * Ni * Ni);
    double* bb = (double*)calloc(Ni, sizeof(double));
    double* xx = (double*)malloc(sizeof(double) * Ni);
    assemble_from_a(n, a, A);
    cholesky(Ni, A);
    for (int ix = 1; ix < n - 1; ++ix)
      for (int iy = 1; iy < n - 1; ++iy)
        for (int iz = 1; iz < n - 1; ++iz)
          bb[interior_index(n, ix, iy, iz)] = b[((size_t)ix * n + iy) * n + iz];
    cholesky_solve(Ni, A, bb, xx);
    memset(x, 0, sizeof(double) * N);
    for (int ix = 1; ix < n - 1; ++ix)
      for (int iy = 1; iy < n - 1; ++iy)
        for (int iz = 1; iz < n - 1; ++iz)
          x[((size_t)ix * n + iy) * n + iz] = xx[interior_index(n, ix, iy, iz)];
    double* tmp = (double*)malloc(sizeof(double) * N);
    *relres_out = true_relres(n, a, b, x, tmp);
    free(tmp); free(A); free(bb); free(xx);
    return 1;
  }
  if (method == OR_SOLVE_CG) return pcg(n, a, NULL, b, x, rtol, maxit, relres_out);
  mg_t mg;
  mg_build(&mg, n, K, c);
  int it = pcg(n, a, &mg, b, x, rtol, maxit, relres_out);
  mg_free(&mg);
  return it;
}

/* Solve A(c) x = b on the interior; returns the iteration count (1 for the
 * dense solve) and the final true relative residual. */
int or_solve(int n, int K, const double* c, const double* b_in, double* x,
             int method, double rtol, int maxit, double* relres_out) {
  size_t N = (size_t)n * n * n;
  double* b = (double*)malloc(sizeof(double) * N);
  memcpy(b, b_in, sizeof(double) * N);
  mask_boundary(n, b);
  double* a = vertex_coeff(n, K, c);
  int it = solve_with_a(n, K, c, a, b, x, method, rtol, maxit, relres_out);
  free(a);
  free(b);
  return it;
}

/* Phi(y) = 1/2 |y - y_d|_H^2 with the discrete L^2 norm h^3 sum over the
 * interior vertices (cost functional, Sec. 2). */
double or_misfit(int n, const double* y, const double* yd) {
  double h = 1.0 / (double)(n - 1);
  double s = 0.0;
  for (int ix = 1; ix < n - 1; ++ix)
    for (int iy = 1; iy < n - 1; ++iy)
      for (int iz = 1; iz < n - 1; ++iz) {
        size_t v = ((size_t)ix * n + iy) * n + iz;
        double d = y[v] - yd[v];
        s += d * d;
      }
  return 0.5 * h * h * h * s;
}

/* Injection of a finest-grid field to the vertices of a nested coarse grid
 * (the target y_d is a pointwise function, so its coarse values are its
 * values at the coarse vertices). */
static void inject(int nf, const double* fine, int nc, double* coarse) {
  int step = (nf - 1) / (nc - 1);
  for (int jx = 0; jx < nc; ++jx)
    for (int jy = 0; jy < nc; ++jy)
      for (int jz = 0; jz < nc; ++jz)
        coarse[((size_t)jx * nc + jy) * nc + jz] =
            fine[(((size_t)jx * step) * nf + (size_t)jy * step) * nf + (size_t)jz * step];
}

/* ------------------------------------------------------------------ */
/* MLMC gradient estimate (Sec. 2.2) and entropic objective.           */
/* ------------------------------------------------------------------ */
typedef struct {
  int level;
  int64_t m;          /* sample index within the level's draw */
  double phi_f, phi_c;
  double* p_f;        /* adjoint on grid level (fine) */
  double* Pp_c;       /* coarse adjoint prolonged to the fine grid */
  int iters;
  double relres;
} pair_t;

static int check_problem(const or_problem* pb, const int64_t* M) {
  if (pb->L < 1 || pb->L > OR_MAX_LEVELS) return -1;
  for (int i = 0; i < pb->L; ++i) {
    if (pb->n[i] < 3 || M[i] < 1) return -1;
    if (i > 0 && pb->n[i] != 2 * (pb->n[i - 1] - 1) + 1) return -1;
  }
  if (pb->theta < 0.0 || pb->K < 1) return -1;
  return 0;
}

/* Right-hand side and target on every level: b_i = R^(L-1 -> i)(f + u) with
 * boundary entries ignored, y_d injected. */
static void level_data(const or_problem* pb, const double* f, const double* u,
                       const double* yd, double** b, double** ydl) {
  int L = pb->L;
  int nL = pb->n[L - 1];
  size_t NL = (size_t)nL * nL * nL;
  b[L - 1] = (double*)malloc(sizeof(double) * NL);
  for (size_t v = 0; v < NL; ++v) b[L - 1][v] = (f ? f[v] : 0.0) + u[v];
  mask_boundary(nL, b[L - 1]);
  for (int i = L - 2; i >= 0; --i) {
    size_t Ni = (size_t)pb->n[i] * pb->n[i] * pb->n[i];
    b[i] = (double*)malloc(sizeof(double) * Ni);
    or_restrict(pb->n[i + 1], b[i + 1], b[i]);
  }
  for (int i = 0; i < L; ++i) {
    size_t Ni = (size_t)pb->n[i] * pb->n[i] * pb->n[i];
    ydl[i] = (double*)malloc(sizeof(double) * Ni);
    inject(nL, yd, pb->n[i], ydl[i]);
  }
}

/* State solve, misfit, and (optionally) adjoint solve A p = y - y_d for one
 * sample on grid n (the adjoint equation of Sec. 2.1, A symmetric). */
static void sample_solve(const or_problem* pb, int n, const double* c,
                         const double* b, const double* yd, double* phi,
                         double* p /* nullable */, int* iters, double* relres) {
  size_t N = (size_t)n * n * n;
  double* a = vertex_coeff(n, pb->K, c);
  double* y = (double*)malloc(sizeof(double) * N);
  double r1 = 0.0, r2 = 0.0;
  int it = solve_with_a(n, pb->K, c, a, b, y, pb->method, pb->rtol, pb->maxit, &r1);
  *phi = or_misfit(n, y, yd);
  int it2 = 0;
  if (p) {
    double* rhs = (double*)malloc(sizeof(double) * N);
    for (size_t v = 0; v < N; ++v) rhs[v] = y[v] - yd[v];
    mask_boundary(n, rhs);
    it2 = solve_with_a(n, pb->K, c, a, rhs, p, pb->method, pb->rtol, pb->maxit, &r2);
    free(rhs);
  }
  *iters = it > it2 ? it : it2;
  *relres = r1 > r2 ? r1 : r2;
  free(a);
  free(y);
}

static int run_pairs(const or_problem* pb, const double* f, const double* u,
                     const double* yd, const int64_t* M, const int64_t* first,
                     int want_adjoint, pair_t** pairs_out, int64_t* npairs_out) {
  if (check_problem(pb, M)) return -1;
  int L = pb->L;
  double* b[OR_MAX_LEVELS];
  double* ydl[OR_MAX_LEVELS];
  level_data(pb, f, u, yd, b, ydl);
  int64_t np = 0;
  for (int i = 0; i < L; ++i) np += M[i];
  pair_t* pairs = (pair_t*)calloc((size_t)np, sizeof(pair_t));
  int64_t q = 0;
  for (int i = 0; i < L; ++i)
    for (int64_t m = 0; m < M[i]; ++m, ++q) {
      pairs[q].level = i;
      pairs[q].m = (first ? first[i] : 0) + m;
    }
  int nthreads = pb->nthreads > 0 ? pb->nthreads : 1;
  (void)nthreads;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
  for (int64_t t = 0; t < np; ++t) {
    /* largest levels first for load balance */
    pair_t* pr = &pairs[np - 1 - t];
    int i = pr->level;
    int nf = pb->n[i];
    int K = pb->K;
    double* c = (double*)malloc(sizeof(double) * (size_t)(K * K * K));
    or_kl_coeffs_law(pb->seed, pb->common_xi ? 0 : i, pr->m, K, pb->sigma2, pb->law, pb->rho,
                     c);
    size_t Nf = (size_t)nf * nf * nf;
    int itf = 0, itc = 0;
    double rf = 0.0, rc = 0.0;
    if (want_adjoint) pr->p_f = (double*)calloc(Nf, sizeof(double));
    sample_solve(pb, nf, c, b[i], ydl[i], &pr->phi_f, pr->p_f, &itf, &rf);
    if (i > 0) {
      int nc = pb->n[i - 1];
      size_t Nc = (size_t)nc * nc * nc;
      double* pc = want_adjoint ? (double*)calloc(Nc, sizeof(double)) : NULL;
      sample_solve(pb, nc, c, b[i - 1], ydl[i - 1], &pr->phi_c, pc, &itc, &rc);
      if (want_adjoint) {
        pr->Pp_c = (double*)calloc(Nf, sizeof(double));
        or_prolong(nc, pc, pr->Pp_c);
        free(pc);
      }
    }
    pr->iters = itf > itc ? itf : itc;
    pr->relres = rf > rc ? rf : rc;
    free(c);
  }
  for (int i = 0; i < L; ++i) {
    free(b[i]);
    free(ydl[i]);
  }
  *pairs_out = pairs;
  *npairs_out = np;
  return 0;
}

static void free_pairs(pair_t* pairs, int64_t np) {
  for (int64_t q = 0; q < np; ++q) {
    free(pairs[q].p_f);
    free(pairs[q].Pp_c);
  }
  free(pairs);
}

/* Shift s = max Phi over every solve of the estimate; weights e^{theta(Phi-s)}.
 * The ratio E^ML[X]/E^ML[Y] is unchanged by the common factor e^{theta s};
 * the truncation max{1, E^ML[Y]} becomes max{e^{-theta s}, E^ML[Y] e^{-theta s}}. */
static double max_phi(const pair_t* pairs, int64_t np) {
  double s = -INFINITY;
  for (int64_t q = 0; q < np; ++q) {
    if (pairs[q].phi_f > s) s = pairs[q].phi_f;
    if (pairs[q].level > 0 && pairs[q].phi_c > s) s = pairs[q].phi_c;
  }
  return s;
}

static double norm2_h(int n, const double* x) {
  double h = 1.0 / (double)(n - 1);
  return h * h * h * dot_int(n, x, x);
}

static void objective_from_pairs(const or_problem* pb, const double* u,
                                 const int64_t* M, const pair_t* pairs, int64_t np,
                                 or_stats* st) {
  int L = pb->L;
  double s = max_phi(pairs, np);
  double th = pb->theta;
  double EY = 0.0, Ephi = 0.0;
  int64_t q = 0;
  for (int i = 0; i < L; ++i) {
    double sy = 0.0, sphi = 0.0, sphif = 0.0;
    for (int64_t m = 0; m < M[i]; ++m, ++q) {
      double wf = exp(th * (pairs[q].phi_f - s));
      double wc = i > 0 ? exp(th * (pairs[q].phi_c - s)) : 0.0;
      sy += wf - wc;
      sphi += pairs[q].phi_f - (i > 0 ? pairs[q].phi_c : 0.0);
      sphif += pairs[q].phi_f;
    }
    st->mean_dY[i] = sy / (double)M[i];
    st->mean_phi_f[i] = sphif / (double)M[i];
    EY += sy / (double)M[i];
    Ephi += sphi / (double)M[i];
  }
  int nL = pb->n[L - 1];
  double reg = 0.5 * pb->alpha * norm2_h(nL, u);
  st->s = s;
  st->EY_shifted = EY;
  if (th > 0.0) {
    double floor_ = exp(-th * s);
    st->truncated = EY < floor_;
    st->J = s + log(EY > floor_ ? EY : floor_) / th + reg;
  } else {
    st->truncated = 0;
    st->J = Ephi + reg;
  }
  st->max_relres = 0.0;
  st->max_iters = 0;
  for (int64_t t = 0; t < np; ++t) {
    if (pairs[t].relres > st->max_relres) st->max_relres = pairs[t].relres;
    if (pairs[t].iters > st->max_iters) st->max_iters = pairs[t].iters;
  }
}

/* MLMC entropic objective: R_theta estimated as theta^-1 log max{1, E^ML[Y]}
 * (theta = 0: the MLMC mean of Phi), plus alpha/2 |u|_h^2. */
int or_mlmc_objective(const or_problem* pb, const double* f, const double* u,
                      const double* yd, const int64_t* M, const int64_t* first,
                      double* J_out, or_stats* st) {
  pair_t* pairs;
  int64_t np;
  if (run_pairs(pb, f, u, yd, M, first, 0, &pairs, &np)) return -1;
  or_stats loc;
  memset(&loc, 0, sizeof(loc));
  objective_from_pairs(pb, u, M, pairs, np, &loc);
  *J_out = loc.J;
  if (st) *st = loc;
  free_pairs(pairs, np);
  return 0;
}

/* grad = E^ML[X] / max{1, E^ML[Y]} + alpha u on the finest grid, with
 * E^ML[X] = sum_i P^(i -> L-1) mean_m dX_i^(m) and E^ML[Y] = sum_i mean dY_i,
 * dX = w_f p_f - w_c P p_c, dY = w_f - w_c, level 0 without coarse part. */
int or_mlmc_gradient(const or_problem* pb, const double* f, const double* u,
                     const double* yd, const int64_t* M, const int64_t* first,
                     double* grad, or_stats* st_out) {
  pair_t* pairs;
  int64_t np;
  if (run_pairs(pb, f, u, yd, M, first, 1, &pairs, &np)) return -1;
  or_stats st;
  memset(&st, 0, sizeof(st));
  objective_from_pairs(pb, u, M, pairs, np, &st);
  int L = pb->L;
  double s = st.s, th = pb->theta;
  double* acc = NULL;
  int64_t q0 = 0;
  for (int i = 0; i < L; ++i) {
    int n = pb->n[i];
    size_t N = (size_t)n * n * n;
    double* mean = (double*)calloc(N, sizeof(double));
    double* dX = (double*)calloc(N, sizeof(double));
    for (int64_t m = 0; m < M[i]; ++m) {
      const pair_t* pr = &pairs[q0 + m];
      double wf = exp(th * (pr->phi_f - s));
      double wc = i > 0 ? exp(th * (pr->phi_c - s)) : 0.0;
      for (size_t v = 0; v < N; ++v)
        mean[v] += wf * pr->p_f[v] - (i > 0 ? wc * pr->Pp_c[v] : 0.0);
    }
    for (size_t v = 0; v < N; ++v) mean[v] /= (double)M[i];
    /* second-order power sums about the level means (Sec. 4.1) */
    double m2x = 0.0, m2y = 0.0;
    for (int64_t m = 0; m < M[i]; ++m) {
      const pair_t* pr = &pairs[q0 + m];
      double wf = exp(th * (pr->phi_f - s));
      double wc = i > 0 ? exp(th * (pr->phi_c - s)) : 0.0;
      for (size_t v = 0; v < N; ++v)
        dX[v] = wf * pr->p_f[v] - (i > 0 ? wc * pr->Pp_c[v] : 0.0) - mean[v];
      m2x += norm2_h(n, dX);
      double dy = (wf - wc) - st.mean_dY[i];
      m2y += dy * dy;
    }
    st.norm2_mean_dX[i] = norm2_h(n, mean);
    st.m2_dX[i] = m2x;
    st.m2_dY[i] = m2y;
    /* telescoping: acc <- P acc + mean_i */
    if (acc) {
      double* pa = (double*)calloc(N, sizeof(double));
      or_prolong(pb->n[i - 1], acc, pa);
      free(acc);
      acc = pa;
      for (size_t v = 0; v < N; ++v) acc[v] += mean[v];
      free(mean);
    } else {
      acc = mean;
    }
    free(dX);
    q0 += M[i];
  }
  int nL = pb->n[L - 1];
  size_t NL = (size_t)nL * nL * nL;
  st.norm2_EX = norm2_h(nL, acc);
  double denom;
  if (th > 0.0) {
    double floor_ = exp(-th * s);
    denom = st.EY_shifted > floor_ ? st.EY_shifted : floor_;
  } else {
    denom = 1.0;
  }
  for (size_t v = 0; v < NL; ++v) grad[v] = acc[v] / denom + pb->alpha * u[v];
  mask_boundary(nL, grad);
  free(acc);
  if (st_out) *st_out = st;
  free_pairs(pairs, np);
  return 0;
}
