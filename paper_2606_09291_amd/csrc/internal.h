// internal.h -- declarations shared by the kernels and the host runtime of
// libmlsgd (gfx950).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace mlsgd {

constexpr int KMAX = 5;
constexpr int RED_BLOCKS = 256;   // fixed block count of the deterministic dot kernels

// Row layout of the batched solver fields (right-hand sides, iterates,
// coefficient caches, reciprocal diagonals) on a grid with n vertices per
// axis: vertex (x, y, z) of a row sits at (x n + y) lay_pitch(n) + lay_off(n)
// + z, and a row holds lay_row(n) elements.  From 129 vertices on, every z
// line is padded so that its first interior vertex starts a 128-byte line and
// the pitch is a whole number of 128-byte lines in FP64; the padding holds
// zeros.  Smaller grids are stored densely.  Fields that callers and the
// epilogue see (controls, targets, level sums, gradients) are always dense
// [n][n][n].
__host__ __device__ __forceinline__ int lay_off(int n) { return n >= 129 ? 15 : 0; }
__host__ __device__ __forceinline__ int lay_pitch(int n) { return n >= 129 ? (n + 30) & ~15 : n; }
__host__ __device__ __forceinline__ long long lay_row(int n) {
  return (long long)n * n * lay_pitch(n);
}

// Tiling of one grid size for the marching stencil kernels: a workgroup owns
// a TY x TZ patch of the (y, z) plane and marches along x over xchunk planes.
struct Tiling {
  int TY, TZ;
  int nty, ntz, nxc, xchunk;
  int tiles_per_row;
};

// tile_y: y extent of the tiles on grids with more than 32 interior points
// (4, 8 or 16); xchunk: x planes per workgroup.
Tiling make_tiling(int n, int tile_y, int xchunk);

// Per-problem state of the batched Krylov solves (all FP64).
struct CgScal {
  double rz;      // <r, z> of the current iterate
  double pq;      // <p, A p>
  double rr;      // <r, r>
  double bb;      // <b, b>
  double alpha, beta;
  int active;     // 1 while the problem iterates
  int iters;
  int pending;    // x += alpha p of the last step not yet applied
  int pbuf;       // which of the two direction buffers holds that p
  int restart;    // the last true-residual check found rr above rtol
};

// Arguments common to every launch over one grid size.
struct GridArgs {
  int n;                // vertices per axis
  int rows;             // rows (problems) in the launch, rows [0, rows)
  int row0;             // problem index of row 0
  long long stride;     // elements per row, lay_row(n)
  Tiling t;
  const double* coef;   // [problem][K^3] KL coefficients sqrt(sigma2 lam) xi
  int K;
  const double* cosT;   // [K][n] cos(pi k x_i)
  const CgScal* scal;   // per problem; inactive problems are skipped (nullable)
  double ih2;           // 1/h^2
  const void* cache;    // [problem][n^3] cached 1/a of the compute type, or null
  int cache_bf16;       // FP32 sweeps: the cache holds bfloat16 values
  double omega1;        // first step of the fused two-step Jacobi sweep
};

// ---- stencil kernels (marching LDS tiles, coefficient regenerated) ----
template <typename T>
void march_resid(const GridArgs& g, const T* x, const T* b, T* r, hipStream_t s);
// partials of |b - A x|^2 (interior points, one slot per problem and tile, as
// group_dot's), without storing the residual
void march_resid_norm(const GridArgs& g, const double* x, const double* b, const int* poff,
                      double* partial, hipStream_t s);
// p_new = z + beta p_old, q = A p_new, <p_new, q>; with x non-null also the
// step of the previous iteration, x += alpha p_old (alpha still in the
// problem's scalars), which the update then leaves out
template <typename T, typename TZ>
void march_matvec(const GridArgs& g, const TZ* z, const T* p_old, T* p_new, T* q,
                  const int* poff, double* partial, hipStream_t s, T* x = nullptr);
template <typename T>
void march_gs(const GridArgs& g, T* x, const T* b, int color, int x_zero,
              const int* poff, double* partial, int top_begin, double omega, hipStream_t s);
// One damped Jacobi (Chebyshev) step out of place: xout = x + omega D^-1 (b - A x)
// with x = xin + P xc (xc nullable; x_zero: x = 0).  partial: <b, xout>.
template <typename T>
void march_jac(const GridArgs& g, const T* xin, const T* xc, const T* b, T* xout, int x_zero,
               double omega, const int* poff, double* partial, int top_begin, hipStream_t s);
// Fused red-black sweep, out of place, cached coefficient required:
// xout = GS(xin + P xc) (xc nullable; x_zero: xin ignored and taken as 0).
template <typename T>
void rb_sweep(const GridArgs& g, const T* xin, const T* xc, const T* b, T* xout,
              int first_color, int x_zero, const int* poff, double* partial, int top_begin,
              double omega, hipStream_t s);
void coef_cache(int n, int rows, const double* coef, int K, const double* cosT, double* out64,
                float* out32, uint16_t* out16, hipStream_t s);
// reciprocal diagonal 1 / (h^-2 sum_f a_f) of every row from the cached 1/a
template <typename T>
void dinv_rows(int n, int rows, const void* cache, int cache_bf16, T* dinv, hipStream_t s);
// two Jacobi steps from x = 0 in one pass: x2 = J(omega2) J(omega1) 0 (the
// first step x1 = omega1 b / D is formed on the fly from b and 1/D)
template <typename T>
void march_jac2z(const GridArgs& g, const T* dinv, const T* b, T* xout, double omega1,
                 double omega2, hipStream_t s);
// the fused smoothing passes below serve the 8x64, 16x64, 8x32 and 16x16
// tiles (grids of 17 and more vertices, tile height 4 excepted) with a cached
// coefficient
inline bool fused_tiles(const GridArgs& g) {
  return g.cache != nullptr && ((g.t.TZ == 64 && g.t.TY >= 8) || g.t.TZ == 32 || g.t.TZ == 16);
}
// the x chunks of g start on odd planes (one chunk, or chunks of even length)
inline bool pre2r_half_tiles(const GridArgs& g) {
  return g.t.nxc == 1 || (g.t.xchunk & 1) == 0;
}
// the same two steps and the residual of their result in one pass:
// xout = J(omega2) J(omega1) 0, rout = b - A xout (tiles and coefficient as
// fused_tiles; returns false, launching nothing, otherwise).  half: rout
// receives instead the x part of the full-weighting restriction of the
// residual, plane I = r(2I-1)/4 + r(2I)/2 + r(2I+1)/4 at interior columns, for
// restrict_yz_rows (also needs pre2r_half_tiles)
template <typename T>
bool march_pre2r(const GridArgs& g, const T* dinv, const T* b, T* xout, T* rout, double omega1,
                 double omega2, bool half, hipStream_t s);
// two Jacobi steps after the coarse-grid correction in one pass:
// xout = J(omega_b) J(omega_a) (xin + P xc), partials of <b, xout> for the
// problems >= top_begin (partial nullable); xin null: x = 0, not read; same
// tile and coefficient conditions (and xc non-null), false otherwise
template <typename T>
bool march_post2(const GridArgs& g, const T* xin, const T* xc, const T* b, T* xout,
                 double omega_a, double omega_b, const int* poff, double* partial, int top_begin,
                 hipStream_t s);

// The V-cycle from 9^3 down (9^3 -> 5^3 -> 3^3 and back) for `rows` problems
// in one kernel: b9 rows in, z rows out (dense 9^3), Chebyshev steps om[0 ..
// deg-1] (deg <= 8) down and reversed up, exact 3^3 solve, and partials of
// <b, z> for the problems >= top_begin (partial nullable; one slot each).
// c9, c5, c3: cached 1/a of the three grids (bfloat16 when cache_bf16).
struct VsArgs {
  double om[8];
  int deg;
  int top_begin;
};
constexpr int VS_MAXDEG = 8;
template <typename T>
void vcycle_small(int rows, const double* om, int deg, int top_begin, const CgScal* scal,
                  const T* b9, const void* c9, const void* c5, const void* c3, int cache_bf16,
                  T* xout, const int* poff, double* partial, hipStream_t s);

// ---- batched grid transfers (rows of one grid size) ----
template <typename T>
void restrict_rows(int nf, int rows, int row0, const CgScal* scal, const T* fine,
                   T* coarse, hipStream_t s);
// the y and z parts of full weighting from march_pre2r's half output
template <typename T>
void restrict_yz_rows(int nf, int rows, int row0, const CgScal* scal, const T* h, T* coarse,
                      hipStream_t s);
template <typename T>
void prolong_add_rows(int nc, int rows, int row0, const CgScal* scal, const T* coarse,
                      T* fine, hipStream_t s);
// fine rows = trilinear prolongation of the coarse rows (interior vertices;
// every row)
template <typename T>
void prolong_rows(int nc, int rows, const T* coarse, T* fine, hipStream_t s);
// dst rows (FP64, n^3 solver rows) = src rows for the problems row0.. that
// are active, zero for the inactive ones
template <typename TS>
void copy_active_rows(int n, int rows, int row0, const CgScal* scal, const TS* src, double* dst,
                      hipStream_t s);

// ---- dense coarsest-grid solve (hierarchies that stop above 3^3) ----
// pitch (and edge) of one problem's dense coarsest matrix with N unknowns:
// padded to a multiple of the 16 x 16 tiles of the factorisation
__host__ __device__ __forceinline__ int dense_pitch(int N) { return (N + 15) / 16 * 16; }
void dense_coarse_inv(int n, int rows, const double* coef, int K, const double* cosT,
                      double* ainv, double* work, hipStream_t s);
template <typename T>
void dense_apply(int n, int rows, const CgScal* scal, const double* ainv, const T* b, T* x,
                 hipStream_t s);
// solver rows [count] to dense rows at per-row destination offsets
void scatter_rows(int n, int count, const long long* dst_off, const double* src, double* dst,
                  hipStream_t s);
void fill_interior(int n, double v, double* out, hipStream_t s);

// ---- random field ----
void kl_coeffs(const int* prob_level, const int64_t* prob_sample, int nprob,
               uint64_t seed, int K, double sigma2, int law, double rho, double* coef,
               hipStream_t s);
void kl_draws(uint64_t seed, int level, int64_t first, int64_t count, int K3, int law,
              double* xi, hipStream_t s);
void philox_words(uint64_t seed, int level, int64_t sample, int tag, int nblocks,
                  uint64_t* out, hipStream_t s);
void cos_table(int n, int K, double* out, hipStream_t s);

// ---- elementwise over the rows of one group (lay_row(n) per row) ----
// one dense field copied into every solver row
void rows_broadcast(int n, int rows, const double* src, double* dst, hipStream_t s);
// solver rows copied (copy_rows) or converted to dense rows (unpack_rows)
void copy_rows(int n, int rows, const double* src, double* dst, hipStream_t s);
// partial slots of problem p0 (pc of them) copied to problems p0+1 .. p0+count-1
void replicate_slots(int p0, int count, int pc, const int* poff, double* partial, hipStream_t s);
void unpack_rows(int n, int rows, const double* src, double* dst, hipStream_t s);
void rows_zero(long long count, double* x, hipStream_t s);
void to_f32(long long count, const double* x, float* y, hipStream_t s);
void group_dot(const GridArgs& g, const double* a, const double* b, const int* poff,
               double* partial, hipStream_t s);
void group_update(const GridArgs& g, double* x, const double* p, double* r,
                  const double* q, const int* poff, double* partial, float* r32,
                  hipStream_t s);
// r -= alpha q and <r, r> (x is updated by the next matvec or group_xflush)
void group_rupdate(const GridArgs& g, double* r, const double* q, const int* poff,
                   double* partial, float* r32, hipStream_t s);
// x += alpha p for every problem with a pending step, p from buffer p0 or p1
// as its scalars record (g.scal must be set; active or not)
void group_xflush(const GridArgs& g, double* x, const double* p0, const double* p1,
                  hipStream_t s);
// b = y - y_d on the interior (y_d dense), y reset to 0, partials of |b|^2
void group_misfit(const GridArgs& g, double* y, const double* yd, double* b_rows,
                  const int* poff, double* partial, hipStream_t s);

// ---- per-problem scalar steps of the batched Krylov method ----
enum ScalPhase {
  PH_INIT_BB = 0,    // bb = rr = sum; active = bb > 0; iters = 0
  PH_RZ0 = 1,        // rz = sum; beta = 0
  PH_RZ0_RR = 2,     // unpreconditioned start: rz = rr; beta = 0
  PH_ALPHA = 3,      // pq = sum; alpha = rz / pq; x += alpha p pending, p in buffer aux
  PH_RR = 4,         // rr = sum; ++iters; converged or out of iterations -> inactive
  PH_RZ = 5,         // rz_new = sum; beta = rz_new / rz; rz = rz_new
  PH_RZ_RR = 6,      // unpreconditioned: rz_new = rr
  PH_TRUE = 7,       // rr = sum (true residual); active = restart = rr > rtol^2 bb; nothing pending
  PH_RECHECK = 8,    // active = restart: the problems the last check restarted (no sum)
  PH_FORCE_RESTART = 9,  // test hook: every even-numbered problem with b != 0 restarts
};
void cg_scalar(int phase, CgScal* scal, int nprob, const int* poff, const int* pcnt,
               const double* partial, double rtol, int max_iters, int* active_count,
               hipStream_t s, int aux = 0);
void scal_to_stats(const CgScal* scal, int nprob, double rtol, int* iters_max,
                   int* nonconv, double* relres_max, hipStream_t s);
void sum_partials(int nprob, const int* poff, const int* pcnt, const double* partial,
                  double scale, double* dst, hipStream_t s);

// ---- whole-field kernels on one grid (epilogue, control transfer) ----
void restrict_full(int nf, const double* fine, double* coarse, hipStream_t s);
void prolong_full(int nc, const double* coarse, double* fine, hipStream_t s);
void inject_full(int nf, const double* fine, int nc, double* coarse, hipStream_t s);
void add_mask(int n, const double* f, const double* u, double* out, hipStream_t s);
void axpy_full(int n, double a, const double* x, double* y, hipStream_t s);
void dot_blocks(long long N, const double* a, const double* b, double* part,
                hipStream_t s);   // RED_BLOCKS partials of sum a*b
void box_step(int n, double* u, const double* g, double tau, double lo, double hi,
              int use_box, hipStream_t s);
void nonfinite_flag(long long count, const double* x, int* flag, hipStream_t s);
void copy_elems(long long count, const double* src, double* dst, hipStream_t s);

// ---- entropic epilogue ----
void shift_weights(int nprob, const double* phi, double theta, double* w, double* s_out,
                   hipStream_t s);
int level_sample_blocks(int M);
// pf, pc: solver rows of the level's fine and coarse solves; part, mean dense
void level_dx_partial(int nf, int M, const double* pf, const double* wf, const double* pc,
                      const double* wc, double* part, hipStream_t s);
void level_dx_mean(int nf, int M, const double* part, double* mean, hipStream_t s);
int level_m2_chunks(int nf);
void level_dx_m2(int nf, int M, const double* pf, const double* wf, const double* pc,
                 const double* wc, const double* mean, double* part2, hipStream_t s);

struct EpiLevel {   // one level of the estimate, for the scalar epilogue
  int M;
  int fine_off;     // problem index of the first fine problem
  int coarse_off;   // problem index of the first coarse problem (-1 on level 0)
  int nf;
  long long m2_off; // offset of this level's M2 partials in the partial buffer
  int m2_cnt;
  long long nm_off; // offset of the RED_BLOCKS partials of |mean|^2
};
struct EpiOut {     // device-side scalar results, copied to the host once
  double s, EY, denom, J, gnorm2, unorm2, exnorm2;
  double mean_dY[8], norm2_mean_dX[8], m2_dX[8], m2_dY[8], mean_phi_f[8];
  int truncated, pad;
  unsigned long long work[8];  // per level: sum of interior unknowns x Krylov iterations
};
// zero the per-level work sums of an estimate
void level_work_zero(EpiOut* out, hipStream_t s);
// add every problem's interior unknowns x iterations (its grid has n vertices
// per axis) to the work sum of the level whose draw it uses
void level_work_add(int count, int n, const int* prob_level, const CgScal* scal, EpiOut* out,
                    hipStream_t s);
void epilogue_scalars(int L, const EpiLevel* lev, const double* phi, const double* w,
                      const double* part, long long u_off, int nL, double theta,
                      double alpha, int with_dx, EpiOut* out, hipStream_t s);
void final_grad(int n, const double* acc, const double* u, const EpiOut* eo, double alpha,
                double* grad, hipStream_t s);
void finish_norm(int n, const double* part, double* dst, hipStream_t s);  // h^3 sum

}  // namespace mlsgd
