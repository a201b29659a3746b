// runtime.hip -- host runtime and C ABI of libmlsgd (gfx950).
//
// A call builds (or reuses) a plan: the list of problems (level, sample,
// grid) of the estimate, sorted by grid size so that every grid size of the
// multigrid hierarchy holds a prefix of the problems.  All problems of all
// levels are then solved in lockstep by one batched Krylov iteration whose
// kernels each cover every problem that lives on one grid size; converged
// problems are skipped by the kernels.  The host only enqueues kernels and
// reads one integer (problems still active) per iteration.
#include "mlsgd.h"
#include "internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <functional>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

using namespace mlsgd;

// Device memory of mlsgd_solve_state_adjoint_noalloc: its solver rows,
// Krylov vectors, coefficient caches and partial sums are carved from this
// array instead of an arena of their own.  Every GPU the library runs on
// holds one copy until the process ends.  Host code never uses the name
// itself as an address: each device's address comes from
// hipGetSymbolAddress at context creation (scratch_on_device).
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

struct Fail {
  int code;
  std::string msg;
};

#define HIPCHK(x)                                                                 \
  do {                                                                            \
    hipError_t e_ = (x);                                                          \
    if (e_ != hipSuccess)                                                         \
      throw Fail{e_ == hipErrorOutOfMemory ? MLSGD_EOOM : MLSGD_EHIP,             \
                 std::string(#x) + ": " + hipGetErrorString(e_)};                 \
  } while (0)

static void require(bool ok, const std::string& msg) {
  if (!ok) throw Fail{MLSGD_EINVAL, msg};
}

static bool is_dyadic(int n) {
  if (n < 3) return false;
  int m = n - 1;
  return (m & (m - 1)) == 0;
}

static inline size_t cube(int n) { return (size_t)n * n * n; }
// elements of one solver row (padded z lines from 129 vertices on)
static inline size_t srow(int n) { return (size_t)lay_row(n); }

// One grid size of the hierarchy: rows [0, rows) are the problems whose top
// grid is at least this size; rows [top_begin, rows) have exactly this top.
struct SizeLvl {
  int n = 0, rows = 0, top_begin = 0;
  Tiling t{};
  double *X = nullptr, *B = nullptr, *R = nullptr;  // FP64 multigrid rows (B: Krylov r on top rows)
  double* C = nullptr;                              // FP64 cache of 1/a (null: regenerate)
  float *Xf = nullptr, *Bf = nullptr, *Rf = nullptr;  // FP32 multigrid rows (mixed precision)
  float* Cf = nullptr;                              // FP32 cache of 1/a (null: regenerate)
  uint16_t* Cb = nullptr;                           // bfloat16 cache of 1/a (BF16 smoothing)
  double* Di = nullptr;                             // FP64 reciprocal diagonal (with C)
  float* Dif = nullptr;                             // FP32 reciprocal diagonal (with Cf / Cb)
  const double* cosT = nullptr;
  int cur = 0;   // fused sweeps: which of X/R (Xf/Rf) holds the current iterate
};

// Problems sharing a top grid: Krylov vectors.
struct Group {
  int n = 0, p0 = 0, count = 0, sl = 0;
  double *x = nullptr, *q = nullptr, *b0 = nullptr;
  double* p[2] = {nullptr, nullptr};
  int pcur = 0;
};

struct Block {   // a run of problems on one grid keyed by one level's draws
  int n;
  int level;
  int64_t first;
  int64_t count;
};

struct Plan {
  std::string key;
  int nprob = 0;
  std::vector<int> h_n, h_level;
  std::vector<int64_t> h_sample;
  std::vector<int> h_poff, h_pcnt;
  std::vector<Group> groups;
  std::vector<SizeLvl> sizes;
  int* d_level = nullptr;
  int64_t* d_sample = nullptr;
  double* d_coef = nullptr;
  CgScal* d_scal = nullptr;
  int* d_poff = nullptr;
  int* d_pcnt = nullptr;
  double* d_partial = nullptr;
  double* d_phi = nullptr;
  double* d_w = nullptr;
  double* ainv = nullptr;  // coarsest-grid inverses [rows][Np][Np] when the hierarchy stops above 3^3
  double* dwork = nullptr; // their factorisation's L^-1, same shape
  int dense_N = 0;
  long long npartial = 0;  // partial-sum slots (one per workgroup tile of every problem)
  void* arena = nullptr;
  size_t arena_bytes = 0;
  uint64_t last_use = 0;   // plan-cache clock at the latest get_plan
};

}  // namespace

struct mlsgd_ctx {
  mlsgd_problem pb{};
  hipStream_t stream = nullptr;
  std::string err;
  int nfin = 0;                            // finest grid of the problem
  double* d_f = nullptr;                   // finest-grid f (zero if not given)
  double* d_yd = nullptr;                  // finest-grid target
  std::map<int, double*> cosT;             // per grid size
  std::map<int, double*> yd_lvl;           // target injected per level grid
  std::map<int, double*> rhs_lvl;          // R(f + u) per level grid
  std::map<int, double*> mean_lvl;         // E_i[dX] per level grid
  std::map<int, double*> acc_lvl;          // telescoped sum per level grid
  double* d_umask = nullptr;               // u with zero boundary (finest)
  double* d_grad = nullptr;                // gradient scratch for mlsgd_step
  double* d_epi_part = nullptr;
  size_t epi_part_len = 0;
  double* d_dxpart = nullptr;
  size_t dxpart_len = 0;
  EpiLevel* d_epi_lev = nullptr;
  EpiOut* d_epi_out = nullptr;
  EpiOut* h_epi_out = nullptr;             // pinned
  int* d_count = nullptr;
  int* h_count = nullptr;                  // pinned
  struct StatDev { int iters, nonconv; double relres; };
  StatDev* d_stat = nullptr;               // [2]: state and adjoint solves
  StatDev* h_stat = nullptr;               // pinned, [2]
  // graph mode: each batch shape runs as one replayed HIP graph
  struct GraphEntry {
    hipGraphExec_t exec = nullptr;
    int it_s = 0, it_a = 0;   // iteration counts the graph runs
    int margin = 1;           // iterations beyond the learned counts
  };
  bool graph = false;
  hipStream_t cap_stream = nullptr;        // capture stream (default priority)
  double* d_u_graph = nullptr;             // u as the graph reads it
  double* d_g_graph = nullptr;             // gradient as the graph writes it
  std::map<std::string, GraphEntry> graphs;
  int* d_flag = nullptr;
  std::map<std::string, std::unique_ptr<Plan>> plans;
  uint64_t plan_clock = 0;
  std::map<int, double*> const_rhs;        // constant interior right-hand sides per grid
  long long* d_dst_off = nullptr;          // packed-output offsets of one solve batch
  size_t dst_off_len = 0;
  std::vector<void*> allocs;
  int device = 0;                          // device current at mlsgd_create
  void* scratch = nullptr;                 // this device's address of `scratch`
  // batch used by mlsgd_step
  int cur_L = 0;
  int64_t cur_M[MLSGD_MAX_LEVELS] = {0};
  int64_t cur_off[MLSGD_MAX_LEVELS] = {0};
  double prev_gnorm = -1.0;
  // adaptive step size: the previous gradient and step
  double* d_gprev = nullptr;
  double* d_gtmp = nullptr;
  double* d_sc1 = nullptr;   // one device double
  bool have_gprev = false;
  double tau_prev = 0.0, tau_pos = 0.0, gnorm_prev = 0.0;
  hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
  // tunables of the solver (defaults from measurement; overridable for tuning)
  int nu = 2;               // smoothing sweeps before and after the coarse correction
  double omega = 1.0;       // red-black relaxation weight
  bool cache64 = true;      // cache 1/a per estimate for FP64 sweeps
  bool cache32 = true;      // cache 1/a per estimate for FP32 sweeps
  bool mixed = false;       // FP32 V-cycles inside the FP64 Krylov iteration
  bool bf16 = false;        // mixed, with the smoother's coefficient stored as bfloat16
  int smoother = 2;         // 0 red-black GS (two in-place passes), 1 fused red-black, 2 Chebyshev
  double cheb_lo = 0.15;    // Chebyshev interval [cheb_lo * 2, 2] for D^-1 A
  int tile_y = 8;           // y extent of the stencil tiles on large grids
  int xchunk = 32;          // x planes per workgroup
  bool pre2r = true;        // fused pre-smoothing and residual pass where it applies
  bool pre2r_half = true;   // that pass writes the residual restricted along x
  bool post2 = true;        // fused two-step post-smoothing pass where it applies
  bool vsmall = true;       // the cycle from 9^3 down as one kernel where it applies
  bool xdefer = true;       // x's Krylov step applied by the next matvec
  bool fmg = true;          // full-multigrid start of the Krylov solves
  double fmg_margin = 0.7;  // recursive-residual target as a fraction of rtol after that start
  // Krylov iterations whose active count the host does not read (no solve
  // of the previous call finished before them); results do not depend on it
  int kry_quiet = 0;
  // test hook: after a solve's first true-residual check, restart every
  // even-numbered problem as well (exercises the restart path on converged
  // problems, whose result then moves by at most the solver tolerance)
  bool force_restart = false;
  // event timing of the smoothing passes on one grid size (roofline figures)
  struct Timing {
    bool on = false;
    int kind = 1;            // 1 plain smoothing step, 2 fused post-smoothing pass
    int n = 0;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
    size_t used = 0;
    std::vector<double> bytes;   // algorithmic bytes of each recorded launch
    double ms = 0.0, total_bytes = 0.0;
    int64_t launches = 0;
  } tm;
};

namespace {

void* dalloc(mlsgd_ctx* c, size_t bytes) {
  void* p = nullptr;
  if (bytes == 0) bytes = 256;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw Fail{MLSGD_EOOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed"};
  }
  c->allocs.push_back(p);
  return p;
}

const double* cos_for(mlsgd_ctx* c, int n) {
  auto it = c->cosT.find(n);
  if (it != c->cosT.end()) return it->second;
  double* d = (double*)dalloc(c, sizeof(double) * (size_t)n * c->pb.kl_K);
  cos_table(n, c->pb.kl_K, d, c->stream);
  HIPCHK(hipGetLastError());
  c->cosT[n] = d;
  return d;
}

// Arena carving with 256-byte alignment.
struct Carver {
  char* base;
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T* p = (T*)(base ? base + off : nullptr);
    off += sizeof(T) * (count ? count : 1);
    return p;
  }
};

void plan_fields(mlsgd_ctx* c, Plan* P);
void drop_graphs(mlsgd_ctx* c);

// Plan cache bounds.  Layouts are kept per batch shape; beyond kMaxPlans
// plans or kPlanBytes of arenas the least recently used one is freed (its
// captured graphs with it), so a caller that meets ever new shapes -- the
// adaptive batch controller's -- keeps a bounded footprint.
constexpr size_t kMaxPlans = 8;
constexpr size_t kPlanBytes = (size_t)96 << 30;

// Free one allocation of dalloc (after the context's queued work, which may
// still use it).
void dfree(mlsgd_ctx* c, void* p) {
  if (!p) return;
  HIPCHK(hipStreamSynchronize(c->stream));
  for (size_t i = 0; i < c->allocs.size(); ++i)
    if (c->allocs[i] == p) {
      c->allocs[i] = c->allocs.back();
      c->allocs.pop_back();
      break;
    }
  HIPCHK(hipFree(p));
}

void free_plan(mlsgd_ctx* c, Plan* P) {
  dfree(c, P->arena);
  P->arena = nullptr;
}

void drop_plans(mlsgd_ctx* c) {
  drop_graphs(c);   // captured graphs point into the plans' memory
  for (auto& kv : c->plans) free_plan(c, kv.second.get());
  c->plans.clear();
}

// Make room for a new plan of `need` arena bytes (not yet in the cache).
void evict_plans(mlsgd_ctx* c, size_t need) {
  for (;;) {
    size_t total = 0;
    for (const auto& kv : c->plans) total += kv.second->arena_bytes;
    if (c->plans.empty() || (c->plans.size() < kMaxPlans && total + need <= kPlanBytes)) return;
    auto lru = c->plans.begin();
    for (auto it = c->plans.begin(); it != c->plans.end(); ++it)
      if (it->second->last_use < lru->second->last_use) lru = it;
    drop_graphs(c);
    free_plan(c, lru->second.get());
    c->plans.erase(lru);
  }
}

// Host-side layout of a list of blocks (grid sizes non-increasing): problem
// order, groups, the grid sizes of the hierarchy and the partial-sum slots.
// Touches no device memory beyond the per-size cosine tables.
void plan_layout(mlsgd_ctx* c, const std::vector<Block>& blocks, Plan* P) {
  long long np = 0;
  for (const auto& b : blocks) np += b.count;
  require(np > 0 && np < (1LL << 30), "problem count out of range");
  P->nprob = (int)np;
  P->h_n.resize(np);
  P->h_level.resize(np);
  P->h_sample.resize(np);
  // groups
  int p = 0;
  for (size_t bi = 0; bi < blocks.size(); ++bi) {
    const Block& b = blocks[bi];
    require(bi == 0 || b.n <= blocks[bi - 1].n, "blocks must have non-increasing grids");
    if (P->groups.empty() || P->groups.back().n != b.n) {
      Group g;
      g.n = b.n;
      g.p0 = p;
      g.count = 0;
      P->groups.push_back(g);
    }
    for (int64_t m = 0; m < b.count; ++m, ++p) P->h_n[p] = b.n;
    P->groups.back().count += (int)b.count;
  }
  // grid sizes from the largest top grid down to 3, or down to the first
  // grid with an odd number of cells, which cannot be coarsened further
  int nmax = blocks.front().n;
  for (int n = nmax;; n = (n - 1) / 2 + 1) {
    SizeLvl s;
    s.n = n;
    s.t = make_tiling(n, c->tile_y, c->xchunk);
    int rows = 0, top = 0;
    for (int q = 0; q < P->nprob; ++q) {
      if (P->h_n[q] >= n) rows = q + 1;
      if (P->h_n[q] > n) top = q + 1;
    }
    s.rows = rows;
    s.top_begin = top;
    s.cosT = cos_for(c, n);
    P->sizes.push_back(s);
    if (n <= 3 || ((n - 1) & 1)) break;
  }
  {
    const SizeLvl& co = P->sizes.back();
    if (co.n > 3) {
      require(co.n <= 9, "the grid hierarchy must coarsen to at most 9^3");
      require(P->sizes.size() >= 2 && co.top_begin == co.rows,
              "a top grid cannot be the dense coarsest grid");
      P->dense_N = (co.n - 2) * (co.n - 2) * (co.n - 2);
    }
  }
  for (auto& g : P->groups) {
    for (size_t k = 0; k < P->sizes.size(); ++k)
      if (P->sizes[k].n == g.n) g.sl = (int)k;
  }
  P->h_pcnt.resize(np);
  P->h_poff.resize(np);
  long long off = 0;
  for (int q = 0; q < P->nprob; ++q) {
    P->h_pcnt[q] = make_tiling(P->h_n[q], c->tile_y, c->xchunk).tiles_per_row;
    P->h_poff[q] = (int)off;
    off += P->h_pcnt[q];
  }
  require(off < (1LL << 31), "partial buffer too large");
  P->npartial = off;
}

// Assign the plan's arrays inside the arena at `base` (nullptr: only
// measure); returns the arena bytes the layout needs.
size_t plan_carve(mlsgd_ctx* c, Plan* P, char* base) {
  const int K = c->pb.kl_K, K3 = K * K * K;
  const long long np = P->nprob;
  Carver cv{base};
  for (auto& s : P->sizes) {
    const size_t e = (size_t)s.rows * srow(s.n);
    s.B = cv.take<double>(e);
    if (!c->mixed) {
      s.X = cv.take<double>(e);
      s.R = cv.take<double>(e);
    } else {
      s.Xf = cv.take<float>(e);
      s.Bf = cv.take<float>(e);
      s.Rf = cv.take<float>(e);
      if (c->cache32 && c->bf16) s.Cb = cv.take<uint16_t>(e);
      else if (c->cache32) s.Cf = cv.take<float>(e);
      if (c->cache32) s.Dif = cv.take<float>(e);
    }
    if (c->cache64) s.C = cv.take<double>(e);
    if (c->cache64 && !c->mixed) s.Di = cv.take<double>(e);
  }
  for (auto& g : P->groups) {
    const size_t e = (size_t)g.count * srow(g.n);
    g.x = cv.take<double>(e);
    g.q = cv.take<double>(e);
    g.b0 = cv.take<double>(e);
    g.p[0] = cv.take<double>(e);
    g.p[1] = cv.take<double>(e);
  }
  P->d_level = cv.take<int>(np);
  P->d_sample = cv.take<int64_t>(np);
  P->d_coef = cv.take<double>((size_t)np * K3);
  P->d_scal = cv.take<CgScal>(np);
  P->d_poff = cv.take<int>(np);
  P->d_pcnt = cv.take<int>(np);
  P->d_partial = cv.take<double>((size_t)P->npartial);
  P->d_phi = cv.take<double>(np);
  P->d_w = cv.take<double>(np);
  if (P->dense_N) {
    const size_t np = (size_t)dense_pitch(P->dense_N);
    P->ainv = cv.take<double>((size_t)P->sizes.back().rows * np * np);
    P->dwork = cv.take<double>((size_t)P->sizes.back().rows * np * np);
  }
  return ((cv.off + 255) & ~(size_t)255) + 256;
}

// Zero a freshly assigned arena (a fill kernel, so no memset node is ever
// recorded) and upload the partial-sum slots.
void plan_init(mlsgd_ctx* c, Plan* P) {
  rows_zero((long long)(P->arena_bytes / sizeof(double)), (double*)P->arena, c->stream);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(P->d_poff, P->h_poff.data(), sizeof(int) * P->nprob,
                        hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(P->d_pcnt, P->h_pcnt.data(), sizeof(int) * P->nprob,
                        hipMemcpyHostToDevice, c->stream));
}

// Upload the (level, sample) keys of this call's draws; `fields` also
// regenerates the coefficient fields from them (kernels only: plan_fields).
void plan_draws(mlsgd_ctx* c, Plan* P, const std::vector<Block>& blocks, bool fields) {
  int p = 0;
  for (const auto& b : blocks)
    for (int64_t m = 0; m < b.count; ++m, ++p) {
      P->h_level[p] = b.level;
      P->h_sample[p] = b.first + m;
    }
  HIPCHK(hipMemcpyAsync(P->d_level, P->h_level.data(), sizeof(int) * P->nprob,
                        hipMemcpyHostToDevice, c->stream));
  HIPCHK(hipMemcpyAsync(P->d_sample, P->h_sample.data(), sizeof(int64_t) * P->nprob,
                        hipMemcpyHostToDevice, c->stream));
  if (fields) plan_fields(c, P);
}

// Build (or reuse) the layout for a list of blocks (grid sizes
// non-increasing) in an arena of its own and upload this call's draws.
Plan* get_plan(mlsgd_ctx* c, const std::vector<Block>& blocks, bool fields = true) {
  std::string key;
  for (const auto& b : blocks) key += std::to_string(b.n) + ":" + std::to_string(b.count) + ";";
  auto it = c->plans.find(key);
  Plan* P = nullptr;
  if (it != c->plans.end()) {
    P = it->second.get();
  } else {
    auto up = std::make_unique<Plan>();
    P = up.get();
    P->key = key;
    plan_layout(c, blocks, P);
    P->arena_bytes = plan_carve(c, P, nullptr);
    evict_plans(c, P->arena_bytes);
    P->arena = dalloc(c, P->arena_bytes);
    plan_carve(c, P, (char*)P->arena);
    plan_init(c, P);
    c->plans[key] = std::move(up);
  }
  P->last_use = ++c->plan_clock;
  plan_draws(c, P, blocks, fields);
  return P;
}

// KL coefficients of the uploaded draws, the per-grid coefficient caches and
// the dense coarsest inverses.
void plan_fields(mlsgd_ctx* c, Plan* P) {
  const int K = c->pb.kl_K;
  kl_coeffs(P->d_level, P->d_sample, P->nprob, c->pb.seed, K, c->pb.kl_sigma2, c->pb.kl_law,
            c->pb.kl_rho, P->d_coef, c->stream);
  // the coefficient is regenerated from the draws once per call for the
  // cached sweeps (the Krylov matvec and residual always run in FP64)
  for (auto& sl : P->sizes) {
    coef_cache(sl.n, sl.rows, P->d_coef, K, sl.cosT, sl.C, sl.Cf, sl.Cb, c->stream);
    if (sl.Di) dinv_rows<double>(sl.n, sl.rows, sl.C, 0, sl.Di, c->stream);
    if (sl.Dif)
      dinv_rows<float>(sl.n, sl.rows, sl.Cb ? (const void*)sl.Cb : (const void*)sl.Cf,
                       sl.Cb ? 1 : 0, sl.Dif, c->stream);
  }
  if (P->dense_N) {
    const SizeLvl& co = P->sizes.back();
    dense_coarse_inv(co.n, co.rows, P->d_coef, K, co.cosT, P->ainv, P->dwork, c->stream);
  }
  HIPCHK(hipGetLastError());
}

GridArgs args_size(mlsgd_ctx* c, Plan* P, const SizeLvl& s) {
  GridArgs g;
  g.n = s.n;
  g.rows = s.rows;
  g.row0 = 0;
  g.stride = (long long)srow(s.n);
  g.t = s.t;
  g.coef = P->d_coef;
  g.K = c->pb.kl_K;
  g.cosT = s.cosT;
  g.scal = P->d_scal;
  g.ih2 = (double)(s.n - 1) * (double)(s.n - 1);
  g.cache = s.C;
  g.cache_bf16 = 0;
  g.omega1 = 0.0;
  return g;
}

// launch arguments of the FP32 multigrid sweeps on one grid size
GridArgs args_size32(mlsgd_ctx* c, Plan* P, const SizeLvl& s) {
  GridArgs g = args_size(c, P, s);
  g.cache = s.Cb ? (const void*)s.Cb : (const void*)s.Cf;
  g.cache_bf16 = s.Cb ? 1 : 0;
  return g;
}

GridArgs args_group(mlsgd_ctx* c, Plan* P, const Group& gr, bool skip_inactive) {
  GridArgs g = args_size(c, P, P->sizes[gr.sl]);
  g.rows = gr.count;
  g.row0 = gr.p0;
  g.scal = skip_inactive ? P->d_scal : nullptr;
  return g;
}

inline double* rows_of(double* base, const Group& gr) { return base + (size_t)gr.p0 * srow(gr.n); }

// Symmetric V(nu,nu) cycle for every active problem: z = V(r) with r in the
// B rows of each problem's top grid and z left in its X rows.  Pre-smoothing
// sweeps are red then black starting from a zero guess, post-smoothing
// sweeps black then red (the cycle is a symmetric preconditioner); the last
// red pass also forms <r, z> for the problems whose top grid it is.  On the
// 3^3 grid the single unknown is black and one sweep is an exact solve.
template <typename T>
struct MgView {
  T *X, *B, *R;
};
template <typename T>
MgView<T> mg_view(SizeLvl& L);
template <>
MgView<double> mg_view<double>(SizeLvl& L) { return {L.X, L.B, L.R}; }
template <>
MgView<float> mg_view<float>(SizeLvl& L) { return {L.Xf, L.Bf, L.Rf}; }

// Algorithmic bytes of one red-black pass over `rows` rows of an n^3 grid:
// x read at every interior point (not when starting from zero), b read and x
// written at the updated half, x zeroed at the other half on a zero start,
// the cached coefficient read at every point, b read at the other half when
// the pass also forms <b, x>.
template <typename T>
double gs_pass_bytes(const mlsgd_ctx* c, int n, int rows, bool x_zero, bool cached, bool dot) {
  const double N = (double)rows * (double)(n - 2) * (double)(n - 2) * (double)(n - 2);
  const double e = (double)sizeof(T);
  double b = 0.5 * e + 0.5 * e;          // b and x on the updated half
  b += x_zero ? 0.5 * e : e;             // x read, or the other half zeroed
  if (dot) b += 0.5 * e;
  (void)c;
  (void)cached;                          // the coefficient counts 0 bytes (regenerated)
  return N * b;
}

template <typename T>
void timed_gs(mlsgd_ctx* c, const GridArgs& g, T* x, const T* b, int color, int x_zero,
              const int* poff, double* partial, int top_begin, double om) {
  mlsgd_ctx::Timing& tm = c->tm;
  const bool rec = tm.on && g.n == tm.n && g.rows > 0;
  if (rec) {
    if (tm.used == tm.pool.size()) {
      hipEvent_t a, e;
      HIPCHK(hipEventCreate(&a));
      HIPCHK(hipEventCreate(&e));
      tm.pool.push_back({a, e});
    }
    HIPCHK(hipEventRecord(tm.pool[tm.used].first, c->stream));
  }
  march_gs<T>(g, x, b, color, x_zero, poff, partial, top_begin, om, c->stream);
  if (rec) {
    HIPCHK(hipEventRecord(tm.pool[tm.used].second, c->stream));
    tm.bytes.push_back(gs_pass_bytes<T>(c, g.n, g.rows, x_zero != 0, g.cache != nullptr,
                                        partial != nullptr));
    ++tm.used;
  }
}

// Fold the recorded event pairs into the totals (the stream is synchronised).
void timing_collect(mlsgd_ctx* c) {
  mlsgd_ctx::Timing& tm = c->tm;
  for (size_t i = 0; i < tm.used; ++i) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, tm.pool[i].first, tm.pool[i].second));
    tm.ms += ms;
    tm.total_bytes += tm.bytes[i];
    ++tm.launches;
  }
  tm.used = 0;
  tm.bytes.clear();
}

// Algorithmic bytes of one fused red-black sweep over `rows` rows: previous
// iterate read (not on a zero start), b read, new iterate written, and, when
// the coarse correction is folded in, the coarse rows read once (the
// coefficient counts 0 bytes: it is regenerated from the draws).
template <typename T>
double sweep_bytes(int n, int rows, bool x_zero, bool prolong) {
  const double N = (double)rows * (double)(n - 2) * (double)(n - 2) * (double)(n - 2);
  const double e = (double)sizeof(T);
  double b = 2.0 * e + (x_zero ? 0.0 : e);
  if (prolong) b += e / 8.0;
  return N * b;
}

template <typename T>
void timed_sweep(mlsgd_ctx* c, const GridArgs& g, const T* xin, const T* xc, const T* b, T* xout,
                 int first_color, int x_zero, const int* poff, double* partial, int top_begin,
                 double om) {
  mlsgd_ctx::Timing& tm = c->tm;
  const bool rec = tm.on && g.n == tm.n && g.rows > 0;
  if (rec) {
    if (tm.used == tm.pool.size()) {
      hipEvent_t a, e;
      HIPCHK(hipEventCreate(&a));
      HIPCHK(hipEventCreate(&e));
      tm.pool.push_back({a, e});
    }
    HIPCHK(hipEventRecord(tm.pool[tm.used].first, c->stream));
  }
  rb_sweep<T>(g, xin, xc, b, xout, first_color, x_zero, poff, partial, top_begin, om, c->stream);
  if (rec) {
    HIPCHK(hipEventRecord(tm.pool[tm.used].second, c->stream));
    tm.bytes.push_back(sweep_bytes<T>(g.n, g.rows, x_zero != 0, xc != nullptr));
    ++tm.used;
  }
}

template <typename F>
void timed_launch(mlsgd_ctx* c, const GridArgs& g, double bytes, F&& fn, int kind = 1) {
  mlsgd_ctx::Timing& tm = c->tm;
  const bool rec = tm.on && tm.kind == kind && g.n == tm.n && g.rows > 0;
  if (rec) {
    if (tm.used == tm.pool.size()) {
      hipEvent_t a, e;
      HIPCHK(hipEventCreate(&a));
      HIPCHK(hipEventCreate(&e));
      tm.pool.push_back({a, e});
    }
    HIPCHK(hipEventRecord(tm.pool[tm.used].first, c->stream));
  }
  fn();
  if (rec) {
    HIPCHK(hipEventRecord(tm.pool[tm.used].second, c->stream));
    tm.bytes.push_back(bytes);
    ++tm.used;
  }
}

// Chebyshev step sizes: omega_j = 1 / (j-th root of T_deg mapped to [a, b]),
// largest root first; [a, b] = [2 lo, 2] bounds the upper spectrum of D^-1 A
// (2 is the Gershgorin bound of the diagonally scaled operator).
std::vector<double> cheb_omegas(int deg, double lo) {
  const double b = 2.0, a = 2.0 * lo;
  std::vector<double> w(deg);
  for (int j = 0; j < deg; ++j) {
    const double root = 0.5 * (a + b) + 0.5 * (b - a) * std::cos(M_PI * (2.0 * j + 1.0) / (2.0 * deg));
    w[j] = 1.0 / root;
  }
  return w;
}

// Algorithmic bytes of one Jacobi step: x read (not from zero), b read, x'
// written, coarse rows once when the correction is folded in.  The
// coefficient counts 0 bytes: the method regenerates it from the draws (a
// per-call cache that a kernel reads is an implementation choice, reported
// apart from these bytes).
template <typename T>
double jac_bytes(int n, int rows, bool x_zero, bool prolong, const GridArgs&) {
  const double N = (double)rows * (double)(n - 2) * (double)(n - 2) * (double)(n - 2);
  const double e = (double)sizeof(T);
  double b = e + (x_zero ? 0.0 : e) + e;
  if (prolong) b += e / 8.0;
  return N * b;
}

// Algorithmic bytes of the fused pre-smoothing pass from x = 0: b read, x2
// written, and the residual (half: its x-restricted half, on every second
// plane) written (coefficient and reciprocal diagonal: 0 bytes).
template <typename T>
double pre2r_bytes(int n, int rows, bool half) {
  const double N = (double)rows * (double)(n - 2) * (double)(n - 2) * (double)(n - 2);
  return N * (half ? 2.5 : 3.0) * (double)sizeof(T);
}

// Algorithmic bytes of the Krylov matvec: z read (z_bytes per point), p_old
// read, p_new and q written, and x read and written when it applies the
// previous step of x (coefficient: 0 bytes).
double matvec_bytes(int n, int rows, double z_bytes, bool defer) {
  const double N = (double)rows * (double)(n - 2) * (double)(n - 2) * (double)(n - 2);
  return N * (z_bytes + 24.0 + (defer ? 16.0 : 0.0));
}

// Algorithmic bytes of the fused post-smoothing pass: x and b read, x''
// written, coarse rows read once (coefficient: 0 bytes, as above).
template <typename T>
double post2_bytes(int n, int rows, const GridArgs&) {
  const double N = (double)rows * (double)(n - 2) * (double)(n - 2) * (double)(n - 2);
  const double e = (double)sizeof(T);
  return N * (3.0 * e + e / 8.0);
}

// Symmetric V(1,1) cycle with degree-nu Chebyshev smoothing (a polynomial in
// D^-1 A, so pre- and post-smoother commute and the cycle is symmetric):
// pre-smoothing from a zero guess, residual, full weighting, coarse cycle,
// post-smoothing whose first step folds in the prolonged coarse correction
// and whose last step forms <r, z> for the problems whose top grid it is.
// The single unknown of the 3^3 grid is solved exactly by one Jacobi step.
// reciprocal diagonal of a grid size in the V-cycle's precision (null when
// the coefficient is regenerated in the sweeps)
template <typename T>
const T* dinv_of(const SizeLvl& L);
template <>
const double* dinv_of<double>(const SizeLvl& L) { return L.Di; }
template <>
const float* dinv_of<float>(const SizeLvl& L) { return L.Dif; }

//
// k0, rlim, xinit serve the full-multigrid start: the cycle then begins on
// grid size k0, covers rows 0 .. rlim-1 of every size (the problems whose top
// grid is k0 or larger), and its pre-smoothing on k0 starts from the
// prolonged current solution of size k0 + 1 instead of from zero.
template <typename T>
void vcycle_cheb(mlsgd_ctx* c, Plan* P, int k0 = 0, int rlim = INT_MAX, bool xinit = false) {
  const int S = (int)P->sizes.size();
  const int deg = c->nu;
  const std::vector<double> om = cheb_omegas(deg, c->cheb_lo);
  auto args = [&](SizeLvl& L) {
    GridArgs g = sizeof(T) == 8 ? args_size(c, P, L) : args_size32(c, P, L);
    g.rows = std::min(g.rows, rlim);
    return g;
  };
  // the levels from 9^3 down run as one LDS-resident kernel where the
  // hierarchy ends 9^3, 5^3, 3^3 with cached coefficients and every problem
  // on 5^3 and 3^3 comes down from 9^3 (none has its top grid there)
  int ks = S;
  if (c->vsmall && S >= 3 && S - 3 >= k0 && !(xinit && S - 3 == k0) && !P->ainv &&
      P->sizes[S - 3].n == 9 && P->sizes[S - 2].n == 5 &&
      P->sizes[S - 1].n == 3 && (int)om.size() <= VS_MAXDEG &&
      P->sizes[S - 2].top_begin == P->sizes[S - 2].rows &&
      P->sizes[S - 1].top_begin == P->sizes[S - 1].rows &&
      P->sizes[S - 2].rows == P->sizes[S - 3].rows) {
    const GridArgs g9 = args(P->sizes[S - 3]), g5 = args(P->sizes[S - 2]),
                   g3 = args(P->sizes[S - 1]);
    // the kernel writes a problem's <r, z> partial into its one 9^3 slot
    if (g9.cache && g5.cache && g3.cache && g9.t.tiles_per_row == 1) ks = S - 3;
  }
  for (int k = k0; k < S; ++k) {
    SizeLvl& L = P->sizes[k];
    MgView<T> v = mg_view<T>(L);
    T* A[2] = {v.X, v.R};
    GridArgs g = args(L);
    if (k == ks) {
      const GridArgs g5 = args(P->sizes[k + 1]), g3 = args(P->sizes[k + 2]);
      vcycle_small<T>(g.rows, om.data(), deg, L.top_begin, P->d_scal, v.B, g.cache, g5.cache,
                      g3.cache, g.cache_bf16, A[0], P->d_poff, P->d_partial, c->stream);
      L.cur = 0;
      break;
    }
    if (k == S - 1) {
      if (P->ainv) {
        dense_apply<T>(L.n, g.rows, P->d_scal, P->ainv, v.B, A[0], c->stream);
      } else {
        timed_launch(c, g, jac_bytes<T>(L.n, g.rows, true, false, g), [&] {
          march_jac<T>(g, nullptr, nullptr, v.B, A[0], 1, 1.0, P->d_poff, P->d_partial,
                       L.top_begin, c->stream);
        });
      }
      L.cur = 0;
      break;
    }
    int cur = 0;
    int j0 = 1;
    const T* dinv = dinv_of<T>(L);
    if (xinit && k == k0) {
      // pre-smoothing from the prolonged solution of the grid below
      SizeLvl& Lc = P->sizes[k + 1];
      const T* xc = Lc.cur ? mg_view<T>(Lc).R : mg_view<T>(Lc).X;
      if (deg == 2 && c->post2 && fused_tiles(g)) {
        // prolongation and both steps in one pass (x = 0 plus the correction)
        march_post2<T>(g, nullptr, xc, v.B, A[1], om[0], om[1], nullptr, nullptr, 0, c->stream);
        cur = 1;
      } else {
        prolong_rows<T>(Lc.n, g.rows, xc, A[0], c->stream);
        for (int j = 0; j < deg; ++j) {
          march_jac<T>(g, A[cur], nullptr, v.B, A[cur ^ 1], 0, om[j], nullptr, nullptr, 0,
                       c->stream);
          cur ^= 1;
        }
      }
      march_resid<T>(g, A[cur], v.B, A[cur ^ 1], c->stream);
      restrict_rows<T>(L.n, g.rows, 0, P->d_scal, A[cur ^ 1], mg_view<T>(P->sizes[k + 1]).B,
                       c->stream);
      L.cur = cur;
      continue;
    }
    if (deg == 2 && dinv && c->pre2r && fused_tiles(g)) {
      // both pre-smoothing steps and the residual in one pass: x2 in A[1],
      // and in A[0] r or (half) r restricted along x, then the rest of the
      // restriction
      const bool half = c->pre2r_half && pre2r_half_tiles(g);
      timed_launch(c, g, pre2r_bytes<T>(L.n, g.rows, half), [&] {
        march_pre2r<T>(g, dinv, v.B, A[1], A[0], om[0], om[1], half, c->stream);
      }, 3);
      if (half)
        restrict_yz_rows<T>(L.n, g.rows, 0, P->d_scal, A[0], mg_view<T>(P->sizes[k + 1]).B,
                            c->stream);
      else
        restrict_rows<T>(L.n, g.rows, 0, P->d_scal, A[0], mg_view<T>(P->sizes[k + 1]).B,
                         c->stream);
      L.cur = 1;
      continue;
    }
    if (deg >= 2 && dinv) {
      // steps 0 and 1 in one pass from the stored reciprocal diagonal
      march_jac2z<T>(g, dinv, v.B, A[1], om[0], om[1], c->stream);
      cur = 1;
      j0 = 2;
    } else {
      timed_launch(c, g, jac_bytes<T>(L.n, g.rows, true, false, g), [&] {
        march_jac<T>(g, nullptr, nullptr, v.B, A[0], 1, om[0], nullptr, nullptr, 0, c->stream);
      });
    }
    for (int j = j0; j < deg; ++j) {
      timed_launch(c, g, jac_bytes<T>(L.n, g.rows, false, false, g), [&] {
        march_jac<T>(g, A[cur], nullptr, v.B, A[cur ^ 1], 0, om[j], nullptr, nullptr, 0,
                     c->stream);
      });
      cur ^= 1;
    }
    march_resid<T>(g, A[cur], v.B, A[cur ^ 1], c->stream);
    restrict_rows<T>(L.n, g.rows, 0, P->d_scal, A[cur ^ 1], mg_view<T>(P->sizes[k + 1]).B,
                     c->stream);
    L.cur = cur;
  }
  // up from the level above the coarsest one handled (the small cycle's 9^3, or S - 1)
  for (int k = (ks < S ? ks : S - 1) - 1; k >= k0; --k) {
    SizeLvl& L = P->sizes[k];
    MgView<T> v = mg_view<T>(L);
    T* A[2] = {v.X, v.R};
    SizeLvl& Lc = P->sizes[k + 1];
    MgView<T> vc = mg_view<T>(Lc);
    const T* xc = Lc.cur ? vc.R : vc.X;
    GridArgs g = args(L);
    int cur = L.cur;
    int j = 0;
    if (deg >= 2 && c->post2 && fused_tiles(g)) {
      // the step with the coarse-grid correction and the next one in one pass
      timed_launch(c, g, post2_bytes<T>(L.n, g.rows, g), [&] {
        march_post2<T>(g, A[cur], xc, v.B, A[cur ^ 1], om[deg - 1], om[deg - 2],
                       deg == 2 ? P->d_poff : nullptr, deg == 2 ? P->d_partial : nullptr,
                       L.top_begin, c->stream);
      }, 2);
      cur ^= 1;
      j = 2;
    }
    for (; j < deg; ++j) {
      const bool last = j == deg - 1;
      const T* corr = j == 0 ? xc : nullptr;
      if (corr) {   // the step with the folded correction is a separate kernel; not timed
        march_jac<T>(g, A[cur], corr, v.B, A[cur ^ 1], 0, om[deg - 1 - j],
                     last ? P->d_poff : nullptr, last ? P->d_partial : nullptr, L.top_begin,
                     c->stream);
      } else {
        timed_launch(c, g, jac_bytes<T>(L.n, g.rows, false, false, g), [&] {
          march_jac<T>(g, A[cur], nullptr, v.B, A[cur ^ 1], 0, om[deg - 1 - j],
                       last ? P->d_poff : nullptr, last ? P->d_partial : nullptr, L.top_begin,
                       c->stream);
        });
      }
      cur ^= 1;
    }
    L.cur = cur;
  }
}

// Symmetric V(nu,nu) cycle with fused red-black sweeps (cached coefficient):
// pre-smoothing red-first sweeps from a zero guess, residual, full weighting,
// coarse cycle, then black-first post-smoothing sweeps whose first one folds
// the prolonged coarse correction into its loads; the last one forms <r, z>
// for the problems whose top grid it is.  Each grid alternates its iterate
// between the X and R rows; `cur` records where it ended.
template <typename T>
void vcycle_fused(mlsgd_ctx* c, Plan* P) {
  const int S = (int)P->sizes.size();
  const int nu = c->nu;
  const double om = c->omega;
  auto args = [&](SizeLvl& L) {
    return sizeof(T) == 8 ? args_size(c, P, L) : args_size32(c, P, L);
  };
  for (int k = 0; k < S; ++k) {
    SizeLvl& L = P->sizes[k];
    MgView<T> v = mg_view<T>(L);
    T* A[2] = {v.X, v.R};
    GridArgs g = args(L);
    if (k == S - 1) {
      if (P->ainv)
        dense_apply<T>(L.n, L.rows, P->d_scal, P->ainv, v.B, A[0], c->stream);
      else
        timed_sweep<T>(c, g, nullptr, nullptr, v.B, A[0], 0, 1, P->d_poff, P->d_partial,
                       L.top_begin, 1.0);
      L.cur = 0;
      break;
    }
    int cur = 0;
    timed_sweep<T>(c, g, nullptr, nullptr, v.B, A[0], 0, 1, nullptr, nullptr, 0, om);
    for (int sw = 1; sw < nu; ++sw) {
      timed_sweep<T>(c, g, A[cur], nullptr, v.B, A[cur ^ 1], 0, 0, nullptr, nullptr, 0, om);
      cur ^= 1;
    }
    march_resid<T>(g, A[cur], v.B, A[cur ^ 1], c->stream);
    restrict_rows<T>(L.n, L.rows, 0, P->d_scal, A[cur ^ 1], mg_view<T>(P->sizes[k + 1]).B,
                     c->stream);
    L.cur = cur;
  }
  for (int k = S - 2; k >= 0; --k) {
    SizeLvl& L = P->sizes[k];
    MgView<T> v = mg_view<T>(L);
    T* A[2] = {v.X, v.R};
    SizeLvl& Lc = P->sizes[k + 1];
    MgView<T> vc = mg_view<T>(Lc);
    const T* xc = Lc.cur ? vc.R : vc.X;
    GridArgs g = args(L);
    int cur = L.cur;
    for (int sw = 0; sw < nu; ++sw) {
      const bool last = sw == nu - 1;
      timed_sweep<T>(c, g, A[cur], sw == 0 ? xc : nullptr, v.B, A[cur ^ 1], 1, 0,
                     last ? P->d_poff : nullptr, last ? P->d_partial : nullptr, L.top_begin, om);
      cur ^= 1;
    }
    L.cur = cur;
  }
}

template <typename T>
void vcycle(mlsgd_ctx* c, Plan* P) {
  hipStream_t s = c->stream;
  const int S = (int)P->sizes.size();
  const int nu = c->nu;
  const double om = c->omega;
  auto args = [&](SizeLvl& L) {
    return sizeof(T) == 8 ? args_size(c, P, L) : args_size32(c, P, L);
  };
  for (int k = 0; k < S; ++k) {
    SizeLvl& L = P->sizes[k];
    MgView<T> v = mg_view<T>(L);
    GridArgs g = args(L);
    if (k == S - 1) {
      if (P->ainv) {
        dense_apply<T>(L.n, L.rows, P->d_scal, P->ainv, v.B, v.X, s);
      } else {
        timed_gs<T>(c, g, v.X, v.B, 0, 1, nullptr, nullptr, 0, 1.0);
        timed_gs<T>(c, g, v.X, v.B, 1, 0, P->d_poff, P->d_partial, L.top_begin, 1.0);
      }
      break;
    }
    for (int sw = 0; sw < nu; ++sw) {
      timed_gs<T>(c, g, v.X, v.B, 0, sw == 0 ? 1 : 0, nullptr, nullptr, 0, om);
      timed_gs<T>(c, g, v.X, v.B, 1, 0, nullptr, nullptr, 0, om);
    }
    march_resid<T>(g, v.X, v.B, v.R, s);
    restrict_rows<T>(L.n, L.rows, 0, P->d_scal, v.R, mg_view<T>(P->sizes[k + 1]).B, s);
  }
  for (int k = S - 2; k >= 0; --k) {
    SizeLvl& L = P->sizes[k];
    MgView<T> v = mg_view<T>(L);
    GridArgs g = args(L);
    prolong_add_rows<T>(P->sizes[k + 1].n, L.rows, 0, P->d_scal, mg_view<T>(P->sizes[k + 1]).X,
                        v.X, s);
    for (int sw = 0; sw < nu; ++sw) {
      const bool last = sw == nu - 1;
      timed_gs<T>(c, g, v.X, v.B, 1, 0, nullptr, nullptr, 0, om);
      timed_gs<T>(c, g, v.X, v.B, 0, 0, last ? P->d_poff : nullptr, last ? P->d_partial : nullptr,
                  L.top_begin, om);
    }
  }
}

void precondition(mlsgd_ctx* c, Plan* P) {
  const bool cached = c->mixed ? c->cache32 : c->cache64;
  // the fused red-black kernel reads a cache of the compute type only and
  // exists for tiles of 4 or 8 rows
  const int sm = (c->smoother == 1 && (!cached || c->bf16 || c->tile_y == 16)) ? 0 : c->smoother;
  if (c->mixed) {
    if (sm == 2)
      vcycle_cheb<float>(c, P);
    else if (sm == 1)
      vcycle_fused<float>(c, P);
    else
      vcycle<float>(c, P);
  } else {
    if (sm == 2)
      vcycle_cheb<double>(c, P);
    else if (sm == 1)
      vcycle_fused<double>(c, P);
    else
      vcycle<double>(c, P);
  }
}

// true when the preconditioner leaves z in X or R according to `cur`
bool out_of_place(const mlsgd_ctx* c) {
  const bool cached = c->mixed ? c->cache32 : c->cache64;
  return c->smoother == 2 || (c->smoother == 1 && cached && !c->bf16 && c->tile_y != 16);
}

// z rows of a group after the preconditioner (where the cycle left them)
const double* z64(mlsgd_ctx* c, Plan* P, const Group& gr) {
  SizeLvl& L = P->sizes[gr.sl];
  const double* A = (out_of_place(c) && L.cur) ? L.R : L.X;
  return A + (size_t)gr.p0 * srow(gr.n);
}
const float* z32(mlsgd_ctx* c, Plan* P, const Group& gr) {
  SizeLvl& L = P->sizes[gr.sl];
  const float* A = (out_of_place(c) && L.cur) ? L.Rf : L.Xf;
  return A + (size_t)gr.p0 * srow(gr.n);
}

int read_count(mlsgd_ctx* c) {
  HIPCHK(hipMemcpyAsync(c->h_count, c->d_count, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  if (c->tm.used) timing_collect(c);
  return *c->h_count;
}

// Full-multigrid start of the Krylov solves (Chebyshev cycles, hierarchies
// ending at 3^3): b restricted to every grid, the exact solve on 3^3, then on
// each larger grid the prolonged solution of the grid below improved by one
// cycle from that grid, over the problems whose top grid is that size or
// larger.  A problem's result on its top grid becomes its starting iterate x0
// (active problems; the others get x = 0, so x need not be cleared before)
// and the B rows of the top grids receive r0 = b - A x0.  bb must already
// hold |b|^2.
bool fmg_applies(mlsgd_ctx* c, Plan* P) {
  return c->fmg && c->pb.solver == MLSGD_SOLVER_MGPCG && c->smoother == 2 && !P->ainv &&
         P->sizes.size() >= 2 && P->sizes.back().n == 3;
}

template <typename T>
void fmg_start(mlsgd_ctx* c, Plan* P) {
  hipStream_t s = c->stream;
  const int S = (int)P->sizes.size();
  if (sizeof(T) == 4) {
    for (auto& gr : P->groups) {
      SizeLvl& L = P->sizes[gr.sl];
      to_f32((long long)gr.count * srow(gr.n), rows_of(L.B, gr),
             L.Bf + (size_t)gr.p0 * srow(gr.n), s);
    }
  }
  for (int k = 0; k + 1 < S; ++k) {
    SizeLvl& L = P->sizes[k];
    restrict_rows<T>(L.n, L.rows, 0, nullptr, mg_view<T>(L).B, mg_view<T>(P->sizes[k + 1]).B, s);
  }
  {
    SizeLvl& L = P->sizes[S - 1];
    GridArgs g = sizeof(T) == 8 ? args_size(c, P, L) : args_size32(c, P, L);
    march_jac<T>(g, nullptr, nullptr, mg_view<T>(L).B, mg_view<T>(L).X, 1, 1.0, nullptr, nullptr,
                 0, s);
    L.cur = 0;
    for (auto& gr : P->groups)
      if (gr.sl == S - 1)
        copy_active_rows<T>(gr.n, gr.count, gr.p0, P->d_scal,
                            mg_view<T>(L).X + (size_t)gr.p0 * srow(gr.n), gr.x, s);
  }
  for (int k = S - 2; k >= 0; --k) {
    SizeLvl& L = P->sizes[k];
    vcycle_cheb<T>(c, P, k, L.rows, true);
    const T* xk = L.cur ? mg_view<T>(L).R : mg_view<T>(L).X;
    for (auto& gr : P->groups)
      if (gr.sl == k)
        copy_active_rows<T>(gr.n, gr.count, gr.p0, P->d_scal, xk + (size_t)gr.p0 * srow(gr.n),
                            gr.x, s);
  }
  for (auto& gr : P->groups) {
    GridArgs g = args_group(c, P, gr, false);
    march_resid<double>(g, gr.x, gr.b0, rows_of(P->sizes[gr.sl].B, gr), s);
  }
  HIPCHK(hipGetLastError());
}

void fmg(mlsgd_ctx* c, Plan* P) {
  if (!fmg_applies(c, P)) return;
  if (c->mixed)
    fmg_start<float>(c, P);
  else
    fmg_start<double>(c, P);
}

// One Krylov step of every active problem after z = M r: p = z + beta p,
// q = A p and alpha, then r -= alpha q with <r, r>.  With xdefer the step
// x += alpha p is applied by the next iteration's matvec, which reads that p
// anyway (8 B per point less than updating x here); the step of a problem's
// last iteration stays pending in its scalars, with the direction buffer
// that holds its p, until flush_steps.  Every iterate is the same in both
// modes: the same x + alpha p is formed, one pass later.
void krylov_step(mlsgd_ctx* c, Plan* P, bool mg, int it) {
  hipStream_t s = c->stream;
  const double rtol = c->pb.rtol;
  const int maxit = c->pb.max_iters;
  const bool defer = c->xdefer;
  int pslot = 0;  // every group writes the new direction into p[pcur ^ 1]
  for (auto& gr : P->groups) {
    GridArgs g = args_group(c, P, gr, true);
    SizeLvl& L = P->sizes[gr.sl];
    double* xd = (defer && it > 0) ? gr.x : nullptr;
    const bool z32b = mg && c->mixed;
    timed_launch(c, g, matvec_bytes(gr.n, gr.count, z32b ? 4.0 : 8.0, xd != nullptr), [&] {
      if (z32b) {
        march_matvec<double, float>(g, z32(c, P, gr), gr.p[gr.pcur], gr.p[gr.pcur ^ 1], gr.q,
                                    P->d_poff, P->d_partial, s, xd);
      } else {
        const double* z = mg ? z64(c, P, gr) : rows_of(L.B, gr);
        march_matvec<double, double>(g, z, gr.p[gr.pcur], gr.p[gr.pcur ^ 1], gr.q, P->d_poff,
                                     P->d_partial, s, xd);
      }
    }, 4);
    pslot = gr.pcur ^ 1;
  }
  cg_scalar(PH_ALPHA, P->d_scal, P->nprob, P->d_poff, P->d_pcnt, P->d_partial, rtol, maxit,
            nullptr, s, pslot);
  for (auto& gr : P->groups) {
    GridArgs g = args_group(c, P, gr, true);
    float* r32 = (mg && c->mixed) ? P->sizes[gr.sl].Bf + (size_t)gr.p0 * srow(gr.n) : nullptr;
    if (defer)
      group_rupdate(g, rows_of(P->sizes[gr.sl].B, gr), gr.q, P->d_poff, P->d_partial, r32, s);
    else
      group_update(g, gr.x, gr.p[gr.pcur ^ 1], rows_of(P->sizes[gr.sl].B, gr), gr.q,
                   P->d_poff, P->d_partial, r32, s);
    gr.pcur ^= 1;
  }
}

// Apply every pending step x += alpha p (active problems and those that
// converged earlier alike) before x is read.
void flush_steps(mlsgd_ctx* c, Plan* P) {
  if (!c->xdefer) return;
  for (auto& gr : P->groups) {
    GridArgs g = args_group(c, P, gr, true);
    group_xflush(g, gr.x, gr.p[0], gr.p[1], c->stream);
  }
}

// Batched (preconditioned) CG on every problem of the plan.  On entry the
// B rows of each top grid hold the right-hand side b, b0 a copy of it, x = 0.
void krylov(mlsgd_ctx* c, Plan* P, int* iters_out, int* nonconv_out, double* relres_out,
            bool bb_ready = false) {
  hipStream_t s = c->stream;
  const bool mg = c->pb.solver == MLSGD_SOLVER_MGPCG;
  const double rtol = c->pb.rtol;
  const int maxit = c->pb.max_iters;
  if (!bb_ready) {
    for (auto& gr : P->groups) {
      GridArgs g = args_group(c, P, gr, false);
      double* r = rows_of(P->sizes[gr.sl].B, gr);
      group_dot(g, r, r, P->d_poff, P->d_partial, s);
    }
  }
  cg_scalar(PH_INIT_BB, P->d_scal, P->nprob, P->d_poff, P->d_pcnt, P->d_partial, rtol, maxit,
            nullptr, s);
  fmg(c, P);
  // after a full-multigrid start r0 carries the evaluation error of b - A x0
  // (near the FP64 residual floor, about 0.3 rtol on 129^3 grids), which the
  // recursion keeps; a recursive target of 0.7 rtol leaves room for it, so the
  // true-residual check at exit (still against rtol) rarely has to restart a
  // solve
  const double rtol_rr = fmg_applies(c, P) ? c->fmg_margin * rtol : rtol;
  for (int restart = 0; restart < 3; ++restart) {
    if (mg && c->mixed) {
      for (auto& gr : P->groups) {
        SizeLvl& L = P->sizes[gr.sl];
        to_f32((long long)gr.count * srow(gr.n), rows_of(L.B, gr),
               L.Bf + (size_t)gr.p0 * srow(gr.n), s);
      }
    }
    if (mg) {
      precondition(c, P);
      cg_scalar(PH_RZ0, P->d_scal, P->nprob, P->d_poff, P->d_pcnt, P->d_partial, rtol, maxit,
                nullptr, s);
    } else {
      cg_scalar(PH_RZ0_RR, P->d_scal, P->nprob, P->d_poff, P->d_pcnt, nullptr, rtol, maxit,
                nullptr, s);
    }
    // the first quiet iterations run without a host read of the active
    // count: a problem that converged there is inactive and skipped, so at
    // worst a few launches run empty
    const int quiet = restart == 0 ? c->kry_quiet : 0;
    for (int it = 0; it < maxit; ++it) {
      krylov_step(c, P, mg, it);
      const bool read = it + 1 > quiet;
      cg_scalar(PH_RR, P->d_scal, P->nprob, P->d_poff, P->d_pcnt, P->d_partial, rtol_rr, maxit,
                read ? c->d_count : nullptr, s);
      HIPCHK(hipGetLastError());
      if (read && read_count(c) == 0) break;
      if (mg) {
        precondition(c, P);
        cg_scalar(PH_RZ, P->d_scal, P->nprob, P->d_poff, P->d_pcnt, P->d_partial, rtol, maxit,
                  nullptr, s);
      } else {
        cg_scalar(PH_RZ_RR, P->d_scal, P->nprob, P->d_poff, P->d_pcnt, nullptr, rtol, maxit,
                  nullptr, s);
      }
    }
    // the norm of the true residual b0 - A x (not stored); restart the
    // problems that drifted.  After a restart only the restarted problems are
    // checked again: the others were not touched, and their partial slots
    // still hold the last check's sums
    flush_steps(c, P);
    if (restart > 0)
      cg_scalar(PH_RECHECK, P->d_scal, P->nprob, P->d_poff, P->d_pcnt, nullptr, rtol, maxit,
                nullptr, s);
    for (auto& gr : P->groups)
      march_resid_norm(args_group(c, P, gr, restart > 0), gr.x, gr.b0, P->d_poff, P->d_partial,
                       s);
    const bool force = c->force_restart && restart == 0;
    cg_scalar(PH_TRUE, P->d_scal, P->nprob, P->d_poff, P->d_pcnt, P->d_partial, rtol, maxit,
              force ? nullptr : c->d_count, s);
    if (force)
      cg_scalar(PH_FORCE_RESTART, P->d_scal, P->nprob, P->d_poff, P->d_pcnt, nullptr, rtol, maxit,
                c->d_count, s);
    HIPCHK(hipGetLastError());
    if (read_count(c) == 0) break;
    // the restarted problems start again from r = b - A x
    for (auto& gr : P->groups)
      march_resid<double>(args_group(c, P, gr, true), gr.x, gr.b0,
                          rows_of(P->sizes[gr.sl].B, gr), s);
  }
  scal_to_stats(P->d_scal, P->nprob, rtol, &c->d_stat->iters, &c->d_stat->nonconv,
                &c->d_stat->relres, s);
  HIPCHK(hipMemcpyAsync(c->h_stat, c->d_stat, sizeof(mlsgd_ctx::StatDev), hipMemcpyDeviceToHost,
                        s));
  HIPCHK(hipStreamSynchronize(s));
  *iters_out = c->h_stat->iters;
  *nonconv_out = c->h_stat->nonconv;
  *relres_out = c->h_stat->relres;
  c->kry_quiet = std::max(0, std::min(*iters_out, maxit) - 2);
}

// The same batched PCG with a fixed iteration count and no host reads, so it
// can be captured in a graph: `iters` iterations, the true-residual check,
// one restart block of up to kRestartIters iterations for the problems
// whose true residual drifted, the check again, and the per-problem
// statistics into d_stat[slot].  Converged problems are inactive, so the
// iterations beyond their convergence only launch early-exiting kernels.
constexpr int kRestartIters = 2;

void krylov_fixed(mlsgd_ctx* c, Plan* P, int iters, int slot, bool bb_ready = false) {
  hipStream_t s = c->stream;
  const bool mg = c->pb.solver == MLSGD_SOLVER_MGPCG;
  const double rtol = c->pb.rtol;
  const int maxit = c->pb.max_iters;
  // the host reads no count here (the stats kernel reports the outcome)
  auto cg = [&](int phase, const double* partial) {
    cg_scalar(phase, P->d_scal, P->nprob, P->d_poff, P->d_pcnt, partial, rtol, maxit, nullptr, s);
  };
  auto start = [&]() {  // z = M r and rz for the active problems
    if (mg && c->mixed) {
      for (auto& gr : P->groups) {
        SizeLvl& L = P->sizes[gr.sl];
        to_f32((long long)gr.count * srow(gr.n), rows_of(L.B, gr),
               L.Bf + (size_t)gr.p0 * srow(gr.n), s);
      }
    }
    if (mg) {
      precondition(c, P);
      cg(PH_RZ0, P->d_partial);
    } else {
      cg(PH_RZ0_RR, nullptr);
    }
  };
  auto iterate = [&](int count) {
    for (int it = 0; it < count; ++it) {
      krylov_step(c, P, mg, it);
      cg_scalar(PH_RR, P->d_scal, P->nprob, P->d_poff, P->d_pcnt, P->d_partial,
                fmg_applies(c, P) ? c->fmg_margin * rtol : rtol, maxit, nullptr, s);
      if (mg) {
        precondition(c, P);
        cg(PH_RZ, P->d_partial);
      } else {
        cg(PH_RZ_RR, nullptr);
      }
    }
  };
  // the true residual of every problem, or (recheck) of the problems the last
  // check restarted: the others were not touched since, and their partial
  // slots still hold that check's sums, so PH_TRUE keeps their verdict
  auto true_residual = [&](bool recheck) {
    flush_steps(c, P);
    if (recheck) cg(PH_RECHECK, nullptr);
    for (auto& gr : P->groups)
      march_resid_norm(args_group(c, P, gr, recheck), gr.x, gr.b0, P->d_poff, P->d_partial, s);
    cg(PH_TRUE, P->d_partial);
  };
  if (!bb_ready) {
    for (auto& gr : P->groups) {
      GridArgs g = args_group(c, P, gr, false);
      double* r = rows_of(P->sizes[gr.sl].B, gr);
      group_dot(g, r, r, P->d_poff, P->d_partial, s);
    }
  }
  cg(PH_INIT_BB, P->d_partial);
  fmg(c, P);
  start();
  iterate(iters);
  true_residual(false);
  if (c->force_restart) cg(PH_FORCE_RESTART, nullptr);
  // restart block: the problems that missed rtol start again from b - A x
  for (auto& gr : P->groups)
    march_resid<double>(args_group(c, P, gr, true), gr.x, gr.b0, rows_of(P->sizes[gr.sl].B, gr),
                        s);
  start();
  iterate(kRestartIters);
  true_residual(true);
  scal_to_stats(P->d_scal, P->nprob, rtol, &c->d_stat[slot].iters, &c->d_stat[slot].nonconv,
                &c->d_stat[slot].relres, s);
  HIPCHK(hipGetLastError());
}

// Right-hand sides R^(finest -> n)(f + u) on every level grid.
void level_rhs(mlsgd_ctx* c, const double* u) {
  const int L = c->pb.n_levels;
  const int nf = c->nfin;
  add_mask(nf, c->d_f, u, c->rhs_lvl[nf], c->stream);
  for (int i = L - 2; i >= 0; --i) {
    const int n = c->pb.grid_n[i];
    restrict_full(c->pb.grid_n[i + 1], c->rhs_lvl[c->pb.grid_n[i + 1]], c->rhs_lvl[n], c->stream);
  }
  HIPCHK(hipGetLastError());
}

// State solves of every problem, then misfits Phi and the adjoint right-hand
// sides y - y_d in the B rows (x reset to 0).
void state_phase(mlsgd_ctx* c, Plan* P, int* it, int* nc, double* rr, double* y_out,
                 int fixed = 0) {
  hipStream_t s = c->stream;
  // x starts at 0 (the full-multigrid start writes every x row itself).
  // Every problem of a group has the same right-hand side, so |b|^2 is
  // summed over the group's first row and its partial slots copied to the
  // others.
  const bool clear = !fmg_applies(c, P);
  for (auto& gr : P->groups) {
    double* b = rows_of(P->sizes[gr.sl].B, gr);
    rows_broadcast(gr.n, gr.count, c->rhs_lvl[gr.n], b, s);
    rows_broadcast(gr.n, gr.count, c->rhs_lvl[gr.n], gr.b0, s);
    if (clear) rows_zero((long long)gr.count * srow(gr.n), gr.x, s);
    GridArgs g1 = args_group(c, P, gr, false);
    g1.rows = 1;
    group_dot(g1, b, b, P->d_poff, P->d_partial, s);
    replicate_slots(gr.p0, gr.count, P->h_pcnt[gr.p0], P->d_poff, P->d_partial, s);
  }
  HIPCHK(hipGetLastError());
  if (fixed > 0)
    krylov_fixed(c, P, fixed, 0, true);
  else
    krylov(c, P, it, nc, rr, true);
  for (auto& gr : P->groups) {
    if (y_out) unpack_rows(gr.n, gr.count, gr.x, y_out, s);
    GridArgs g = args_group(c, P, gr, false);
    double* b = rows_of(P->sizes[gr.sl].B, gr);
    group_misfit(g, gr.x, c->yd_lvl[gr.n], b, P->d_poff, P->d_partial, s);
    copy_rows(gr.n, gr.count, b, gr.b0, s);
    const double h = 1.0 / (double)(gr.n - 1);
    sum_partials(gr.count, P->d_poff + gr.p0, P->d_pcnt + gr.p0, P->d_partial, 0.5 * h * h * h,
                 P->d_phi + gr.p0, s);
  }
  HIPCHK(hipGetLastError());
}

void check_u(mlsgd_ctx* c, const double* u) {
  require(u != nullptr, "u_fine is null");
  HIPCHK(hipMemsetAsync(c->d_flag, 0, sizeof(int), c->stream));
  nonfinite_flag((long long)cube(c->nfin), u, c->d_flag, c->stream);
  HIPCHK(hipMemcpyAsync(c->h_count, c->d_flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  if (*c->h_count) throw Fail{MLSGD_ENONFINITE, "u_fine holds NaN or Inf"};
}

// Problem blocks of an MLMC estimate over levels 0..L-1, grouped by grid:
// grid n_i holds the fine solves of level i, then the coarse solves of
// level i+1 (both keyed by their own level's draws).
std::vector<Block> mlmc_blocks(mlsgd_ctx* c, int L, const int64_t* M, const int64_t* first) {
  std::vector<Block> b;
  for (int i = L - 1; i >= 0; --i) {
    b.push_back(Block{c->pb.grid_n[i], i, first ? first[i] : 0, M[i]});
    if (i + 1 <= L - 1) b.push_back(Block{c->pb.grid_n[i], i + 1, first ? first[i + 1] : 0, M[i + 1]});
  }
  return b;
}

struct LevelRows {
  int fine_prob, coarse_prob;   // problem index of the first fine / coarse problem
  const Group* gf;
  const Group* gc;
  int fine_row, coarse_row;     // row within the group
};

std::vector<LevelRows> level_rows(Plan* P, mlsgd_ctx* c, int L, const int64_t* M) {
  std::vector<LevelRows> out(L);
  // blocks are: for i = L-1..0: [fine i][coarse i+1]
  int p = 0;
  std::vector<int> fine_p(L), coarse_p(L, -1);
  for (int i = L - 1; i >= 0; --i) {
    fine_p[i] = p;
    p += (int)M[i];
    if (i + 1 <= L - 1) {
      coarse_p[i + 1] = p;
      p += (int)M[i + 1];
    }
  }
  for (int i = 0; i < L; ++i) {
    LevelRows lr;
    lr.fine_prob = fine_p[i];
    lr.coarse_prob = coarse_p[i];
    lr.gf = lr.gc = nullptr;
    lr.fine_row = lr.coarse_row = 0;
    for (const auto& g : P->groups) {
      if (g.n == c->pb.grid_n[i]) {
        lr.gf = &g;
        lr.fine_row = fine_p[i] - g.p0;
      }
      if (i > 0 && g.n == c->pb.grid_n[i - 1]) {
        lr.gc = &g;
        lr.coarse_row = coarse_p[i] - g.p0;
      }
    }
    out[i] = lr;
  }
  return out;
}

// Epilogue buffers grow to the largest estimate seen (the old buffer is
// freed; captured graphs that point into it are dropped).
void ensure_epi(mlsgd_ctx* c, size_t part_len, size_t dx_len) {
  if (part_len > c->epi_part_len) {
    drop_graphs(c);
    dfree(c, c->d_epi_part);
    c->d_epi_part = (double*)dalloc(c, sizeof(double) * part_len);
    c->epi_part_len = part_len;
  }
  if (dx_len > c->dxpart_len) {
    drop_graphs(c);
    dfree(c, c->d_dxpart);
    c->d_dxpart = (double*)dalloc(c, sizeof(double) * dx_len);
    c->dxpart_len = dx_len;
  }
}

// One estimate (gradient or objective only).
// Host side of one estimate: plan and draws, epilogue metadata and buffers.
struct EstPrep {
  Plan* P = nullptr;
  std::vector<LevelRows> lr;
  std::vector<EpiLevel> ev;
  long long g_off = 0;
};

EstPrep estimate_prep(mlsgd_ctx* c, int L, const int64_t* M, const int64_t* first,
                      bool fields) {
  EstPrep e;
  e.P = get_plan(c, mlmc_blocks(c, L, M, first), fields);
  e.lr = level_rows(e.P, c, L, M);
  e.ev.resize(L);
  size_t part_len = RED_BLOCKS, dx_len = 0;
  for (int i = 0; i < L; ++i) {
    const int nf = c->pb.grid_n[i];
    e.ev[i].M = (int)M[i];
    e.ev[i].fine_off = e.lr[i].fine_prob;
    e.ev[i].coarse_off = e.lr[i].coarse_prob;
    e.ev[i].nf = nf;
    e.ev[i].m2_off = (long long)part_len;
    e.ev[i].m2_cnt = level_sample_blocks((int)M[i]) * level_m2_chunks(nf);
    part_len += e.ev[i].m2_cnt;
    e.ev[i].nm_off = (long long)part_len;
    part_len += RED_BLOCKS;
    dx_len = std::max(dx_len, (size_t)level_sample_blocks((int)M[i]) * cube(nf));
  }
  e.g_off = (long long)part_len;
  part_len += RED_BLOCKS;
  ensure_epi(c, part_len, dx_len);
  HIPCHK(hipMemcpyAsync(c->d_epi_lev, e.ev.data(), sizeof(EpiLevel) * L, hipMemcpyHostToDevice,
                        c->stream));
  return e;
}

// Device side of one estimate on c->stream.  fixed_s > 0 (graph mode): the
// coefficient fields are regenerated here, the solves run fixed iteration
// counts and nothing is read back, so the whole sequence is kernels only.
void estimate_enqueue(mlsgd_ctx* c, const EstPrep& e, int L, const int64_t* M, const double* u,
                      double* grad_out, int fixed_s, int fixed_a, int* it_s, int* nc_s,
                      double* rr_s, int* it_a, int* nc_a, double* rr_a) {
  hipStream_t s = c->stream;
  Plan* P = e.P;
  level_rhs(c, u);
  if (fixed_s > 0) plan_fields(c, P);
  level_work_zero(c->d_epi_out, s);
  auto add_work = [&]() {   // the iterations of the solves just finished, per level
    for (const auto& gr : P->groups)
      level_work_add(gr.count, gr.n, P->d_level + gr.p0, P->d_scal + gr.p0, c->d_epi_out, s);
  };
  state_phase(c, P, it_s, nc_s, rr_s, nullptr, fixed_s);
  add_work();
  if (grad_out) {   // the misfit pass left |y - y_d|^2 in the partial slots
    if (fixed_a > 0)
      krylov_fixed(c, P, fixed_a, 1, true);
    else
      krylov(c, P, it_a, nc_a, rr_a, true);
    add_work();
  }
  if (fixed_s <= 0) HIPCHK(hipEventRecord(c->ev[1], s));
  shift_weights(P->nprob, P->d_phi, c->pb.theta, P->d_w, &c->d_epi_out->s, s);
  add_mask(c->nfin, nullptr, u, c->d_umask, s);
  dot_blocks((long long)cube(c->nfin), c->d_umask, c->d_umask, c->d_epi_part, s);
  if (grad_out) {
    for (int i = 0; i < L; ++i) {
      const int nf = c->pb.grid_n[i];
      const double* pf = e.lr[i].gf->x + (size_t)e.lr[i].fine_row * srow(nf);
      const double* wf = P->d_w + e.lr[i].fine_prob;
      const double* pc = nullptr;
      const double* wc = nullptr;
      if (i > 0) {
        pc = e.lr[i].gc->x + (size_t)e.lr[i].coarse_row * srow(c->pb.grid_n[i - 1]);
        wc = P->d_w + e.lr[i].coarse_prob;
      }
      double* mean = c->mean_lvl[nf];
      level_dx_partial(nf, (int)M[i], pf, wf, pc, wc, c->d_dxpart, s);
      level_dx_mean(nf, (int)M[i], c->d_dxpart, mean, s);
      level_dx_m2(nf, (int)M[i], pf, wf, pc, wc, mean, c->d_epi_part + e.ev[i].m2_off, s);
      dot_blocks((long long)cube(nf), mean, mean, c->d_epi_part + e.ev[i].nm_off, s);
    }
  }
  // the fine-grid misfit scale is the one of the level's own grid; u norm on the finest grid
  epilogue_scalars(L, c->d_epi_lev, P->d_phi, P->d_w, c->d_epi_part, 0, c->nfin, c->pb.theta,
                   c->pb.alpha, grad_out ? 1 : 0, c->d_epi_out, s);
  if (grad_out) {
    // telescoping: acc_i = P acc_{i-1} + E_i[dX], then up to the finest grid
    const double* acc = c->mean_lvl[c->pb.grid_n[0]];
    for (int i = 1; i < c->pb.n_levels; ++i) {
      const int n = c->pb.grid_n[i];
      double* dst = c->acc_lvl[n];
      prolong_full(c->pb.grid_n[i - 1], acc, dst, s);
      if (i < L) axpy_full(n, 1.0, c->mean_lvl[n], dst, s);
      acc = dst;
    }
    dot_blocks((long long)cube(c->nfin), acc, acc, c->d_epi_part + e.g_off, s);
    finish_norm(c->nfin, c->d_epi_part + e.g_off, &c->d_epi_out->exnorm2, s);
    final_grad(c->nfin, acc, u, c->d_epi_out, c->pb.alpha, grad_out, s);
    dot_blocks((long long)cube(c->nfin), grad_out, grad_out, c->d_epi_part + e.g_off, s);
    finish_norm(c->nfin, c->d_epi_part + e.g_off, &c->d_epi_out->gnorm2, s);
  }
  HIPCHK(hipGetLastError());
}

void validate_batch(mlsgd_ctx* c, int L, const int64_t* M, const int64_t* first) {
  require(L >= 1 && L <= c->pb.n_levels, "L out of range");
  require(M != nullptr, "M is null");
  for (int i = 0; i < L; ++i) {
    require(M[i] >= 1, "sample counts must be >= 1");
    if (first) require(first[i] >= 0, "sample offsets must be >= 0");
  }
}

// Statistics of a finished estimate from the epilogue record.
int finish_stats(mlsgd_ctx* c, int L, const int64_t* M, bool grad, double* J_out,
                 mlsgd_grad_stats* st, int it_s, int it_a, int nc, double rr) {
  const EpiOut& eo = *c->h_epi_out;
  if (J_out) *J_out = eo.J;
  if (st) {
    std::memset(st, 0, sizeof(*st));
    st->s = eo.s;
    st->EY_shifted = eo.EY;
    st->J = eo.J;
    st->truncated = eo.truncated;
    st->iters_state = it_s;
    st->iters_adjoint = it_a;
    st->nonconverged = nc;
    st->max_relres = rr;
    for (int i = 0; i < L; ++i) {
      st->mean_dY[i] = eo.mean_dY[i];
      st->norm2_mean_dX[i] = eo.norm2_mean_dX[i];
      st->m2_dX[i] = eo.m2_dX[i];
      st->m2_dY[i] = eo.m2_dY[i];
      st->mean_phi_f[i] = eo.mean_phi_f[i];
    }
    for (int i = 0; i < L; ++i) st->work_per_sample[i] = (double)eo.work[i] / (double)M[i];
    st->grad_norm = grad ? std::sqrt(eo.gnorm2) : 0.0;
    st->norm2_EX = grad ? eo.exnorm2 : 0.0;
    float ms1 = 0, ms2 = 0;
    HIPCHK(hipEventElapsedTime(&ms1, c->ev[0], c->ev[1]));
    HIPCHK(hipEventElapsedTime(&ms2, c->ev[0], c->ev[2]));
    st->ms_solve = ms1;
    st->ms_total = ms2;
  }
  if (!std::isfinite(eo.J)) throw Fail{MLSGD_ENONFINITE, "non-finite objective"};
  if (nc > 0) {
    c->err = "some solves missed rtol";
    return MLSGD_ENOCONV;
  }
  return MLSGD_OK;
}

int run_estimate_eager(mlsgd_ctx* c, const double* u, int L, const int64_t* M,
                       const int64_t* first, double* grad_out, double* J_out,
                       mlsgd_grad_stats* st) {
  validate_batch(c, L, M, first);
  check_u(c, u);
  hipStream_t s = c->stream;
  HIPCHK(hipEventRecord(c->ev[0], s));
  EstPrep e = estimate_prep(c, L, M, first, true);
  int it_s = 0, nc_s = 0, it_a = 0, nc_a = 0;
  double rr_s = 0, rr_a = 0;
  estimate_enqueue(c, e, L, M, u, grad_out, 0, 0, &it_s, &nc_s, &rr_s, &it_a, &nc_a, &rr_a);
  HIPCHK(hipEventRecord(c->ev[2], s));
  HIPCHK(hipMemcpyAsync(c->h_epi_out, c->d_epi_out, sizeof(EpiOut), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return finish_stats(c, L, M, grad_out != nullptr, J_out, st, it_s, it_a, nc_s + nc_a,
                      std::max(rr_s, rr_a));
}

void drop_graphs(mlsgd_ctx* c) {
  for (auto& kv : c->graphs)
    if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
  c->graphs.clear();
}

// Graph mode: the first call of a batch shape runs eagerly and learns the
// iteration counts; the shape is then captured once (fixed counts plus a
// margin) and every later call uploads its draws and u and replays it.  A
// replay whose solves miss rtol is redone eagerly and the shape is captured
// again with a larger margin.
int run_estimate_graph(mlsgd_ctx* c, const double* u, int L, const int64_t* M,
                       const int64_t* first, double* grad_out, double* J_out,
                       mlsgd_grad_stats* st) {
  validate_batch(c, L, M, first);
  std::string key = std::to_string(L) + (grad_out ? "g|" : "j|");
  for (int i = 0; i < L; ++i) key += std::to_string(M[i]) + ",";
  auto it = c->graphs.find(key);
  if (it == c->graphs.end() || !it->second.exec) {
    const int margin = it == c->graphs.end() ? 1 : it->second.margin;
    mlsgd_grad_stats loc{};
    const int rc = run_estimate_eager(c, u, L, M, first, grad_out, J_out, &loc);
    if (st) *st = loc;
    if (rc != MLSGD_OK) return rc;
    mlsgd_ctx::GraphEntry ge;
    ge.margin = margin;
    ge.it_s = loc.iters_state + margin;
    ge.it_a = grad_out ? loc.iters_adjoint + margin : 0;
    EstPrep e = estimate_prep(c, L, M, first, false);
    hipStream_t saved = c->stream;
    HIPCHK(hipStreamSynchronize(saved));
    c->stream = c->cap_stream;
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeRelaxed));
    try {
      int d0 = 0, d1 = 0, d2 = 0, d3 = 0;
      double r0 = 0, r1 = 0;
      estimate_enqueue(c, e, L, M, c->d_u_graph, grad_out ? c->d_g_graph : nullptr, ge.it_s,
                       std::max(ge.it_a, 1), &d0, &d1, &r0, &d2, &d3, &r1);
    } catch (...) {
      (void)hipStreamEndCapture(c->cap_stream, &g);
      if (g) (void)hipGraphDestroy(g);
      c->stream = saved;
      throw;
    }
    const hipError_t ec = hipStreamEndCapture(c->cap_stream, &g);
    c->stream = saved;
    if (ec != hipSuccess) throw Fail{MLSGD_EHIP, std::string("graph capture: ") + hipGetErrorString(ec)};
    const hipError_t ei = hipGraphInstantiate(&ge.exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess)
      throw Fail{MLSGD_EHIP, std::string("graph instantiate: ") + hipGetErrorString(ei)};
    c->graphs[key] = ge;
    return rc;
  }
  check_u(c, u);
  hipStream_t s = c->stream;
  // upload this call's draws; a plan or buffer change drops the graphs, and
  // the shape then runs eagerly and is captured again
  (void)estimate_prep(c, L, M, first, false);
  it = c->graphs.find(key);
  if (it == c->graphs.end() || !it->second.exec)
    return run_estimate_eager(c, u, L, M, first, grad_out, J_out, st);
  mlsgd_ctx::GraphEntry& ge = it->second;
  HIPCHK(hipMemcpyAsync(c->d_u_graph, u, sizeof(double) * cube(c->nfin), hipMemcpyDeviceToDevice,
                        s));
  HIPCHK(hipEventRecord(c->ev[0], s));
  HIPCHK(hipGraphLaunch(ge.exec, s));
  HIPCHK(hipEventRecord(c->ev[1], s));
  HIPCHK(hipEventRecord(c->ev[2], s));
  HIPCHK(hipMemcpyAsync(c->h_epi_out, c->d_epi_out, sizeof(EpiOut), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(c->h_stat, c->d_stat, 2 * sizeof(mlsgd_ctx::StatDev),
                        hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const mlsgd_ctx::StatDev st_s = c->h_stat[0], st_a = c->h_stat[1];
  const int nc = st_s.nonconv + (grad_out ? st_a.nonconv : 0);
  if (nc > 0) {  // the learned counts were too small for these draws
    HIPCHK(hipGraphExecDestroy(ge.exec));
    ge.exec = nullptr;
    ge.margin += 1;
    return run_estimate_eager(c, u, L, M, first, grad_out, J_out, st);
  }
  if (grad_out)
    HIPCHK(hipMemcpyAsync(grad_out, c->d_g_graph, sizeof(double) * cube(c->nfin),
                          hipMemcpyDeviceToDevice, s));
  const double rr = std::max(st_s.relres, grad_out ? st_a.relres : 0.0);
  return finish_stats(c, L, M, grad_out != nullptr, J_out, st, st_s.iters,
                      grad_out ? st_a.iters : 0, 0, rr);
}

int run_estimate(mlsgd_ctx* c, const double* u, int L, const int64_t* M, const int64_t* first,
                 double* grad_out, double* J_out, mlsgd_grad_stats* st) {
  if (c->graph && !c->tm.on) return run_estimate_graph(c, u, L, M, first, grad_out, J_out, st);
  return run_estimate_eager(c, u, L, M, first, grad_out, J_out, st);
}

// Adaptive controller (Sec. 4.1): second-order power sums v^2 per level,
// optimal batch sizes for a sampling error eps^2/2, sampling-error estimate,
// squared-bias estimate and the level update.  Units: the paper's unshifted
// X, Y (statistics are rescaled by e^{theta s}).  Costs: the measured work
// per sample of each level in the estimate just made (interior unknowns x
// Krylov iterations over its state and adjoint solves, fine and coarse), an
// exact integer count, so the batch sequence is reproducible.  eps = 0.9 |g|
// of the gradient just computed.
// Every level's batch, an added level's included, is capped at the samples
// whose solver arrays (14 arrays of n^3 doubles each) fit 32 GiB.
struct CtrlOut {
  int64_t M[MLSGD_MAX_LEVELS];
  int L;
  double err_sam, err_num, eps, alpha_hat;
};

// Largest batch of one level on an n^3 grid (at least 2).
int64_t batch_cap(int n) {
  const double per_sample = 14.0 * 8.0 * (double)n * n * n;
  return std::max<int64_t>(2, (int64_t)std::floor(32.0 * (double)(1ull << 30) / per_sample));
}

CtrlOut controller(const mlsgd_ctx* c, const mlsgd_grad_stats& g, int L, const int64_t* M) {
  CtrlOut o{};
  const double th = c->pb.theta;
  const double sc = std::exp(th * g.s);
  const double Chat = g.norm2_EX / (g.EY_shifted * g.EY_shifted);  // the shift cancels
  double v2[MLSGD_MAX_LEVELS], C[MLSGD_MAX_LEVELS];
  for (int i = 0; i < L; ++i) {
    v2[i] = (g.m2_dX[i] + Chat * g.m2_dY[i]) * sc * sc;
    // cost per sample: the estimate's measured work on the level (interior
    // unknowns x Krylov iterations of its fine and coarse, state and adjoint
    // solves); the unknown count where no work was recorded
    const double nf = (double)(c->pb.grid_n[i] - 2);
    const double ncs = i > 0 ? (double)(c->pb.grid_n[i - 1] - 2) : 0.0;
    C[i] = g.work_per_sample[i] > 0.0 ? g.work_per_sample[i] : nf * nf * nf + ncs * ncs * ncs;
  }
  const double eps = 0.9 * g.grad_norm;
  o.eps = eps;
  double sum = 0.0;
  for (int i = 0; i < L; ++i)
    sum += std::sqrt(v2[i] * C[i] / (double)std::max<int64_t>(M[i] - 1, 1));
  double err_sam = 0.0;
  for (int i = 0; i < L; ++i) {
    const double Mi = (double)M[i];
    err_sam += v2[i] / (Mi * std::max(Mi - 1.0, 1.0));
    double mo = (2.0 / (eps * eps)) *
                std::sqrt(v2[i] / ((double)std::max<int64_t>(M[i] - 1, 1) * C[i])) * sum;
    const double mmax = (double)batch_cap(c->pb.grid_n[i]);
    if (!std::isfinite(mo) || mo > mmax) mo = mmax;
    o.M[i] = std::max<int64_t>(2, (int64_t)std::ceil(mo));
  }
  o.err_sam = err_sam;
  // alpha_hat: least-squares slope of log2 sqrt(|E dX_i|^2 + C_hat |E dY_i|^2)
  // over levels 1..L-1 (fallback 2)
  double ahat = 2.0;
  {
    double sx = 0, sy = 0, sxx = 0, sxy = 0;
    int cnt = 0;
    for (int i = 1; i < L; ++i) {
      const double e = std::sqrt(g.norm2_mean_dX[i] + Chat * g.mean_dY[i] * g.mean_dY[i]) * sc;
      if (!(e > 0)) continue;
      const double y = std::log2(e);
      sx += i; sy += y; sxx += (double)i * i; sxy += i * y; ++cnt;
    }
    if (cnt >= 2) {
      const double slope = (cnt * sxy - sx * sy) / (cnt * sxx - sx * sx);
      if (std::isfinite(slope) && -slope > 0.5) ahat = -slope;
    }
  }
  o.alpha_hat = ahat;
  // squared bias, Giles extrapolation of each level's correction to the finest
  double err_num = 0.0;
  for (int i = 1; i < L; ++i) {
    const double e2 = (g.norm2_mean_dX[i] + Chat * g.mean_dY[i] * g.mean_dY[i]) * sc * sc;
    const double d = std::pow(2.0, ahat) - 1.0;
    err_num = std::max(err_num, e2 / (d * d) * std::pow(2.0, -2.0 * ahat * (double)(L - 1 - i)));
  }
  o.err_num = err_num;
  // level update: one more level when the bias dominates (capped at the grid list)
  o.L = L;
  if (err_num > 0.5 * eps * eps && L < c->pb.n_levels) {
    o.M[L] = std::max<int64_t>(2, std::min<int64_t>(batch_cap(c->pb.grid_n[L]), o.M[L - 1] / 4));
    o.L = L + 1;
  }
  return o;
}

// Address of `scratch` on each device, looked up once per device with that
// device current.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {nullptr};

void* scratch_on_device(int dev) {
  require(dev >= 0 && dev < kMaxDevices, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* ptr = nullptr;
    HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    require(ptr != nullptr, "no device address for the scratch array");
    g_scratch_addr[dev] = ptr;
  }
  return g_scratch_addr[dev];
}

// State (and adjoint) solves of one level block on a prepared plan; shared
// by mlsgd_solve_state_adjoint and its allocation-free variant.
int solve_block(mlsgd_ctx* c, Plan* P, int n, int64_t count, double* y_out, double* p_out,
                double* phi_out, mlsgd_solve_stats* st) {
  int it1 = 0, nc1 = 0, it2 = 0, nc2 = 0;
  double r1 = 0, r2 = 0;
  state_phase(c, P, &it1, &nc1, &r1, y_out);
  if (phi_out)
    HIPCHK(hipMemcpyAsync(phi_out, P->d_phi, sizeof(double) * count, hipMemcpyDeviceToDevice,
                          c->stream));
  if (p_out) {   // the misfit pass left |y - y_d|^2 in the partial slots
    krylov(c, P, &it2, &nc2, &r2, true);
    unpack_rows(n, (int)count, P->groups[0].x, p_out, c->stream);
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(c->stream));
  if (st) {
    st->iterations = std::max(it1, it2);
    st->nonconverged = nc1 + nc2;
    st->max_relres = std::max(r1, r2);
  }
  if (nc1 + nc2 > 0) {
    c->err = "some solves missed rtol";
    return MLSGD_ENOCONV;
  }
  return MLSGD_OK;
}

int guard_impl(mlsgd_ctx* c, const std::function<int()>& fn) {
  try {
    if (c) c->err.clear();
    return fn();
  } catch (const Fail& f) {
    if (c) c->err = f.msg;
    return f.code;
  } catch (const std::exception& e) {
    if (c) c->err = e.what();
    return MLSGD_EHIP;
  }
}
}  // namespace

extern "C" {

int mlsgd_create(mlsgd_ctx** out, const mlsgd_problem* pb, void* stream) {
  if (!out || !pb) return MLSGD_EINVAL;
  *out = nullptr;
  auto c = std::make_unique<mlsgd_ctx>();
  int rc = guard_impl(c.get(), [&]() -> int {
    require(pb->n_levels >= 1 && pb->n_levels <= MLSGD_MAX_LEVELS, "n_levels out of range");
    for (int i = 0; i < pb->n_levels; ++i) {
      require(is_dyadic(pb->grid_n[i]) && pb->grid_n[i] >= 5 && pb->grid_n[i] <= 1025,
              "grid sizes must be 2^m + 1 between 5 and 1025");
      if (i > 0) require(pb->grid_n[i] == 2 * pb->grid_n[i - 1] - 1, "levels must be nested");
    }
    require(pb->kl_K >= 1 && pb->kl_K <= MLSGD_MAX_K, "kl_K out of range");
    require(pb->kl_sigma2 >= 0.0 && std::isfinite(pb->kl_sigma2), "kl_sigma2 must be >= 0");
    require(pb->theta >= 0.0 && std::isfinite(pb->theta), "theta must be >= 0");
    require(pb->kl_law == MLSGD_LAW_ALGEBRAIC || pb->kl_law == MLSGD_LAW_EXPONENTIAL,
            "kl_law must be MLSGD_LAW_ALGEBRAIC or MLSGD_LAW_EXPONENTIAL");
    require(pb->kl_law != MLSGD_LAW_EXPONENTIAL || (pb->kl_rho > 0.0 && std::isfinite(pb->kl_rho)),
            "kl_rho must be > 0 for MLSGD_LAW_EXPONENTIAL");
    require(pb->alpha >= 0.0 && std::isfinite(pb->alpha), "alpha must be >= 0");
    require(pb->precision == MLSGD_FP64 || pb->precision == MLSGD_MIXED_FP32 ||
                pb->precision == MLSGD_MIXED_BF16,
            "precision must be MLSGD_FP64, MLSGD_MIXED_FP32 or MLSGD_MIXED_BF16");
    require(pb->precision == MLSGD_FP64 || pb->solver == MLSGD_SOLVER_MGPCG,
            "mixed precision needs the multigrid solver");
    require(pb->solver == MLSGD_SOLVER_CG || pb->solver == MLSGD_SOLVER_MGPCG, "unknown solver");
    require(pb->rtol > 0.0 && pb->rtol < 1.0, "rtol must be in (0, 1)");
    require(pb->max_iters >= 1, "max_iters must be >= 1");
    require(pb->y_d != nullptr, "y_d is null");
    c->pb = *pb;
    c->stream = (hipStream_t)stream;
    c->mixed = pb->precision == MLSGD_MIXED_FP32 || pb->precision == MLSGD_MIXED_BF16;
    c->bf16 = pb->precision == MLSGD_MIXED_BF16;
    // measured defaults: Chebyshev smoothing of degree 2 on [0.3, 2], the
    // autotuner's choice for FP64, FP32 and bfloat16-coefficient V-cycles
    c->nu = 2;
    c->cheb_lo = 0.15;
    if (const char* e = getenv("MLSGD_NU")) c->nu = std::max(1, atoi(e));
    if (const char* e = getenv("MLSGD_OMEGA")) c->omega = atof(e);
    if (const char* e = getenv("MLSGD_CACHE64")) c->cache64 = atoi(e) != 0;
    if (const char* e = getenv("MLSGD_CACHE32")) c->cache32 = atoi(e) != 0;
    if (const char* e = getenv("MLSGD_SMOOTHER")) {
      const std::string v(e);
      c->smoother = v == "rbgs" ? 0 : v == "rbfused" ? 1 : 2;
    }
    if (const char* e = getenv("MLSGD_CHEB_LO")) c->cheb_lo = atof(e);
    if (const char* e = getenv("MLSGD_TY64")) c->tile_y = atoi(e);
    if (const char* e = getenv("MLSGD_XCHUNK")) c->xchunk = atoi(e);
    if (const char* e = getenv("MLSGD_PRE2R")) c->pre2r = atoi(e) != 0;
    if (const char* e = getenv("MLSGD_PRE2R_HALF")) c->pre2r_half = atoi(e) != 0;
    if (const char* e = getenv("MLSGD_POST2")) c->post2 = atoi(e) != 0;
    if (const char* e = getenv("MLSGD_VSMALL")) c->vsmall = atoi(e) != 0;
    if (const char* e = getenv("MLSGD_XDEFER")) c->xdefer = atoi(e) != 0;
    if (const char* e = getenv("MLSGD_FMG")) c->fmg = atoi(e) != 0;
    if (const char* e = getenv("MLSGD_FMG_MARGIN")) c->fmg_margin = atof(e);
    if (const char* e = getenv("MLSGD_FORCE_RESTART")) c->force_restart = atoi(e) != 0;
    if (!(c->fmg_margin > 0.0 && c->fmg_margin <= 1.0)) c->fmg_margin = 0.7;
    c->nfin = pb->grid_n[pb->n_levels - 1];
    const size_t NF = cube(c->nfin);
    c->d_f = (double*)dalloc(c.get(), sizeof(double) * NF);
    c->d_yd = (double*)dalloc(c.get(), sizeof(double) * NF);
    if (pb->f)
      HIPCHK(hipMemcpyAsync(c->d_f, pb->f, sizeof(double) * NF, hipMemcpyDeviceToDevice, c->stream));
    else
      HIPCHK(hipMemsetAsync(c->d_f, 0, sizeof(double) * NF, c->stream));
    HIPCHK(hipMemcpyAsync(c->d_yd, pb->y_d, sizeof(double) * NF, hipMemcpyDeviceToDevice,
                          c->stream));
    c->pb.f = c->d_f;
    c->pb.y_d = c->d_yd;
    for (int i = 0; i < pb->n_levels; ++i) {
      const int n = pb->grid_n[i];
      const size_t N = cube(n);
      c->yd_lvl[n] = (double*)dalloc(c.get(), sizeof(double) * N);
      c->rhs_lvl[n] = (double*)dalloc(c.get(), sizeof(double) * N);
      c->mean_lvl[n] = (double*)dalloc(c.get(), sizeof(double) * N);
      c->acc_lvl[n] = (double*)dalloc(c.get(), sizeof(double) * N);
      HIPCHK(hipMemsetAsync(c->mean_lvl[n], 0, sizeof(double) * N, c->stream));
      inject_full(c->nfin, c->d_yd, n, c->yd_lvl[n], c->stream);
    }
    c->d_umask = (double*)dalloc(c.get(), sizeof(double) * NF);
    c->d_grad = (double*)dalloc(c.get(), sizeof(double) * NF);
    c->d_epi_lev = (EpiLevel*)dalloc(c.get(), sizeof(EpiLevel) * MLSGD_MAX_LEVELS);
    c->d_epi_out = (EpiOut*)dalloc(c.get(), sizeof(EpiOut));
    c->d_count = (int*)dalloc(c.get(), sizeof(int));
    c->d_flag = (int*)dalloc(c.get(), sizeof(int));
    c->d_stat = (mlsgd_ctx::StatDev*)dalloc(c.get(), 2 * sizeof(mlsgd_ctx::StatDev));
    HIPCHK(hipHostMalloc((void**)&c->h_epi_out, sizeof(EpiOut), hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void**)&c->h_count, sizeof(int), hipHostMallocDefault));
    HIPCHK(hipHostMalloc((void**)&c->h_stat, 2 * sizeof(mlsgd_ctx::StatDev),
                         hipHostMallocDefault));
    for (auto& e : c->ev) HIPCHK(hipEventCreate(&e));
    // every grid of the hierarchy gets its cosine table now, so that a solve
    // on these grids allocates nothing but its plan's arena
    for (int i = 0; i < pb->n_levels; ++i)
      for (int n = pb->grid_n[i];; n = (n - 1) / 2 + 1) {
        cos_for(c.get(), n);
        if (n <= 3) break;
      }
    HIPCHK(hipGetDevice(&c->device));
    c->scratch = scratch_on_device(c->device);
    c->cur_L = pb->n_levels;
    HIPCHK(hipStreamSynchronize(c->stream));
    return MLSGD_OK;
  });
  if (rc != MLSGD_OK) {
    mlsgd_destroy(c.release());
    return rc;
  }
  *out = c.release();
  return MLSGD_OK;
}

int mlsgd_kernel_timing(mlsgd_ctx* c, int enable, int n, double* ms_total, int64_t* launches,
                        double* bytes) {
  if (!c) return MLSGD_EINVAL;
  return guard_impl(c, [&]() -> int {
    HIPCHK(hipStreamSynchronize(c->stream));
    if (c->tm.used) timing_collect(c);
    if (ms_total) *ms_total = c->tm.ms;
    if (launches) *launches = c->tm.launches;
    if (bytes) *bytes = c->tm.total_bytes;
    if (enable >= 0) {
      require(enable <= 4, "enable must be -1, 0, 1, 2, 3 or 4");
      c->tm.on = enable != 0;
      c->tm.kind = enable != 0 ? enable : 1;
      c->tm.n = n;
      c->tm.ms = 0.0;
      c->tm.total_bytes = 0.0;
      c->tm.launches = 0;
    }
    return MLSGD_OK;
  });
}

int mlsgd_set_graph(mlsgd_ctx* c, int enable) {
  if (!c) return MLSGD_EINVAL;
  return guard_impl(c, [&]() -> int {
    require(enable == 0 || enable == 1, "enable must be 0 or 1");
    if (enable && !c->cap_stream) {
      HIPCHK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
      c->d_u_graph = (double*)dalloc(c, sizeof(double) * cube(c->nfin));
      c->d_g_graph = (double*)dalloc(c, sizeof(double) * cube(c->nfin));
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    if (!enable) drop_graphs(c);
    c->graph = enable != 0;
    return MLSGD_OK;
  });
}

int mlsgd_get_tuning(const mlsgd_ctx* c, mlsgd_tuning* t) {
  if (!c || !t) return MLSGD_EINVAL;
  t->smoother = c->smoother;
  t->sweeps = c->nu;
  t->omega = c->omega;
  t->cheb_lo = c->cheb_lo;
  t->tile_y = c->tile_y;
  t->xchunk = c->xchunk;
  t->cache = c->mixed ? (c->cache32 ? 1 : 0) : (c->cache64 ? 1 : 0);
  return MLSGD_OK;
}

int mlsgd_set_tuning(mlsgd_ctx* c, const mlsgd_tuning* t) {
  if (!c) return MLSGD_EINVAL;
  return guard_impl(c, [&]() -> int {
    require(t != nullptr, "tuning is null");
    require(t->smoother >= 0 && t->smoother <= 2, "unknown smoother");
    require(t->sweeps >= 1 && t->sweeps <= 8, "sweeps must be in 1..8");
    require(t->omega > 0.0 && t->omega < 2.0, "omega must be in (0, 2)");
    require(t->cheb_lo > 0.0 && t->cheb_lo < 1.0, "cheb_lo must be in (0, 1)");
    require(t->tile_y == 4 || t->tile_y == 8 || t->tile_y == 16, "tile_y must be 4, 8 or 16");
    require(t->xchunk >= 8 && t->xchunk <= 1024, "xchunk must be in 8..1024");
    HIPCHK(hipStreamSynchronize(c->stream));
    c->smoother = t->smoother;
    c->nu = t->sweeps;
    c->omega = t->omega;
    c->cheb_lo = t->cheb_lo;
    c->tile_y = t->tile_y;
    c->xchunk = t->xchunk;
    if (c->mixed)
      c->cache32 = t->cache != 0;
    else
      c->cache64 = t->cache != 0;
    drop_plans(c);      // layouts depend on the tiling and the caches
    return MLSGD_OK;
  });
}

int mlsgd_destroy(mlsgd_ctx* c) {
  if (!c) return MLSGD_OK;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  (void)hipDeviceSynchronize();
  for (auto& pr : c->tm.pool) {
    (void)hipEventDestroy(pr.first);
    (void)hipEventDestroy(pr.second);
  }
  for (auto& kv : c->graphs)
    if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  for (void* p : c->allocs) (void)hipFree(p);
  if (c->h_epi_out) (void)hipHostFree(c->h_epi_out);
  if (c->h_count) (void)hipHostFree(c->h_count);
  if (c->h_stat) (void)hipHostFree(c->h_stat);
  for (auto& e : c->ev)
    if (e) (void)hipEventDestroy(e);
  delete c;
  return MLSGD_OK;
}

const char* mlsgd_last_error(const mlsgd_ctx* c) { return c ? c->err.c_str() : "null context"; }

int mlsgd_sample_fields(mlsgd_ctx* c, int level, int64_t first, int64_t count, double* xi_out) {
  if (!c) return MLSGD_EINVAL;
  return guard_impl(c, [&]() -> int {
    require(level >= 0 && level < c->pb.n_levels, "level out of range");
    require(first >= 0 && count >= 0, "first and count must be >= 0");
    require(count == 0 || xi_out != nullptr, "xi_out is null");
    const int K3 = c->pb.kl_K * c->pb.kl_K * c->pb.kl_K;
    kl_draws(c->pb.seed, level, first, count, K3, c->pb.kl_law, xi_out, c->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
    return MLSGD_OK;
  });
}

int mlsgd_philox_words(uint64_t seed, int level, int64_t sample, int tag, int nblocks,
                       uint64_t* out, void* stream) {
  if (nblocks < 0 || (nblocks > 0 && !out)) return MLSGD_EINVAL;
  philox_words(seed, level, sample, tag, nblocks, out, (hipStream_t)stream);
  if (hipGetLastError() != hipSuccess) return MLSGD_EHIP;
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return MLSGD_EHIP;
  return MLSGD_OK;
}

int mlsgd_solve_state_adjoint(mlsgd_ctx* c, int level, int coarse, int64_t first, int64_t count,
                              const double* u, double* y_out, double* p_out, double* phi_out,
                              mlsgd_solve_stats* st) {
  if (!c) return MLSGD_EINVAL;
  return guard_impl(c, [&]() -> int {
    require(level >= 0 && level < c->pb.n_levels, "level out of range");
    require(coarse == 0 || (coarse == 1 && level >= 1), "coarse solve needs level >= 1");
    require(first >= 0 && count >= 1, "need first >= 0 and count >= 1");
    check_u(c, u);
    const int n = c->pb.grid_n[level - coarse];
    level_rhs(c, u);
    std::vector<Block> b{Block{n, level, first, count}};
    Plan* P = get_plan(c, b);
    return solve_block(c, P, n, count, y_out, p_out, phi_out, st);
  });
}

int mlsgd_solve_state_adjoint_noalloc(mlsgd_ctx* c, int level, int coarse, int64_t first,
                                      int64_t count, const double* u, double* y_out,
                                      double* p_out, double* phi_out, mlsgd_solve_stats* st,
                                      int64_t* scratch_bytes) {
  if (!c) return MLSGD_EINVAL;
  return guard_impl(c, [&]() -> int {
    require(level >= 0 && level < c->pb.n_levels, "level out of range");
    require(coarse == 0 || (coarse == 1 && level >= 1), "coarse solve needs level >= 1");
    require(first >= 0 && count >= 1, "need first >= 0 and count >= 1");
    require(!c->tm.on, "kernel timing is on (its event pool may grow)");
    require(c->scratch != nullptr, "no scratch address for this context's device");
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    require(dev == c->device, "the context's device must be current");
    const int n = c->pb.grid_n[level - coarse];
    std::vector<Block> b{Block{n, level, first, count}};
    Plan T;   // transient: never enters the plan cache
    plan_layout(c, b, &T);
    const size_t need = plan_carve(c, &T, nullptr);
    if (scratch_bytes) *scratch_bytes = (int64_t)need;
    if (need > kScratchBytes)
      throw Fail{MLSGD_EINVAL, "the batch needs " + std::to_string(need) +
                                   " bytes of scratch; the limit is " +
                                   std::to_string(kScratchBytes)};
    check_u(c, u);
    level_rhs(c, u);
    T.arena = c->scratch;
    T.arena_bytes = need;
    plan_carve(c, &T, (char*)c->scratch);
    plan_init(c, &T);   // the array keeps the previous call's contents
    plan_draws(c, &T, b, true);
    return solve_block(c, &T, n, count, y_out, p_out, phi_out, st);
  });
}

int mlsgd_dense_coarse_inverse(mlsgd_ctx* c, int n, int level, int64_t first, int count,
                               double* out) {
  if (!c) return MLSGD_EINVAL;
  return guard_impl(c, [&]() -> int {
    require(n >= 4 && n <= 9, "n must be between 4 and 9");
    require(level >= 0 && first >= 0 && count >= 1 && count <= 4096,
            "need level >= 0, first >= 0 and 1 <= count <= 4096");
    require(out != nullptr, "out is null");
    const int K = c->pb.kl_K, K3 = K * K * K;
    const int N = (n - 2) * (n - 2) * (n - 2), Np = dense_pitch(N);
    std::vector<int> lv(count, level);
    std::vector<int64_t> sm(count);
    for (int j = 0; j < count; ++j) sm[j] = first + j;
    char* buf = (char*)dalloc(c, sizeof(int) * count + sizeof(int64_t) * count +
                                     sizeof(double) * ((size_t)count * K3 + 2 * (size_t)count * Np * Np) + 1024);
    Carver cv{buf};
    int* d_lv = cv.take<int>(count);
    int64_t* d_sm = cv.take<int64_t>(count);
    double* d_coef = cv.take<double>((size_t)count * K3);
    double* d_ainv = cv.take<double>((size_t)count * Np * Np);
    double* d_work = cv.take<double>((size_t)count * Np * Np);
    HIPCHK(hipMemcpyAsync(d_lv, lv.data(), sizeof(int) * count, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(d_sm, sm.data(), sizeof(int64_t) * count, hipMemcpyHostToDevice,
                          c->stream));
    kl_coeffs(d_lv, d_sm, count, c->pb.seed, K, c->pb.kl_sigma2, c->pb.kl_law, c->pb.kl_rho,
              d_coef, c->stream);
    dense_coarse_inv(n, count, d_coef, K, cos_for(c, n), d_ainv, d_work, c->stream);
    HIPCHK(hipGetLastError());
    for (int j = 0; j < count; ++j)
      HIPCHK(hipMemcpy2DAsync(out + (size_t)j * N * N, sizeof(double) * N,
                              d_ainv + (size_t)j * Np * Np, sizeof(double) * Np,
                              sizeof(double) * N, (size_t)N, hipMemcpyDeviceToDevice, c->stream));
    dfree(c, buf);   // synchronises the stream first
    return MLSGD_OK;
  });
}

// grid halved while its cell count is even: the coarsest grid of n's hierarchy
static int coarsest_of(int n) {
  while (n > 3 && !((n - 1) & 1)) n = (n - 1) / 2 + 1;
  return n;
}

int mlsgd_solve_sizes(mlsgd_ctx* c, int count, const int* n_list, int level, int64_t first,
                      double f_value, double* y_out, mlsgd_solve_stats* st) {
  if (!c) return MLSGD_EINVAL;
  return guard_impl(c, [&]() -> int {
    require(count >= 1 && n_list != nullptr, "need count >= 1 and a size list");
    require(first >= 0 && level >= 0, "need first >= 0 and level >= 0");
    require(std::isfinite(f_value), "f_value is not finite");
    std::vector<long long> off(count);
    long long tot = 0;
    std::map<int, std::vector<int>, std::greater<int>> fam;  // grid -> problems, largest first
    for (int j = 0; j < count; ++j) {
      const int n = n_list[j];
      require(n >= 5 && n <= 1025 && (n & 1), "grid sizes must be odd, 5 .. 1025");
      require(coarsest_of(n) <= 9, "grid must coarsen to at most 9 vertices per axis");
      off[j] = tot;
      tot += (long long)n * n * n;
      fam[n].push_back(j);
    }
    hipStream_t s = c->stream;
    int iters = 0, nonconv = 0;
    double relres = 0.0;
    for (auto& kv : fam) {
      const int n = kv.first;
      const std::vector<int>& js = kv.second;
      std::vector<Block> blocks;
      for (int j : js) blocks.push_back(Block{n, level, first + j, 1});
      Plan* P = get_plan(c, blocks);
      double*& rhs = c->const_rhs[n];
      if (!rhs) rhs = (double*)dalloc(c, sizeof(double) * cube(n));
      fill_interior(n, f_value, rhs, s);
      Group& gr = P->groups[0];
      rows_broadcast(n, gr.count, rhs, rows_of(P->sizes[gr.sl].B, gr), s);
      rows_broadcast(n, gr.count, rhs, gr.b0, s);
      rows_zero((long long)gr.count * srow(n), gr.x, s);
      HIPCHK(hipGetLastError());
      int it = 0, nc = 0;
      double rr = 0.0;
      krylov(c, P, &it, &nc, &rr);
      iters = std::max(iters, it);
      nonconv += nc;
      relres = std::max(relres, rr);
      if (y_out) {
        if (c->dst_off_len < js.size()) {
          c->d_dst_off = (long long*)dalloc(c, sizeof(long long) * js.size());
          c->dst_off_len = js.size();
        }
        std::vector<long long> h(js.size());
        for (size_t k = 0; k < js.size(); ++k) h[k] = off[js[k]];
        HIPCHK(hipMemcpyAsync(c->d_dst_off, h.data(), sizeof(long long) * h.size(),
                              hipMemcpyHostToDevice, s));
        scatter_rows(n, (int)js.size(), c->d_dst_off, gr.x, y_out, s);
        HIPCHK(hipStreamSynchronize(s));  // h and d_dst_off are reused by the next family
      }
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    if (st) {
      st->iterations = iters;
      st->nonconverged = nonconv;
      st->max_relres = relres;
    }
    if (nonconv > 0) {
      c->err = "some solves missed rtol";
      return MLSGD_ENOCONV;
    }
    return MLSGD_OK;
  });
}

int mlsgd_mlmc_gradient(mlsgd_ctx* c, const double* u, int L, const int64_t* M,
                        const int64_t* first, double* grad_out, mlsgd_grad_stats* st) {
  if (!c) return MLSGD_EINVAL;
  return guard_impl(c, [&]() -> int {
    require(grad_out != nullptr, "grad_out is null");
    return run_estimate(c, u, L, M, first, grad_out, nullptr, st);
  });
}

int mlsgd_mlmc_objective(mlsgd_ctx* c, const double* u, int L, const int64_t* M,
                         const int64_t* first, double* J_out, mlsgd_grad_stats* st) {
  if (!c) return MLSGD_EINVAL;
  return guard_impl(c, [&]() -> int {
    require(J_out != nullptr, "J_out is null");
    return run_estimate(c, u, L, M, first, nullptr, J_out, st);
  });
}

int mlsgd_set_batch(mlsgd_ctx* c, int L, const int64_t* M, const int64_t* offsets) {
  if (!c) return MLSGD_EINVAL;
  return guard_impl(c, [&]() -> int {
    require(L >= 1 && L <= c->pb.n_levels, "L out of range");
    require(M != nullptr, "M is null");
    for (int i = 0; i < L; ++i) {
      require(M[i] >= 1, "sample counts must be >= 1");
      if (offsets) require(offsets[i] >= 0, "offsets must be >= 0");
    }
    c->cur_L = L;
    for (int i = 0; i < MLSGD_MAX_LEVELS; ++i) {
      c->cur_M[i] = i < L ? M[i] : 0;
      c->cur_off[i] = (offsets && i < L) ? offsets[i] : 0;
    }
    c->prev_gnorm = -1.0;
    c->have_gprev = false;
    return MLSGD_OK;
  });
}

// Adaptive step size (Sec. 5, eq. adaptive-step-size): with g_k the
// estimate just computed and g_{k-1}, tau_{k-1} those of the previous step,
//   Lhat  = |g_k - g_{k-1}|_h / (tau_{k-1} |g_{k-1}|_h)
//   tau_k = (|g_k|_h^2 - err_sam_k) / (Lhat |g_k|_h^2),
// clamped at 0 from below.  The first step of a batch uses the given tau; a
// step after a zero step, or an undefined Lhat, reuses the last positive one.
double adaptive_tau(mlsgd_ctx* c, double tau0, double gnorm, double err_sam) {
  if (!c->have_gprev) return tau0;
  if (!(c->tau_prev > 0.0) || !(c->gnorm_prev > 0.0)) return c->tau_pos > 0.0 ? c->tau_pos : tau0;
  hipStream_t s = c->stream;
  const long long N = (long long)cube(c->nfin);
  copy_elems((long long)cube(c->nfin), c->d_grad, c->d_gtmp, s);
  axpy_full(c->nfin, -1.0, c->d_gprev, c->d_gtmp, s);
  dot_blocks(N, c->d_gtmp, c->d_gtmp, c->d_epi_part, s);
  finish_norm(c->nfin, c->d_epi_part, c->d_sc1, s);
  double diff2 = 0.0;
  HIPCHK(hipMemcpyAsync(&diff2, c->d_sc1, sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const double Lhat = std::sqrt(diff2) / (c->tau_prev * c->gnorm_prev);
  const double g2 = gnorm * gnorm;
  if (!(Lhat > 0.0) || !std::isfinite(Lhat) || !(g2 > 0.0))
    return c->tau_pos > 0.0 ? c->tau_pos : tau0;
  return std::max(0.0, (g2 - err_sam) / (Lhat * g2));
}

int mlsgd_step(mlsgd_ctx* c, double* u, double tau, int adapt, mlsgd_step_stats* st) {
  if (!c) return MLSGD_EINVAL;
  return guard_impl(c, [&]() -> int {
    require(u != nullptr, "u is null");
    require(std::isfinite(tau), "tau must be finite");
    require(adapt >= 0 && adapt <= (MLSGD_ADAPT_BATCH | MLSGD_ADAPT_STEP),
            "adapt must combine MLSGD_ADAPT_BATCH and MLSGD_ADAPT_STEP");
    require(c->cur_M[0] >= 1, "call mlsgd_set_batch first");
    if (adapt)
      for (int i = 0; i < c->cur_L; ++i) require(c->cur_M[i] >= 2, "adapt needs M >= 2");
    if ((adapt & MLSGD_ADAPT_STEP) && !c->d_gprev) {
      c->d_gprev = (double*)dalloc(c, sizeof(double) * cube(c->nfin));
      c->d_gtmp = (double*)dalloc(c, sizeof(double) * cube(c->nfin));
      c->d_sc1 = (double*)dalloc(c, sizeof(double));
    }
    mlsgd_grad_stats g{};
    const int rc = run_estimate(c, u, c->cur_L, c->cur_M, c->cur_off, c->d_grad, nullptr, &g);
    if (rc != MLSGD_OK && rc != MLSGD_ENOCONV) return rc;
    mlsgd_step_stats loc{};
    CtrlOut o{};
    if (adapt) {
      o = controller(c, g, c->cur_L, c->cur_M);
      loc.err_sam = o.err_sam;
      loc.err_num = o.err_num;
      loc.eps = o.eps;
    }
    double tk = tau;
    if (adapt & MLSGD_ADAPT_STEP) {
      tk = adaptive_tau(c, tau, g.grad_norm, o.err_sam);
      copy_elems((long long)cube(c->nfin), c->d_grad, c->d_gprev, c->stream);
      c->have_gprev = true;
      c->tau_prev = tk;
      if (tk > 0.0) c->tau_pos = tk;
      c->gnorm_prev = g.grad_norm;
    }
    loc.tau = tk;
    const bool box = c->pb.u_lo <= c->pb.u_hi;
    box_step(c->nfin, u, c->d_grad, tk, c->pb.u_lo, c->pb.u_hi, box ? 1 : 0, c->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
    for (int i = 0; i < c->cur_L; ++i) c->cur_off[i] += c->cur_M[i];
    c->prev_gnorm = g.grad_norm;
    if (adapt & MLSGD_ADAPT_BATCH) {
      for (int i = 0; i < o.L; ++i) c->cur_M[i] = o.M[i];
      c->cur_L = o.L;
    }
    if (st) {
      loc.grad = g;
      for (int i = 0; i < MLSGD_MAX_LEVELS; ++i) {
        loc.M_next[i] = i < c->cur_L ? c->cur_M[i] : 0;
        loc.offset[i] = i < c->cur_L ? c->cur_off[i] : 0;
      }
      *st = loc;
    }
    return rc;
  });
}

}  // extern "C"
