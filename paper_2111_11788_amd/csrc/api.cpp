// C-ABI of the MLMC finite-element library: context, arena carving, the
// batched GMG-PCG engine and the multilevel estimator.
//
// Whole path of one batch (Sec. 2.2: a level-l sample evaluates the n_l and
// n_{l-1} meshes on one draw and contributes Y_l = Q_l - Q_{l-1}):
//   xi (Philox) -> kappa on each mesh (MFMA KLE) -> GMG-PCG solve per mesh ->
//   QoI -> Y -> running statistics of the level.
// Solver: conjugate gradients preconditioned by one V-cycle (Chebyshev-Jacobi
// smoothing, rediscretised coarse operators down to the 2^3 mesh).  Mixed
// precision runs that PCG in fp32 vectors (fp64 scalars) as the inner solver
// of an fp64 iterative refinement whose residual b - A x is formed in fp64.
#include "mlmc.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "common.hpp"
#include "grid.hpp"
#include "kernels.hpp"
#include "kl_host.hpp"

using namespace mlmc;

namespace {

constexpr double kChebHi = 2.0;      // Gershgorin bound of D^-1 A for this operator
constexpr double kChebRatio = 4.0;   // smoothing interval [hi / ratio, hi]
constexpr double kInnerRtol = 1e-4;  // fp32 inner solve tolerance (mixed precision)
constexpr int kMaxOuter = 30;

inline size_t align256(size_t b) { return (b + 255) / 256 * 256; }
inline int ilog2i(int n) { int l = 0; while ((1 << l) < n) ++l; return l; }
inline bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

// Bump carver over the caller's arena; a dry run only counts bytes.
struct Carver {
  char* base = nullptr;
  size_t top = 0, cap = 0;
  bool dry = true;
  template <class T>
  T* take(size_t count) {
    const size_t bytes = align256(count * sizeof(T));
    T* p = dry ? nullptr : reinterpret_cast<T*>(base + top);
    top += bytes;
    return p;
  }
};

struct ChebCoeffs {
  int degree = 2;
  double c1[16] = {0}, c2[16] = {0};
};

// Three-term Chebyshev semi-iteration on [lo, hi] (Saad, Iterative Methods, Alg. 12.1)
ChebCoeffs cheb_coeffs(int degree, double lo, double hi) {
  ChebCoeffs c;
  c.degree = degree;
  const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
  c.c1[0] = 0.0;
  c.c2[0] = 1.0 / theta;
  double rho = 1.0 / sigma;
  for (int s = 1; s < degree; ++s) {
    const double rn = 1.0 / (2.0 * sigma - rho);
    c.c1[s] = rn * rho;
    c.c2[s] = 2.0 * rn / delta;
    rho = rn;
  }
  return c;
}

template <class T>
struct Level {
  int n = 0;
  T* kap = nullptr;
  T *b = nullptr, *x = nullptr, *xo = nullptr, *t = nullptr;
};

struct StateBufs {
  SolveState s{};
  void carve(Carver& cv, int B, int n) {
    s.pstride = max_parts(n, B);
    s.rz = cv.take<double>(B);
    s.alpha = cv.take<double>(B);
    s.beta = cv.take<double>(B);
    s.rr = cv.take<double>(B);
    s.bb = cv.take<double>(B);
    s.partial = cv.take<double>((size_t)B * s.pstride);
    s.active = cv.take<int>(B);
    s.iters = cv.take<int>(B);
    s.nactive = cv.take<int>(1);
  }
};

// Work space of one batched solve on an n^3 mesh.
struct SolveWork {
  int n = 0, B = 0, precision = 0, solver = 0;
  std::vector<Level<double>> L64;   // fp64 hierarchy (level 0 kappa is the caller's)
  std::vector<Level<float>> L32;    // fp32 hierarchy (mixed precision)
  double *r = nullptr, *p = nullptr, *q = nullptr;          // fp64 PCG
  double* r64 = nullptr;                                    // fp64 refinement residual
  float *d = nullptr, *rin = nullptr, *p32 = nullptr, *q32 = nullptr;  // fp32 inner PCG
  StateBufs outer, inner;
  // captured PCG iteration per precision (0: fp64, 1: fp32); tied to the buffers above
  hipGraphExec_t iter_exec[2] = {nullptr, nullptr};

  void release_graphs() {
    for (auto& g : iter_exec)
      if (g) {
        hipGraphExecDestroy(g);
        g = nullptr;
      }
  }

  void carve(Carver& cv, int n_, int B_, int prec, int solv) {
    n = n_; B = B_; precision = prec; solver = solv;
    const int nl = solv == MLMC_SOLVER_GMG_PCG ? std::max(1, ilog2i(n)) : 1;
    const size_t S0 = grid_stride(n);
    outer.carve(cv, B, n);
    if (prec == MLMC_PREC_FP64) {
      r = cv.take<double>(B * S0);
      p = cv.take<double>(B * S0);
      q = cv.take<double>(B * S0);
      L64.assign(nl, Level<double>{});
      for (int l = 0; l < nl; ++l) {
        const int nn = n >> l;
        const size_t S = grid_stride(nn);
        L64[l].n = nn;
        if (l > 0) {
          L64[l].kap = cv.take<double>(B * elem_count(nn));
          L64[l].b = cv.take<double>(B * S);
        }
        L64[l].x = cv.take<double>(B * S);
        L64[l].xo = cv.take<double>(B * S);
        if (nl > 1 || l > 0) L64[l].t = cv.take<double>(B * S);
      }
    } else {
      inner.carve(cv, B, n);
      r64 = cv.take<double>(B * S0);
      d = cv.take<float>(B * S0);
      rin = cv.take<float>(B * S0);
      p32 = cv.take<float>(B * S0);
      q32 = cv.take<float>(B * S0);
      L32.assign(nl, Level<float>{});
      for (int l = 0; l < nl; ++l) {
        const int nn = n >> l;
        const size_t S = grid_stride(nn);
        L32[l].n = nn;
        L32[l].kap = cv.take<float>(B * elem_count(nn));
        if (l > 0) L32[l].b = cv.take<float>(B * S);
        L32[l].x = cv.take<float>(B * S);
        L32[l].xo = cv.take<float>(B * S);
        if (nl > 1 || l > 0) L32[l].t = cv.take<float>(B * S);
      }
    }
  }
};

// Work space of one batch of sample_level: draws, fields, solutions, QoIs.
struct BatchWork {
  int level = -1, B = 0;
  double* xi = nullptr;
  double *kf = nullptr, *kc = nullptr, *uf = nullptr, *uc = nullptr;
  double *qf = nullptr, *qc = nullptr;
  SolveWork wf, wc;
};

struct ProfRec {
  int id;
  hipEvent_t a, b;
  double bytes;
};

struct Running {
  uint64_t n = 0;
  double mean = 0.0, m2 = 0.0, cost = 0.0;
  double seconds = 0.0;     // wall time spent sampling this level
  uint64_t timed = 0;       // samples covered by `seconds`
  uint64_t next = 0;        // next unused sample index of the level
  void push(double y) {
    n += 1;
    const double d = y - mean;
    mean += d / (double)n;
    m2 += d * (y - mean);
  }
};

}  // namespace

struct mlmc_ctx {
  mlmc_config cfg{};
  hipStream_t st = nullptr;
  std::string err;
  KLModes modes;
  int K1 = 0;
  double* d_sqrtlam = nullptr;
  int* d_triples = nullptr;
  std::map<int, double*> d_tab;
  size_t persistent_top = 0;
  ChebCoeffs cheb;
  // cached work space (one at a time)
  int ws_kind = -1;              // 0: solve work, 1: batch work
  std::tuple<int, int, int, int> ws_key{-1, -1, -1, -1};
  SolveWork sw;
  BatchWork bw;
  std::vector<Running> stats;
  bool profiling = false;
  std::vector<ProfRec> prof;
  std::vector<hipEvent_t> event_pool;
  int64_t k_launch[2 * MLMC_K_COUNT] = {0};   // [precision][kernel]
  double k_ms[2 * MLMC_K_COUNT] = {0}, k_bytes[2 * MLMC_K_COUNT] = {0};
  int* h_nactive = nullptr;
  int zvar[2] = {0, 0};           // z-march kernel variant for fp64 / fp32
  int vsmall_n0[2] = {8, 16};     // mesh at which the single-kernel coarse V-cycle takes over (0: off)
  bool use_graphs = true;         // replay the PCG iteration from a captured hipGraph
  bool own_stream = false;        // the context created st itself
  int graph_batch = 2;            // graph launches per convergence check
};

static std::string g_create_error;

#define FAIL(code, msg)      \
  do {                       \
    ctx->err = (msg);        \
    return (code);           \
  } while (0)

#define HIPCHK(expr)                                                                 \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess) {                                                          \
      ctx->err = std::string("HIP error: ") + hipGetErrorString(e_) + " at " #expr; \
      return MLMC_E_DEVICE;                                                          \
    }                                                                                \
  } while (0)

namespace {

hipEvent_t take_event(mlmc_ctx* ctx) {
  if (!ctx->event_pool.empty()) {
    hipEvent_t e = ctx->event_pool.back();
    ctx->event_pool.pop_back();
    return e;
  }
  hipEvent_t e;
  hipEventCreate(&e);
  return e;
}

// Launch wrapper: optional event timing and algorithmic-byte accounting.
template <class F>
int launch(mlmc_ctx* ctx, int id, double bytes, F&& f) {
  hipEvent_t a = nullptr, b = nullptr;
  if (ctx->profiling) {
    a = take_event(ctx);
    b = take_event(ctx);
    hipEventRecord(a, ctx->st);
  }
  const hipError_t e = f();
  if (e != hipSuccess) {
    ctx->err = std::string("kernel launch failed: ") + hipGetErrorString(e);
    return MLMC_E_DEVICE;
  }
  if (ctx->profiling) {
    hipEventRecord(b, ctx->st);
    ctx->prof.push_back(ProfRec{id, a, b, bytes});
  }
  return MLMC_OK;
}

#define LAUNCH(id, bytes, call)                          \
  do {                                                   \
    int rc_ = launch(ctx, (id), (double)(bytes), [&] { return (call); }); \
    if (rc_) return rc_;                                 \
  } while (0)

// profiling slot of kernel `id` in the precision of T (fp32 slots follow the fp64 ones)
template <class T>
constexpr int kid(int id) { return id + (sizeof(T) == 4 ? MLMC_K_COUNT : 0); }
template <class T>
int zv(const mlmc_ctx* ctx) { return ctx->zvar[sizeof(T) == 4 ? 1 : 0]; }

inline double dofs(int n) { return (double)(n - 1) * (n - 1) * (n - 1); }
inline double elems(int n) { return (double)n * n * n; }

int validate(const mlmc_config* c, std::string& why) {
  if (!c) { why = "config is NULL"; return MLMC_E_INVALID; }
  if (c->n0 < 2 || !is_pow2(c->n0)) { why = "n0 must be a power of two >= 2"; return MLMC_E_INVALID; }
  if (c->levels < 1 || c->levels > 16) { why = "levels must be in 1..16"; return MLMC_E_INVALID; }
  if (((int64_t)c->n0 << (c->levels - 1)) > 1024) { why = "finest mesh above 1024^3"; return MLMC_E_INVALID; }
  if (!(c->sigma2 >= 0.0) || !(c->corr_len > 0.0)) { why = "need sigma2 >= 0 and corr_len > 0"; return MLMC_E_INVALID; }
  if (c->n_modes < 1 || c->n_modes > 4096) { why = "n_modes must be in 1..4096"; return MLMC_E_INVALID; }
  if (c->qoi != 0 && c->qoi != 1) { why = "unknown qoi"; return MLMC_E_INVALID; }
  // the subcube QoI needs 4 | n on every mesh that is solved
  if (c->qoi == 1 && c->n0 < 4) { why = "subcube QoI needs n0 >= 4"; return MLMC_E_INVALID; }
  if (!(c->rtol > 0.0) || c->max_iter < 1) { why = "need rtol > 0 and max_iter >= 1"; return MLMC_E_INVALID; }
  if (c->precision != 0 && c->precision != 1) { why = "unknown precision"; return MLMC_E_INVALID; }
  if (c->solver != 0 && c->solver != 1) { why = "unknown solver"; return MLMC_E_INVALID; }
  if (c->cheb_degree < 0 || c->cheb_degree > 8) { why = "cheb_degree must be in 0..8"; return MLMC_E_INVALID; }
  if (c->max_batch < 1) { why = "max_batch must be >= 1"; return MLMC_E_INVALID; }
  if (c->arena_bytes && !c->arena) { why = "arena_bytes > 0 with a NULL arena"; return MLMC_E_INVALID; }
  if (((uintptr_t)c->arena) % 256) { why = "arena must be 256-byte aligned"; return MLMC_E_INVALID; }
  return MLMC_OK;
}

size_t persistent_bytes(const mlmc_config* c, int K1) {
  Carver cv;
  cv.take<double>(c->n_modes);
  cv.take<int>(3 * (size_t)c->n_modes);
  for (int l = 0; l < c->levels; ++l) cv.take<double>((size_t)(c->n0 << l) * K1);
  return cv.top;
}

// Carve a solve work space for (n, B) unless the cached one matches.
int ensure_solve_work(mlmc_ctx* ctx, int n, int B) {
  const auto key = std::make_tuple(0, n, B, ctx->cfg.precision * 2 + ctx->cfg.solver);
  if (ctx->ws_kind == 0 && ctx->ws_key == key) return MLMC_OK;
  Carver cv;
  cv.base = (char*)ctx->cfg.arena;
  cv.cap = ctx->cfg.arena_bytes;
  cv.top = ctx->persistent_top;
  cv.dry = false;
  Carver dry = cv;
  dry.dry = true;
  SolveWork probe;
  probe.carve(dry, n, B, ctx->cfg.precision, ctx->cfg.solver);
  if (dry.top > cv.cap) {
    ctx->ws_kind = -1;
    FAIL(MLMC_E_NOMEM, "arena too small for a solve of " + std::to_string(B) + " samples on " +
                           std::to_string(n) + "^3: need " + std::to_string(dry.top) + " bytes");
  }
  ctx->sw.release_graphs();
  ctx->sw = SolveWork{};
  ctx->sw.carve(cv, n, B, ctx->cfg.precision, ctx->cfg.solver);
  HIPCHK(hipMemsetAsync((char*)ctx->cfg.arena + ctx->persistent_top, 0, cv.top - ctx->persistent_top, ctx->st));
  ctx->ws_kind = 0;
  ctx->ws_key = key;
  return MLMC_OK;
}

void carve_batch(Carver& cv, BatchWork& w, const mlmc_config& c, int level, int B) {
  const int nf = c.n0 << level;
  w.level = level;
  w.B = B;
  w.xi = cv.take<double>((size_t)B * c.n_modes);
  w.kf = cv.take<double>((size_t)B * elem_count(nf));
  w.uf = cv.take<double>((size_t)B * grid_stride(nf));
  w.qf = cv.take<double>(B);
  w.qc = cv.take<double>(B);
  w.wf.carve(cv, nf, B, c.precision, c.solver);
  if (level > 0) {
    const int nc = nf / 2;
    w.kc = cv.take<double>((size_t)B * elem_count(nc));
    w.uc = cv.take<double>((size_t)B * grid_stride(nc));
    w.wc.carve(cv, nc, B, c.precision, c.solver);
  }
}

int ensure_batch_work(mlmc_ctx* ctx, int level, int B) {
  const auto key = std::make_tuple(1, level, B, 0);
  if (ctx->ws_kind == 1 && ctx->ws_key == key) return MLMC_OK;
  Carver dry;
  dry.top = ctx->persistent_top;
  BatchWork probe;
  carve_batch(dry, probe, ctx->cfg, level, B);
  if (dry.top > ctx->cfg.arena_bytes) {
    ctx->ws_kind = -1;
    FAIL(MLMC_E_NOMEM, "arena too small for a batch of " + std::to_string(B) + " samples at level " +
                           std::to_string(level) + ": need " + std::to_string(dry.top) + " bytes");
  }
  Carver cv;
  cv.base = (char*)ctx->cfg.arena;
  cv.cap = ctx->cfg.arena_bytes;
  cv.top = ctx->persistent_top;
  cv.dry = false;
  ctx->bw.wf.release_graphs();
  ctx->bw.wc.release_graphs();
  ctx->bw = BatchWork{};
  carve_batch(cv, ctx->bw, ctx->cfg, level, B);
  HIPCHK(hipMemsetAsync((char*)ctx->cfg.arena + ctx->persistent_top, 0, cv.top - ctx->persistent_top, ctx->st));
  ctx->ws_kind = 1;
  ctx->ws_key = key;
  return MLMC_OK;
}

int ensure_tables(mlmc_ctx* ctx, int n, double** tab) {
  auto it = ctx->d_tab.find(n);
  if (it == ctx->d_tab.end()) FAIL(MLMC_E_INVALID, "mesh " + std::to_string(n) + " is not a level mesh");
  *tab = it->second;
  return MLMC_OK;
}

int field_impl(mlmc_ctx* ctx, int n, int B, const double* xi, double* kap, float* kap32) {
  double* tab = nullptr;
  if (int rc = ensure_tables(ctx, n, &tab)) return rc;
  const int M = ctx->cfg.n_modes;
  LAUNCH(MLMC_K_FIELD, (double)B * elems(n) * (8.0 + (kap32 ? 4.0 : 0.0)) + (double)B * M * 8.0,
         launch_field(n, M, B, xi, ctx->d_sqrtlam, ctx->d_triples, tab, ctx->K1, kap, kap32, ctx->st));
  return MLMC_OK;
}

// One V-cycle on levels l.. of L; returns the buffer that holds the result.
// With `dot` the last smoothing step of level l also writes the partial sums
// of b . result (*dot_np per sample).
template <class T>
int vcycle(mlmc_ctx* ctx, std::vector<Level<T>>& L, int l, int B, const T* b, T* x, T* xo, T* t,
           const int* active, T** result, SolveState* dot = nullptr, uint32_t* dot_np = nullptr) {
  const int n = L[l].n;
  const double sz = sizeof(T);
  const double d = dofs(n) * B, e = elems(n) * B;
  hipStream_t st = ctx->st;
  const int var = zv<T>(ctx);
  if (n == 2) {
    LAUNCH(kid<T>(MLMC_K_COARSEST), B * (8 + 2) * sz, launch_coarsest<T>(B, L[l].kap, b, x, active, st));
    *result = x;
    if (dot) FAIL(MLMC_E_INVALID, "fused r.z needs a mesh n >= 4");
    return MLMC_OK;
  }
  const ChebCoeffs& ch = ctx->cheb;
  const T* kap = L[l].kap;
  const int small = ctx->vsmall_n0[sizeof(T) == 4 ? 1 : 0];
  if (small && n <= small && n >= 4) {
    // the rest of the V-cycle in one kernel (coarse data in LDS)
    const T* kl[4] = {nullptr, nullptr, nullptr, nullptr};
    for (size_t q = l; q < L.size() && q - l < 4; ++q) kl[q - l] = L[q].kap;
    LAUNCH(kid<T>(MLMC_K_COARSEST), (2 * d + e * 8.0 / 7.0) * sz,
           launch_vsmall<T>(n, B, ch.degree, ch.c1, ch.c2, kl, b, x, active, st));
    *result = x;
    return MLMC_OK;
  }
  LAUNCH(kid<T>(MLMC_K_CHEB_ZERO), (2 * d + e) * sz,
         launch_cheb<T>(n, B, kap, b, nullptr, nullptr, x, 0.0, ch.c2[0], true, false, active, st, nullptr, nullptr,
                        var));
  T* cur = x;
  T* oth = xo;
  for (int s = 1; s < ch.degree; ++s) {
    const bool use_xo = s > 1;
    LAUNCH(kid<T>(use_xo ? MLMC_K_CHEB_XO : MLMC_K_CHEB), ((use_xo ? 4 : 3) * d + e) * sz,
           launch_cheb<T>(n, B, kap, b, cur, oth, oth, ch.c1[s], ch.c2[s], false, use_xo, active, st, nullptr,
                          nullptr, var));
    std::swap(cur, oth);
  }
  LAUNCH(kid<T>(MLMC_K_RESIDUAL), (3 * d + e) * sz, launch_residual<T>(n, B, kap, b, cur, t, active, st, var));
  Level<T>& nx = L[l + 1];
  const double dc = dofs(n / 2) * B;
  LAUNCH(kid<T>(MLMC_K_RESTRICT), (d + dc) * sz, launch_restrict<T>(n, B, t, nx.b, active, st));
  T* xc = nullptr;
  if (int rc = vcycle<T>(ctx, L, l + 1, B, nx.b, nx.x, nx.xo, nx.t, active, &xc)) return rc;
  LAUNCH(kid<T>(MLMC_K_PROLONG), (2 * d + dc) * sz, launch_prolong_add<T>(n, B, xc, cur, active, st));
  for (int s = 0; s < ch.degree; ++s) {
    const bool use_xo = s > 0;
    const bool last = s == ch.degree - 1;
    LAUNCH(kid<T>(use_xo ? MLMC_K_CHEB_XO : MLMC_K_CHEB), ((use_xo ? 4 : 3) * d + e) * sz,
           launch_cheb<T>(n, B, kap, b, cur, oth, oth, s == 0 ? 0.0 : ch.c1[s], ch.c2[s], false, use_xo, active, st,
                          last ? dot : nullptr, last ? dot_np : nullptr, var));
    std::swap(cur, oth);
  }
  *result = cur;
  return MLMC_OK;
}

// z = M^-1 r.  When *fused_np is set on return, the partial sums of r . z
// are already in S.partial (GMG path); otherwise the caller computes them.
template <class T>
int precondition(mlmc_ctx* ctx, std::vector<Level<T>>& L, int B, const T* r, T** z, SolveState& S,
                 uint32_t* fused_np) {
  const int n = L[0].n;
  *fused_np = 0;
  if (L.size() == 1 || n == 2) {
    if (n == 2) return vcycle<T>(ctx, L, 0, B, r, L[0].x, L[0].xo, L[0].t, S.active, z);
    // Jacobi: z = D^-1 r
    LAUNCH(kid<T>(MLMC_K_CHEB_ZERO), (2 * dofs(n) + elems(n)) * B * sizeof(T),
           launch_cheb<T>(n, B, L[0].kap, r, nullptr, nullptr, L[0].x, 0.0, 1.0, true, false, S.active, ctx->st,
                          nullptr, nullptr, zv<T>(ctx)));
    *z = L[0].x;
    return MLMC_OK;
  }
  return vcycle<T>(ctx, L, 0, B, r, L[0].x, L[0].xo, L[0].t, S.active, z, &S, fused_np);
}

int count_active(mlmc_ctx* ctx, SolveState& s, int B, int* out) {
  LAUNCH(MLMC_K_MISC, 0, launch_count_active(B, s, ctx->st));
  HIPCHK(hipMemcpyAsync(ctx->h_nactive, s.nactive, sizeof(int), hipMemcpyDeviceToHost, ctx->st));
  HIPCHK(hipStreamSynchronize(ctx->st));
  *out = *ctx->h_nactive;
  return MLMC_OK;
}

// PCG on the current iterate x with residual r (both already set, S.active
// and S.bb set).  Stops per sample at ||r|| <= tol ||b|| (recurrence).
// One PCG iteration after the initial preconditioning: q = A p, alpha, x and r
// updates with the convergence test, z = M^-1 r, beta, p = z + beta p, and
// the count of samples still active copied to pinned host memory.
template <class T>
int pcg_iteration(mlmc_ctx* ctx, std::vector<Level<T>>& L, int B, SolveState& S, T* x, T* r, T* p, T* q,
                  double tol2) {
  const int n = L[0].n;
  const double sz = sizeof(T), d = dofs(n) * B, e = elems(n) * B;
  hipStream_t st = ctx->st;
  const int var = zv<T>(ctx);
  uint32_t np = 0;
  T* z = nullptr;
  LAUNCH(kid<T>(MLMC_K_PCG_APPLY), (2 * d + e) * sz, launch_pcg_apply_dot<T>(n, B, L[0].kap, p, q, S, &np, st, var));
  LAUNCH(MLMC_K_REDUCE, 0, launch_reduce(B, RED_ALPHA, 0.0, np, S, nullptr, st));
  LAUNCH(kid<T>(MLMC_K_PCG_UPDATE), 6 * d * sz, launch_pcg_update<T>(n, B, x, p, r, q, S, &np, st));
  LAUNCH(MLMC_K_REDUCE, 0, launch_reduce(B, RED_RR, tol2, np, S, nullptr, st));
  if (int rc = precondition<T>(ctx, L, B, r, &z, S, &np)) return rc;
  if (!np) LAUNCH(kid<T>(MLMC_K_PCG_DOT), 2 * d * sz, (launch_dot<T>(n, B, r, z, S, &np, st)));
  LAUNCH(MLMC_K_REDUCE, 0, launch_reduce(B, RED_BETA, 0.0, np, S, nullptr, st));
  LAUNCH(kid<T>(MLMC_K_PCG_DIRECTION), 3 * d * sz, launch_pcg_direction<T>(n, B, z, p, S, st));
  LAUNCH(MLMC_K_MISC, 0, launch_count_active(B, S, st));
  HIPCHK(hipMemcpyAsync(ctx->h_nactive, S.nactive, sizeof(int), hipMemcpyDeviceToHost, st));
  return MLMC_OK;
}

// PCG on the current iterate x with residual r (both already set, S.active
// and S.bb set).  Stops per sample at ||r|| <= tol ||b|| (recurrence).
// `graph` caches the captured iteration for this work space (may be null).
template <class T>
int pcg(mlmc_ctx* ctx, std::vector<Level<T>>& L, int B, SolveState& S, T* x, T* r, T* p, T* q, double tol,
        int max_iter, int* done_iters, hipGraphExec_t* graph) {
  const int n = L[0].n;
  const double sz = sizeof(T), d = dofs(n) * B;
  hipStream_t st = ctx->st;
  uint32_t np = 0;
  T* z = nullptr;
  if (int rc = precondition<T>(ctx, L, B, r, &z, S, &np)) return rc;
  if (!np) LAUNCH(kid<T>(MLMC_K_PCG_DOT), 2 * d * sz, (launch_dot<T>(n, B, r, z, S, &np, st)));
  LAUNCH(MLMC_K_REDUCE, 0, launch_reduce(B, RED_RZ_INIT, 0.0, np, S, nullptr, st));
  LAUNCH(kid<T>(MLMC_K_PCG_DIRECTION), 2 * d * sz, launch_copy<T>(n, B, z, p, S, st));
  const double tol2 = tol * tol;
  const bool use_graph = graph && ctx->use_graphs && !ctx->profiling;
  if (use_graph && !*graph) {
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    const int rc = pcg_iteration<T>(ctx, L, B, S, x, r, p, q, tol2);
    const hipError_t ec = hipStreamEndCapture(st, &g);
    if (rc) {
      if (g) hipGraphDestroy(g);
      return rc;
    }
    HIPCHK(ec);
    const hipError_t ei = hipGraphInstantiate(graph, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    HIPCHK(ei);
  }
  int it = 0;
  while (it < max_iter) {
    const int k = use_graph ? std::min(ctx->graph_batch, max_iter - it) : 1;
    for (int j = 0; j < k; ++j) {
      if (use_graph) {
        HIPCHK(hipGraphLaunch(*graph, st));
      } else if (int rc = pcg_iteration<T>(ctx, L, B, S, x, r, p, q, tol2)) {
        return rc;
      }
    }
    it += k;
    HIPCHK(hipStreamSynchronize(st));
    if (*ctx->h_nactive == 0) break;
  }
  *done_iters = it;
  return MLMC_OK;
}

// kap32_ready: the fp32 copy of kap is already in the fp32 hierarchy (mixed precision)
int solve_impl(mlmc_ctx* ctx, SolveWork& w, const double* kap, double* u, int32_t* iters_host, bool* all_conv,
               bool kap32_ready = false) {
  const int n = w.n, B = w.B;
  hipStream_t st = ctx->st;
  const double h = 1.0 / n, h3 = h * h * h;
  const double rtol = ctx->cfg.rtol;
  const size_t S0 = grid_stride(n);
  const double d = dofs(n) * B, e = elems(n) * B;
  SolveState& O = w.outer.s;
  uint32_t np = 0;
  LAUNCH(MLMC_K_MISC, 0, launch_set_active(B, O, 1, st));
  HIPCHK(hipMemsetAsync(O.iters, 0, B * sizeof(int), st));
  int total_it = 0;
  if (w.precision == MLMC_PREC_FP64) {
    auto& L = w.L64;
    L[0].kap = const_cast<double*>(kap);
    for (size_t l = 1; l < L.size(); ++l)
      LAUNCH(MLMC_K_COARSEN, (elems(L[l - 1].n) + elems(L[l].n)) * B * 8,
             launch_coarsen<double>(L[l - 1].n, B, L[l - 1].kap, L[l].kap, st));
    LAUNCH(MLMC_K_MISC, d * 8, launch_fill_interior<double>(n, B, u, 0.0, nullptr, st));
    LAUNCH(MLMC_K_MISC, d * 8, launch_fill_interior<double>(n, B, w.r, h3, nullptr, st));
    LAUNCH(MLMC_K_PCG_DOT, 2 * d * 8, (launch_dot<double>(n, B, w.r, w.r, O, &np, st)));
    LAUNCH(MLMC_K_REDUCE, 0, launch_reduce(B, RED_BB, 0.0, np, O, nullptr, st));
    for (int round = 0; round < 4 && total_it < ctx->cfg.max_iter; ++round) {
      int it = 0;
      if (int rc = pcg<double>(ctx, L, B, O, u, w.r, w.p, w.q, rtol, ctx->cfg.max_iter - total_it, &it,
                              &w.iter_exec[0]))
        return rc;
      total_it += it;
      // confirm with the true residual; samples above tolerance continue
      LAUNCH(MLMC_K_MISC, 0, launch_set_active(B, O, 1, st));
      LAUNCH(MLMC_K_TRUE_RESIDUAL, (2 * d + e) * 8, launch_true_residual(n, B, kap, h3, u, w.r, O, &np, st, zv<double>(ctx)));
      LAUNCH(MLMC_K_REDUCE, 0, launch_reduce(B, RED_RR, rtol * rtol, np, O, nullptr, st));
      int na = 0;
      if (int rc = count_active(ctx, O, B, &na)) return rc;
      if (na == 0) break;
    }
  } else {
    auto& L = w.L32;
    SolveState& I = w.inner.s;
    if (!kap32_ready)
      LAUNCH(MLMC_K_MISC, e * 12, (launch_convert<double, float>((size_t)B * elem_count(n), kap, L[0].kap, st)));
    for (size_t l = 1; l < L.size(); ++l)
      LAUNCH(kid<float>(MLMC_K_COARSEN), (elems(L[l - 1].n) + elems(L[l].n)) * B * 4,
             launch_coarsen<float>(L[l - 1].n, B, L[l - 1].kap, L[l].kap, st));
    LAUNCH(MLMC_K_MISC, d * 8, launch_fill_interior<double>(n, B, u, 0.0, nullptr, st));
    LAUNCH(MLMC_K_MISC, d * 8, launch_fill_interior<double>(n, B, w.r64, h3, nullptr, st));
    LAUNCH(MLMC_K_PCG_DOT, 2 * d * 8, (launch_dot<double>(n, B, w.r64, w.r64, O, &np, st)));
    LAUNCH(MLMC_K_REDUCE, 0, launch_reduce(B, RED_BB, 0.0, np, O, nullptr, st));
    HIPCHK(hipMemsetAsync(I.iters, 0, B * sizeof(int), st));
    for (int outer = 0; outer < kMaxOuter && total_it < ctx->cfg.max_iter; ++outer) {
      LAUNCH(MLMC_K_MISC, d * 12, launch_demote(n, B, w.r64, w.rin, O, st));
      HIPCHK(hipMemcpyAsync(I.active, O.active, B * sizeof(int), hipMemcpyDeviceToDevice, st));
      LAUNCH(MLMC_K_MISC, d * 4, launch_fill_interior<float>(n, B, w.d, 0.0, O.active, st));
      LAUNCH(kid<float>(MLMC_K_PCG_DOT), 2 * d * 4, (launch_dot<float>(n, B, w.rin, w.rin, I, &np, st)));
      LAUNCH(MLMC_K_REDUCE, 0, launch_reduce(B, RED_BB, 0.0, np, I, nullptr, st));
      int it = 0;
      if (int rc = pcg<float>(ctx, L, B, I, w.d, w.rin, w.p32, w.q32, kInnerRtol, ctx->cfg.max_iter - total_it, &it,
                             &w.iter_exec[1]))
        return rc;
      total_it += it;
      LAUNCH(MLMC_K_MISC, d * 20, launch_add_correction(n, B, u, w.d, O, st));
      LAUNCH(MLMC_K_TRUE_RESIDUAL, (2 * d + e) * 8, launch_true_residual(n, B, kap, h3, u, w.r64, O, &np, st, zv<double>(ctx)));
      LAUNCH(MLMC_K_REDUCE, 0, launch_reduce(B, RED_RR, rtol * rtol, np, O, nullptr, st));
      int na = 0;
      if (int rc = count_active(ctx, O, B, &na)) return rc;
      if (na == 0) break;
    }
    // report inner iterations as the sample's iteration count
    HIPCHK(hipMemcpyAsync(O.iters, I.iters, B * sizeof(int), hipMemcpyDeviceToDevice, st));
  }
  std::vector<int> act(B);
  HIPCHK(hipMemcpyAsync(act.data(), O.active, B * sizeof(int), hipMemcpyDeviceToHost, st));
  if (iters_host) HIPCHK(hipMemcpyAsync(iters_host, O.iters, B * sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  bool ok = true;
  for (int b = 0; b < B; ++b) ok = ok && act[b] == 0;
  *all_conv = ok;
  return MLMC_OK;
}

int qoi_impl(mlmc_ctx* ctx, SolveState& S, int n, int B, const double* u, double* q) {
  uint32_t np = 0;
  LAUNCH(MLMC_K_QOI, dofs(n) * B * 8, launch_qoi_partial(n, B, ctx->cfg.qoi, u, S, &np, ctx->st));
  LAUNCH(MLMC_K_REDUCE, 0, launch_reduce(B, RED_STORE, 0.0, np, S, q, ctx->st));
  return MLMC_OK;
}

bool mesh_of_config(const mlmc_ctx* ctx, int n) { return ctx->d_tab.count(n) > 0; }

}  // namespace

extern "C" {

size_t mlmc_grid_stride(int32_t n) { return n >= 2 ? grid_stride(n) : 0; }

const char* mlmc_last_error(const mlmc_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

int mlmc_create(const mlmc_config* cfg, mlmc_ctx** out) {
  if (!out) return MLMC_E_INVALID;
  *out = nullptr;
  std::string why;
  if (int rc = validate(cfg, why)) {
    g_create_error = why;
    return rc;
  }
  auto* ctx = new mlmc_ctx();
  ctx->cfg = *cfg;
  if (ctx->cfg.cheb_degree == 0) ctx->cfg.cheb_degree = 2;
  ctx->st = (hipStream_t)cfg->stream;
  if (!ctx->st) {
    // graphs cannot be captured on the legacy null stream: use a blocking stream
    // of default priority (ordered with the null stream both ways)
    if (hipStreamCreate(&ctx->st) != hipSuccess) {
      g_create_error = "cannot create a stream";
      delete ctx;
      return MLMC_E_DEVICE;
    }
    ctx->own_stream = true;
  }
  ctx->modes = kl_select(cfg->corr_len, cfg->sigma2, cfg->n_modes);
  ctx->K1 = (int)ctx->modes.omega.size();
  ctx->cheb = cheb_coeffs(ctx->cfg.cheb_degree, kChebHi / kChebRatio, kChebHi);
  if (const char* zvs = std::getenv("MLMC_ZVAR")) ctx->zvar[0] = ctx->zvar[1] = std::atoi(zvs);
  if (const char* gs = std::getenv("MLMC_GRAPHS"))
    if (std::atoi(gs) == 0) ctx->use_graphs = false;
  if (const char* vs = std::getenv("MLMC_VSMALL"))
    if (std::atoi(vs) == 0) ctx->vsmall_n0[0] = ctx->vsmall_n0[1] = 0;
  ctx->stats.assign(cfg->levels, Running{});
  const size_t need = persistent_bytes(cfg, ctx->K1);
  if (need > cfg->arena_bytes) {
    g_create_error = "arena smaller than the " + std::to_string(need) + " bytes of KL tables";
    if (ctx->own_stream) hipStreamDestroy(ctx->st);
    delete ctx;
    return MLMC_E_NOMEM;
  }
  Carver cv;
  cv.base = (char*)cfg->arena;
  cv.cap = cfg->arena_bytes;
  cv.dry = false;
  ctx->d_sqrtlam = cv.take<double>(cfg->n_modes);
  ctx->d_triples = cv.take<int>(3 * (size_t)cfg->n_modes);
  std::vector<double> sq(cfg->n_modes);
  for (int m = 0; m < cfg->n_modes; ++m) sq[m] = std::sqrt(ctx->modes.lambda[m]);
  hipError_t e = hipMemcpyAsync(ctx->d_sqrtlam, sq.data(), sq.size() * sizeof(double), hipMemcpyHostToDevice, ctx->st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ctx->d_triples, ctx->modes.triples.data(), ctx->modes.triples.size() * sizeof(int),
                       hipMemcpyHostToDevice, ctx->st);
  std::vector<std::vector<double>> tabs;
  for (int l = 0; l < cfg->levels && e == hipSuccess; ++l) {
    const int n = cfg->n0 << l;
    tabs.push_back(kl_centroid_table(ctx->modes, n));
    double* d = cv.take<double>((size_t)n * ctx->K1);
    ctx->d_tab[n] = d;
    e = hipMemcpyAsync(d, tabs.back().data(), tabs.back().size() * sizeof(double), hipMemcpyHostToDevice, ctx->st);
  }
  if (e == hipSuccess) e = hipHostMalloc((void**)&ctx->h_nactive, sizeof(int), hipHostMallocDefault);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->st);
  if (e != hipSuccess) {
    g_create_error = std::string("HIP error during create: ") + hipGetErrorString(e);
    if (ctx->h_nactive) hipHostFree(ctx->h_nactive);
    if (ctx->own_stream) hipStreamDestroy(ctx->st);
    delete ctx;
    return MLMC_E_DEVICE;
  }
  ctx->persistent_top = cv.top;
  *out = ctx;
  return MLMC_OK;
}

void mlmc_destroy(mlmc_ctx* ctx) {
  if (!ctx) return;
  hipStreamSynchronize(ctx->st);
  for (auto& r : ctx->prof) {
    hipEventDestroy(r.a);
    hipEventDestroy(r.b);
  }
  for (auto e : ctx->event_pool) hipEventDestroy(e);
  ctx->sw.release_graphs();
  ctx->bw.wf.release_graphs();
  ctx->bw.wc.release_graphs();
  if (ctx->h_nactive) hipHostFree(ctx->h_nactive);
  if (ctx->own_stream) hipStreamDestroy(ctx->st);
  delete ctx;
}

size_t mlmc_workspace_bytes(const mlmc_config* cfg, int32_t level, int32_t batch) {
  std::string why;
  if (validate(cfg, why) || level < 0 || level >= cfg->levels || batch < 1) return 0;
  const KLModes md = kl_select(cfg->corr_len, cfg->sigma2, cfg->n_modes);
  mlmc_config c = *cfg;
  if (c.cheb_degree == 0) c.cheb_degree = 2;
  Carver dry;
  dry.top = persistent_bytes(&c, (int)md.omega.size());
  BatchWork w;
  carve_batch(dry, w, c, level, batch);
  return dry.top;
}

int mlmc_modes(const mlmc_ctx* ctx, int32_t* triples, double* lambda) {
  if (!ctx) return MLMC_E_INVALID;
  const int M = ctx->cfg.n_modes;
  if (triples) std::memcpy(triples, ctx->modes.triples.data(), 3 * (size_t)M * sizeof(int32_t));
  if (lambda) std::memcpy(lambda, ctx->modes.lambda.data(), (size_t)M * sizeof(double));
  return MLMC_OK;
}

int mlmc_draw_xi(mlmc_ctx* ctx, int32_t level, uint64_t first, int64_t count, double* xi) {
  if (!ctx) return MLMC_E_INVALID;
  if (count < 0 || (count > 0 && !xi) || level < 0) FAIL(MLMC_E_INVALID, "bad draw_xi arguments");
  LAUNCH(MLMC_K_XI, (double)count * ctx->cfg.n_modes * 8,
         launch_draw_xi(ctx->cfg.seed, level, first, count, ctx->cfg.n_modes, xi, ctx->st));
  return MLMC_OK;
}

int mlmc_field(mlmc_ctx* ctx, int32_t n, int64_t count, const double* xi, double* kappa, float* kappa32) {
  if (!ctx) return MLMC_E_INVALID;
  if (count < 0 || count > (1 << 30) || (count > 0 && (!xi || !kappa))) FAIL(MLMC_E_INVALID, "bad field arguments");
  if (!mesh_of_config(ctx, n)) FAIL(MLMC_E_INVALID, "mesh " + std::to_string(n) + " is not a level mesh");
  if (count == 0) return MLMC_OK;
  return field_impl(ctx, n, (int)count, xi, kappa, kappa32);
}

int mlmc_apply(mlmc_ctx* ctx, int32_t n, int64_t count, const double* kappa, const double* u, double* y) {
  if (!ctx) return MLMC_E_INVALID;
  if (n < 2 || !is_pow2(n) || count < 0 || count > (1 << 30) || (count > 0 && (!kappa || !u || !y)) ||
      (count > 0 && u == y))
    FAIL(MLMC_E_INVALID, "bad apply arguments");
  if (count == 0) return MLMC_OK;
  LAUNCH(MLMC_K_APPLY, (2 * dofs(n) + elems(n)) * count * 8,
         launch_apply<double>(n, (int)count, kappa, u, y, nullptr, ctx->st));
  return MLMC_OK;
}

int mlmc_vcycle(mlmc_ctx* ctx, int32_t n, int64_t count, const double* kappa, const double* r, double* z) {
  if (!ctx) return MLMC_E_INVALID;
  if (n < 2 || !is_pow2(n) || count < 1 || count > (1 << 30) || !kappa || !r || !z)
    FAIL(MLMC_E_INVALID, "bad vcycle arguments");
  const int B = (int)count;
  mlmc_config saved = ctx->cfg;
  ctx->cfg.precision = MLMC_PREC_FP64;
  ctx->cfg.solver = MLMC_SOLVER_GMG_PCG;
  int rc = ensure_solve_work(ctx, n, B);
  ctx->cfg = saved;
  if (rc) return rc;
  auto& L = ctx->sw.L64;
  L[0].kap = const_cast<double*>(kappa);
  hipStream_t st = ctx->st;
  for (size_t l = 1; l < L.size(); ++l)
    LAUNCH(MLMC_K_COARSEN, 0, launch_coarsen<double>(L[l - 1].n, B, L[l - 1].kap, L[l].kap, st));
  LAUNCH(MLMC_K_MISC, 0, launch_set_active(B, ctx->sw.outer.s, 1, st));
  double* res = nullptr;
  if ((rc = vcycle<double>(ctx, L, 0, B, r, L[0].x, L[0].xo, L[0].t, ctx->sw.outer.s.active, &res))) return rc;
  HIPCHK(hipMemcpyAsync(z, res, (size_t)B * grid_stride(n) * sizeof(double), hipMemcpyDeviceToDevice, st));
  return MLMC_OK;
}

int mlmc_solve(mlmc_ctx* ctx, int32_t n, int64_t count, const double* kappa, double* u, int32_t* iters) {
  if (!ctx) return MLMC_E_INVALID;
  if (n < 2 || !is_pow2(n) || count < 1 || count > (1 << 30) || !kappa || !u)
    FAIL(MLMC_E_INVALID, "bad solve arguments");
  if (int rc = ensure_solve_work(ctx, n, (int)count)) return rc;
  bool conv = false;
  if (int rc = solve_impl(ctx, ctx->sw, kappa, u, iters, &conv)) return rc;
  if (!conv) FAIL(MLMC_E_NOCONV, "some samples did not reach rtol within max_iter");
  return MLMC_OK;
}

int mlmc_qoi(mlmc_ctx* ctx, int32_t n, int64_t count, const double* u, double* q) {
  if (!ctx) return MLMC_E_INVALID;
  if (n < 2 || !is_pow2(n) || count < 1 || count > (1 << 30) || !u || !q) FAIL(MLMC_E_INVALID, "bad qoi arguments");
  if (ctx->cfg.qoi == 1 && n % 4) FAIL(MLMC_E_INVALID, "subcube QoI needs 4 | n");
  if (int rc = ensure_solve_work(ctx, n, (int)count)) return rc;
  return qoi_impl(ctx, ctx->sw.outer.s, n, (int)count, u, q);
}

int mlmc_sample_level(mlmc_ctx* ctx, int32_t level, uint64_t first, uint64_t count, double* y, double* q_fine,
                      double* q_coarse, int32_t* iters) {
  if (!ctx) return MLMC_E_INVALID;
  if (level < 0 || level >= ctx->cfg.levels) FAIL(MLMC_E_INVALID, "level out of range");
  if (count > 0 && (!y || !q_fine || !q_coarse)) FAIL(MLMC_E_INVALID, "NULL output array");
  const int nf = ctx->cfg.n0 << level;
  if (ctx->cfg.qoi == 1 && ((nf % 4) || (level > 0 && (nf / 2) % 4)))
    FAIL(MLMC_E_INVALID, "subcube QoI needs 4 | n on both meshes");
  bool all_conv = true, finite = true;
  const auto t_start = std::chrono::steady_clock::now();
  for (uint64_t done = 0; done < count;) {
    const int B = (int)std::min<uint64_t>(count - done, (uint64_t)ctx->cfg.max_batch);
    if (int rc = ensure_batch_work(ctx, level, B)) return rc;
    BatchWork& w = ctx->bw;
    const uint64_t start = first + done;
    LAUNCH(MLMC_K_XI, (double)B * ctx->cfg.n_modes * 8,
           launch_draw_xi(ctx->cfg.seed, level, start, B, ctx->cfg.n_modes, w.xi, ctx->st));
    const bool mixed = ctx->cfg.precision == MLMC_PREC_MIXED;
    if (int rc = field_impl(ctx, nf, B, w.xi, w.kf, mixed ? w.wf.L32[0].kap : nullptr)) return rc;
    bool conv = false;
    if (int rc = solve_impl(ctx, w.wf, w.kf, w.uf, iters ? iters + done : nullptr, &conv, mixed)) return rc;
    all_conv = all_conv && conv;
    if (int rc = qoi_impl(ctx, w.wf.outer.s, nf, B, w.uf, w.qf)) return rc;
    if (level > 0) {
      if (int rc = field_impl(ctx, nf / 2, B, w.xi, w.kc, mixed ? w.wc.L32[0].kap : nullptr)) return rc;
      if (int rc = solve_impl(ctx, w.wc, w.kc, w.uc, nullptr, &conv, mixed)) return rc;
      all_conv = all_conv && conv;
      if (int rc = qoi_impl(ctx, w.wc.outer.s, nf / 2, B, w.uc, w.qc)) return rc;
    }
    HIPCHK(hipMemcpyAsync(q_fine + done, w.qf, B * sizeof(double), hipMemcpyDeviceToHost, ctx->st));
    if (level > 0)
      HIPCHK(hipMemcpyAsync(q_coarse + done, w.qc, B * sizeof(double), hipMemcpyDeviceToHost, ctx->st));
    HIPCHK(hipStreamSynchronize(ctx->st));
    const double cost = dofs(nf) + (level > 0 ? dofs(nf / 2) : 0.0);
    for (int b = 0; b < B; ++b) {
      if (level == 0) q_coarse[done + b] = 0.0;
      y[done + b] = q_fine[done + b] - q_coarse[done + b];
      finite = finite && std::isfinite(y[done + b]);
      ctx->stats[level].push(y[done + b]);
    }
    ctx->stats[level].cost = cost;
    done += (uint64_t)B;
  }
  if (count) {
    Running& r = ctx->stats[level];
    r.seconds += std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    r.timed += count;
    r.next = std::max(r.next, first + count);
  }
  if (!finite) FAIL(MLMC_E_NONFINITE, "non-finite QoI");
  if (!all_conv) FAIL(MLMC_E_NOCONV, "some samples did not reach rtol within max_iter");
  return MLMC_OK;
}

int mlmc_get_estimate(const mlmc_ctx* ctx, mlmc_estimate_out* out) {
  if (!ctx || !out) return MLMC_E_INVALID;
  std::memset(out, 0, sizeof(*out));
  out->levels = std::min(16, ctx->cfg.levels);
  for (int l = 0; l < out->levels; ++l) {
    const Running& r = ctx->stats[l];
    auto& o = out->level[l];
    o.n = r.n;
    o.mean = r.mean;
    o.m2 = r.m2;
    o.var = r.n ? r.m2 / (double)r.n : 0.0;
    o.cost = r.cost;
    out->qtilde += r.mean;
    if (r.n) out->var_qtilde += o.var / (double)r.n;
  }
  return MLMC_OK;
}

int mlmc_estimate(mlmc_ctx* ctx, const mlmc_estimate_opts* o, uint64_t* n_per_level, mlmc_estimate_out* out) {
  if (!ctx) return MLMC_E_INVALID;
  if (!o || !(o->eps > 0.0) || o->n_pilot < 2 || o->cost_model < 0 || o->cost_model > 1 || !(o->extra_fraction >= 0.0) ||
      o->max_rounds < 1)
    FAIL(MLMC_E_INVALID, "bad estimate options");
  const int L = ctx->cfg.levels;
  auto cost_of = [&](int l) {
    const Running& r = ctx->stats[l];
    if (o->cost_model == 1 || r.timed == 0) {
      const int nf = ctx->cfg.n0 << l;
      return dofs(nf) + (l > 0 ? dofs(nf / 2) : 0.0);
    }
    return r.seconds / (double)r.timed;
  };
  std::vector<uint64_t> target(L, 0);
  // pilot
  for (int l = 0; l < L; ++l) {
    const uint64_t have = ctx->stats[l].n;
    target[l] = std::max<uint64_t>(have, (uint64_t)o->n_pilot);
  }
  for (int round = 0; round <= o->max_rounds; ++round) {
    bool more = false;
    for (int l = 0; l < L; ++l) {
      const uint64_t have = ctx->stats[l].n;
      if (target[l] > have) {
        more = true;
        const uint64_t need = target[l] - have;
        std::vector<double> y(need), qf(need), qc(need);
        const int rc = mlmc_sample_level(ctx, l, ctx->stats[l].next, need, y.data(), qf.data(), qc.data(), nullptr);
        if (rc != MLMC_OK && rc != MLMC_E_NOCONV) return rc;
      }
    }
    if (!more && round > 0) break;
    if (round == o->max_rounds) break;
    // eq. mlmc_num_samples on the current estimates
    double tot = 0.0;
    std::vector<double> V(L), C(L);
    for (int l = 0; l < L; ++l) {
      const Running& r = ctx->stats[l];
      V[l] = r.n ? r.m2 / (double)r.n : 0.0;
      C[l] = cost_of(l);
      tot += std::sqrt(V[l] * C[l]);
    }
    bool grow = false;
    for (int l = 0; l < L; ++l) {
      const double nl = 2.0 / (o->eps * o->eps) * std::sqrt(V[l] / C[l]) * tot * (1.0 + o->extra_fraction);
      const uint64_t want = std::max<uint64_t>((uint64_t)std::ceil(nl), (uint64_t)o->n_pilot);
      if (want > target[l]) {
        target[l] = want;
        grow = true;
      }
    }
    if (!grow) break;
  }
  for (int l = 0; l < L; ++l) {
    ctx->stats[l].cost = cost_of(l);
    if (n_per_level) n_per_level[l] = ctx->stats[l].n;
  }
  if (out) return mlmc_get_estimate(ctx, out);
  return MLMC_OK;
}

int mlmc_reset_stats(mlmc_ctx* ctx) {
  if (!ctx) return MLMC_E_INVALID;
  ctx->stats.assign(ctx->cfg.levels, Running{});
  return MLMC_OK;
}

int mlmc_set_profiling(mlmc_ctx* ctx, int32_t on) {
  if (!ctx) return MLMC_E_INVALID;
  HIPCHK(hipStreamSynchronize(ctx->st));
  for (auto& r : ctx->prof) {
    ctx->event_pool.push_back(r.a);
    ctx->event_pool.push_back(r.b);
  }
  ctx->prof.clear();
  std::fill(std::begin(ctx->k_launch), std::end(ctx->k_launch), 0);
  std::fill(std::begin(ctx->k_ms), std::end(ctx->k_ms), 0.0);
  std::fill(std::begin(ctx->k_bytes), std::end(ctx->k_bytes), 0.0);
  ctx->profiling = on != 0;
  return MLMC_OK;
}

int mlmc_kernel_time(mlmc_ctx* ctx, int32_t kernel_id, int32_t precision, int64_t* launches, double* total_ms,
                     double* bytes) {
  if (!ctx || kernel_id < 0 || kernel_id >= MLMC_K_COUNT || precision < 0 || precision > 1) return MLMC_E_INVALID;
  HIPCHK(hipStreamSynchronize(ctx->st));
  for (auto& r : ctx->prof) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, r.a, r.b));
    ctx->k_launch[r.id] += 1;
    ctx->k_ms[r.id] += ms;
    ctx->k_bytes[r.id] += r.bytes;
    ctx->event_pool.push_back(r.a);
    ctx->event_pool.push_back(r.b);
  }
  ctx->prof.clear();
  const int slot = kernel_id + precision * MLMC_K_COUNT;
  if (launches) *launches = ctx->k_launch[slot];
  if (total_ms) *total_ms = ctx->k_ms[slot];
  if (bytes) *bytes = ctx->k_bytes[slot];
  return MLMC_OK;
}

}  // extern "C"
