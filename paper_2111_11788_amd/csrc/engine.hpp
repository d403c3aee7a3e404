// Internal engine of the MLMC library: context, arena carving, batched
// GMG-PCG solves (fp64 and fp32-in-fp64 refinement), the whole-path sample
// runner and the tuning knobs.  Shared by the C-ABI (api.cpp) and the serving
// loop (serve.cpp); not part of the public interface.
#pragma once

#include "mlmc.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "common.hpp"
#include "grid.hpp"
#include "kernels.hpp"
#include "kl_host.hpp"

struct mlmc_server;
struct mlmc_ctx;

namespace mlmc {
namespace eng {


// Upper end of the smoothing interval of D^-1 A.  Gershgorin bounds the
// spectrum by 2 (every off-diagonal of the Q1 element matrix is <= 0); the
// constant-coefficient symbol peaks at 1.5.  1.75 keeps the degree-1 and
// degree-2 residual polynomials below 1 in magnitude up to 2 (0.83 and 0.62),
// and measured best on the 64^3 batch (2.0: 5.83e9, 1.75: 5.93e9, 1.6: 5.88e9
// sample-DOFs/s; on 256^3, 1.6 was faster still but leaves |p(2)| = 1 at
// degree 1)
constexpr double kChebHi = 1.75;
constexpr double kChebRatio = 4.0;   // smoothing interval [hi / ratio, hi]
constexpr double kInnerRtol = 1e-4;  // fp32 inner solve tolerance (mixed precision)
constexpr int kMaxOuter = 30;
constexpr int kMaxLevelBatch = 65536;   // samples per batch on a coarse level (see level_cap)

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
inline ChebCoeffs cheb_coeffs(int degree, double lo, double hi) {
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
    s.pstate = cv.take<int>(B);
    s.began = cv.take<int>(B);
  }
};

// Work space of one batched solve on an n^3 mesh.
struct SolveWork {
  int n = 0, B = 0, precision = 0, solver = 0;
  std::vector<Level<double>> L64;   // fp64 hierarchy (level 0 kappa is the caller's)
  std::vector<Level<float>> L32;    // fp32 hierarchy (mixed precision)
  double *r = nullptr, *r2 = nullptr, *p = nullptr, *p2 = nullptr, *q = nullptr;   // fp64 PCG (r2, p2: second buffers)
  double* r64 = nullptr;                                    // fp64 refinement residual
  float *d = nullptr, *rin = nullptr, *rin2 = nullptr, *p32 = nullptr, *p32b = nullptr, *q32 = nullptr;  // fp32 inner PCG
  int* alt = nullptr;   // mixed: 1 where the sample's last refined iterate is in r64 (second buffer)
  StateBufs outer, inner;
  // captured PCG iteration per precision (0: fp64, 1: fp32); tied to the buffers above
  hipGraphExec_t iter_exec[2] = {nullptr, nullptr};

  void release_graphs() {
    for (auto& g : iter_exec)
      if (g) {
        (void)hipGraphExecDestroy(g);
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
      r2 = cv.take<double>(B * S0);
      p = cv.take<double>(B * S0);
      p2 = cv.take<double>(B * S0);
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
      alt = cv.take<int>(B);
      r64 = cv.take<double>(B * S0);
      d = cv.take<float>(B * S0);
      rin = cv.take<float>(B * S0);
      rin2 = cv.take<float>(B * S0);
      p32 = cv.take<float>(B * S0);
      p32b = cv.take<float>(B * S0);
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

// Work space of one task: a batched solve of B samples of MLMC level `level`
// on one mesh n (the level's own mesh or, for level > 0, its coarse partner
// n/2 on the same draws): draws, field, solution, QoIs, solver vectors, and
// for the random forcing xi_f, the element values of f and the load vector.
struct MeshWork {
  int level = -1, n = 0, B = 0;
  double* xi = nullptr;
  double *kap = nullptr, *u = nullptr, *q = nullptr;
  double *xif = nullptr, *fe = nullptr, *bvec = nullptr;
  SolveWork sw;
  void carve(Carver& cv, const mlmc_config& c, int level_, int n_, int B_) {
    level = level_;
    n = n_;
    B = B_;
    xi = cv.take<double>((size_t)B * c.n_modes);
    kap = cv.take<double>((size_t)B * elem_count(n));
    u = cv.take<double>((size_t)B * grid_stride(n));
    q = cv.take<double>(B);
    sw.carve(cv, n, B, c.precision, c.solver);
    if (c.forcing == MLMC_FORCING_LOGNORMAL) {
      xif = cv.take<double>((size_t)B * c.n_modes);
      fe = cv.take<double>((size_t)B * elem_count(n));
      bvec = cv.take<double>((size_t)B * grid_stride(n));
    }
  }
};

// A part of a task: `count` samples of `level` from sample index `first`, on
// the level's own mesh (which = 0) or the coarse mesh of its pair (1); `req`
// indexes the level request and `off` the samples' position in it.
struct Part {
  int level = 0, which = 0, req = 0;
  uint64_t first = 0, off = 0;
  int count = 0;
};

// One task of a sampling round: a batched solve of its parts' samples, in
// order, on mesh n, on lane `lane` (parts of different levels on the same mesh
// share the task when packing is on).
struct Task {
  int n = 0, lane = 0, count = 0;
  double work = 0.0;   // estimated cost: interior DOFs x samples
  std::vector<Part> parts;
};

// A level's share of a round: samples first .. first+count-1 of `level`;
// host outputs (each may be null) of count entries.
struct LevelReq {
  int level = 0;
  uint64_t first = 0, count = 0;
  double *y = nullptr, *qf = nullptr, *qc = nullptr;
  int32_t* iters = nullptr;
};

// Device record of a level's running statistics (eq. sample_variance,
// eq. mlmc_average), folded in push order: the Chan et al. merge, in block
// order, of every complete block of kStatsBlock consecutive pushes (n, mean,
// m2) and the Welford state of the incomplete block (pn, pmean, pm2); the
// result therefore does not depend on how the pushes were split into batches.
// Non-finite values are counted and not pushed.
struct DevStats {
  double n, mean, m2, pn, pmean, pm2;
  unsigned long long nonfinite, pad;
};
static_assert(sizeof(DevStats) == 64, "device statistics record");

// One timed launch.  `cnt` >= 0 indexes the device count of active samples
// taken just before a masked launch: its bytes count the active share only.
struct ProfRec {
  int id;
  hipEvent_t a, b;
  double bytes;
  int cnt, B;
};

struct Running {
  uint64_t n = 0;            // host mirror of the device record (read after each round)
  double mean = 0.0, m2 = 0.0, cost = 0.0;
  uint64_t nonfinite = 0;
  double seconds = 0.0;     // lane time spent sampling this level
  uint64_t timed = 0;       // samples covered by `seconds`
  uint64_t next = 0;        // next unused sample index of the level
};

}  // namespace eng
}  // namespace mlmc

using namespace mlmc;
using namespace mlmc::eng;

struct mlmc_ctx {
  mlmc_config cfg{};
  hipStream_t st = nullptr;
  std::string err;
  KLModes modes;
  int K1 = 0;
  double* d_sqrtlam = nullptr;
  int* d_triples = nullptr;
  int* d_xperm = nullptr;         // the modes ordered by their x-factor (stable)
  int* d_xoff = nullptr;          // [K1 + 1]: modes of x-factor a at d_xperm[xoff[a] .. xoff[a + 1])
  int field_kernel = 0;           // mlmc_tuning.field
  std::map<int, double*> d_tab;
  size_t persistent_top = 0;
  ChebCoeffs cheb;
  // cached work space (one at a time)
  int ws_kind = -1;              // 0: solve work, 1: batch work
  std::tuple<int, int, int, int> ws_key{-1, -1, -1, -1};
  SolveWork sw;
  std::vector<Running> stats;
  DevStats* d_stats = nullptr;    // [levels] device records of the level statistics (persistent arena)
  // lanes of the sampling rounds: lane 0 runs on this context's stream, lane
  // i > 0 on a sub-context with its own stream, pinned counter and host thread
  std::vector<std::unique_ptr<struct LaneState>> lanes;
  int n_lanes = 4;                // mlmc_tuning.lanes: concurrent lanes of a round (1: one after another)
  std::vector<Task> last_plan;    // tasks of the last round, in assignment order
  double last_busy = 0.0, last_wall = 0.0;   // lane-seconds busy and wall seconds of the last call's rounds
  int last_lanes = 1;
  bool profiling = false;
  std::vector<ProfRec> prof;
  std::vector<hipEvent_t> event_pool;
  int* prof_counts = nullptr;     // device (persistent arena): active-sample counts of masked timed launches
  int prof_used = 0;
  static constexpr int kProfCap = 1 << 16;
  int64_t k_launch[2 * MLMC_K_COUNT] = {0};   // [precision][kernel]
  double k_ms[2 * MLMC_K_COUNT] = {0}, k_bytes[2 * MLMC_K_COUNT] = {0};
  int* h_nactive = nullptr;
  // stencil engine variant bits for fp64 / fp32 (fp32: the LDS engine also for
  // the corrected post-smoothing step, measured faster on the 64^3 batch)
  int zvar[2] = {ZVAR_LDS, ZVAR_LDS | ZVAR_LDS_PRO};
  int vsmall_n0[2] = {8, 16};     // mesh at which the single-kernel coarse V-cycle takes over (0: off)
  bool use_graphs = true;         // replay the PCG iteration from a captured hipGraph
  bool own_stream = false;        // the context created st itself
  int graph_batch = 2;            // graph launches per convergence check
  // MLMC_FUSE_* bits in use: all but RUPDATE, which measured slower on the
  // 64^3 batch (its convergence test moves into the next iteration's first
  // kernel, so each solve runs one more residual restriction) and is left to
  // the autotuner
  int fuse = MLMC_FUSE_PROLONG | MLMC_FUSE_UPDATE | MLMC_FUSE_REFINE | MLMC_FUSE_RESTRICT | MLMC_FUSE_PRESMOOTH |
             MLMC_FUSE_DIRECTION | MLMC_FUSE_SOLVE | MLMC_FUSE_PACK;
  mlmc_server* server = nullptr;  // serving pools and threads while serving
  int device = 0;                 // the GPU current at creation
  void* scratch = nullptr;        // device address of that GPU's static scratch (mlmc_qoi_noalloc)
};

// A lane of the sampling rounds: its engine view (null for lane 0, which runs
// on the context itself), its work space (a region of the arena) and the
// layout carved there, kept while the next task has the same layout.
struct LaneState {
  std::unique_ptr<mlmc_ctx> sub;
  MeshWork w;
  size_t offset = 0, bytes = 0;     // region of the arena
  std::tuple<int, int, int> key{-1, -1, -1};   // (level, n, B) of the carved layout
  std::vector<int> tasks;           // indices into the round's task list
  double busy = 0.0;                // seconds spent on tasks in the current round
  int rc = MLMC_OK;
  int status = MLMC_OK;             // worst solve status of its tasks (NOCONV, NONFINITE)
};

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

namespace mlmc {
namespace eng {

hipEvent_t take_event(mlmc_ctx* ctx);

template <class F>
int launch(mlmc_ctx* ctx, int id, double bytes, const int* mask, int B, F&& f) {
  hipEvent_t a = nullptr, b = nullptr;
  int cnt = -1;
  if (ctx->profiling) {
    if (mask && ctx->prof_counts && ctx->prof_used < mlmc_ctx::kProfCap) {
      cnt = ctx->prof_used++;
      const hipError_t ec = launch_count_mask(mask, B, ctx->prof_counts + cnt, ctx->st);
      if (ec != hipSuccess) {
        ctx->err = std::string("kernel launch failed: ") + hipGetErrorString(ec);
        return MLMC_E_DEVICE;
      }
    }
    a = take_event(ctx);
    b = take_event(ctx);
    if (!a || !b || hipEventRecord(a, ctx->st) != hipSuccess) {
      ctx->err = "profiling event failed";
      return MLMC_E_DEVICE;
    }
  }
  const hipError_t e = f();
  if (e != hipSuccess) {
    ctx->err = std::string("kernel launch failed: ") + hipGetErrorString(e);
    return MLMC_E_DEVICE;
  }
  if (ctx->profiling) {
    if (hipEventRecord(b, ctx->st) != hipSuccess) {
      ctx->err = "profiling event failed";
      return MLMC_E_DEVICE;
    }
    ctx->prof.push_back(ProfRec{id, a, b, bytes, cnt, B});
  }
  return MLMC_OK;
}

}  // namespace eng
}  // namespace mlmc

#define LAUNCH(id, bytes, call)                          \
  do {                                                   \
    int rc_ = launch(ctx, (id), (double)(bytes), nullptr, 0, [&] { return (call); }); \
    if (rc_) return rc_;                                 \
  } while (0)

// A launch whose kernel skips the samples with mask[b] == 0 (B samples).
#define LAUNCHM(id, bytes, mask, nb, call)               \
  do {                                                   \
    int rc_ = launch(ctx, (id), (double)(bytes), (mask), (nb), [&] { return (call); }); \
    if (rc_) return rc_;                                 \
  } while (0)

namespace mlmc {
namespace eng {

// profiling slot of kernel `id` in the precision of T (fp32 slots follow the fp64 ones)
template <class T>
constexpr int kid(int id) { return id + (sizeof(T) == 4 ? MLMC_K_COUNT : 0); }
template <class T>
int zv(const mlmc_ctx* ctx) { return ctx->zvar[sizeof(T) == 4 ? 1 : 0]; }

inline double dofs(int n) { return (double)(n - 1) * (n - 1) * (n - 1); }
inline double elems(int n) { return (double)n * n * n; }

int validate(const mlmc_config* c, std::string& why);
size_t persistent_bytes(const mlmc_config* c, int K1);
int ensure_solve_work(mlmc_ctx* ctx, int n, int B);
// Drop every cached work space (the step-level one and the lanes'), with the
// graphs captured on them: the caller is about to use the arena after the
// persistent tables for something else.
void drop_work(mlmc_ctx* ctx);
size_t mesh_work_bytes(const mlmc_config& c, int level, int n, int B);
int ensure_tables(mlmc_ctx* ctx, int n, double** tab);
// The PCG residual update r -= alpha q fused into the first kernel of the next
// iteration's V-cycle (level 0, pre-smoothed residual restriction): q, the
// second residual buffer (the first is the V-cycle's right-hand side), the
// reduce op and tolerance of the convergence test that follows it.  `first`
// only sets the byte count (no update on a solve's first iteration).
template <class T>
struct RUpdate {
  const T* q = nullptr;
  T* r1 = nullptr;
  int rr_op = RED_RR_UPD;
  double tol2 = 0.0;
  bool first = false;
};
// whether the fp64 KLE of `count` samples takes the separable evaluation (mlmc_tuning.field)
bool field_separable(const mlmc_ctx* ctx, int64_t count);
// exact: fp64 whatever the precision (the forcing's field)
int field_impl(mlmc_ctx* ctx, int n, int B, const double* xi, double* kap, float* kap32, bool exact = false);
// One V-cycle on levels l.. of L; returns the buffer that holds the result.
// With `dot` the last smoothing step of level l also writes the partial sums
// of b . result (*dot_np per sample).  zero_done: x already holds the first
// (zero-iterate) smoothing step of level l (see zero_step_fusable).
template <class T>
int vcycle(mlmc_ctx* ctx, std::vector<Level<T>>& L, int l, int B, const T* b, T* x, T* xo, T* t,
           const int* active, T** result, SolveState* dot = nullptr, uint32_t* dot_np = nullptr,
           bool zero_done = false, const RUpdate<T>* ru = nullptr);
// z = M^-1 r.  When *fused_np is set on return, the partial sums of r . z
// are already in S.partial (GMG path); otherwise the caller computes them.
template <class T>
int precondition(mlmc_ctx* ctx, std::vector<Level<T>>& L, int B, const T* r, T** z, SolveState& S,
                 uint32_t* fused_np, bool zero_done = false, const RUpdate<T>* ru = nullptr);
// Whether the preconditioner's first smoothing step on the finest level runs
// through the level-by-level kernels, so a PCG update can produce it.
template <class T>
bool zero_step_fusable(const mlmc_ctx* ctx, const std::vector<Level<T>>& L, int B);
int count_active(mlmc_ctx* ctx, SolveState& s, int B, int* out);
template <class T>
int pcg_iteration(mlmc_ctx* ctx, std::vector<Level<T>>& L, int B, SolveState& S, T* x, T* r, T* p, T* q,
                  double tol2, int rr_op = RED_RR, bool count = true);
// Whether the PCG on this hierarchy runs with the direction fused into the
// operator apply (MLMC_FUSE_DIRECTION and the LDS engine usable on L[0]).
template <class T>
bool dir_fusable(const mlmc_ctx* ctx, const std::vector<Level<T>>& L, int B);
// Whether the fused-direction iteration also fuses its residual update into
// the next V-cycle (MLMC_FUSE_RUPDATE, and the pre-smoothed level 0).
template <class T>
bool rupd_fusable(const mlmc_ctx* ctx, const std::vector<Level<T>>& L, int B);
// One fused-direction PCG iteration: z = M^-1 r and beta; p = z + beta p
// (buffers p0/p1 by S.pstate), q = A p, alpha, and the previous x += alpha p;
// r -= alpha q with the convergence test.  The start of a solve sets S.pstate
// (launch_dir_begin) and, when the zero step is fused into the update, the
// zero-iterate smoothing step of the first V-cycle.  `first`: only for the
// byte count of the apply (no previous direction is read).
// r2 (may be null): the second residual buffer; with it and rupd_fusable the
// residual update r -= alpha q moves into the next iteration's V-cycle.
template <class T>
int pcg_iteration_dir(mlmc_ctx* ctx, std::vector<Level<T>>& L, int B, SolveState& S, T* x, T* r, T* p0, T* p1,
                      T* q, double tol2, int rr_op = RED_RR, bool count = true, bool first = false,
                      T* r2 = nullptr);
// Start of a fused-direction solve on the samples with mask[b] (see
// pcg_iteration_dir); fresh: x holds no value yet (it is written, not updated,
// by its first update, so it needs no zero fill).
template <class T>
int pcg_dir_begin(mlmc_ctx* ctx, std::vector<Level<T>>& L, int B, SolveState& S, const T* r, const int* mask,
                  bool fresh);
// PCG of x (residual r) to ||r|| <= tol ||b||.  With p2 (a second direction
// buffer) and dir_fusable, the fused-direction iteration runs (fresh as in
// pcg_dir_begin) and x gets its last update before return unless `defer`, in
// which case the caller applies it (S.pstate, S.alpha and the direction
// buffers describe it).
template <class T>
int pcg(mlmc_ctx* ctx, std::vector<Level<T>>& L, int B, SolveState& S, T* x, T* r, T* p, T* q, double tol,
        int max_iter, int* done_iters, hipGraphExec_t* graph, T* p2 = nullptr, bool fresh = false,
        bool defer = false, T* r2 = nullptr);
// kap32_ready: the fp32 copy of kap is already in the fp32 hierarchy (mixed precision)
// bvec: the right-hand side (grid layout, boundary positions 0), or NULL for f = 1
// *status: MLMC_OK when every sample reached rtol, MLMC_E_NONFINITE when some
// sample's residual became NaN or Inf (its solve stops there), else
// MLMC_E_NOCONV
int solve_impl(mlmc_ctx* ctx, SolveWork& w, const double* kap, double* u, int32_t* iters_host, int* status,
               bool kap32_ready = false, const double* bvec = nullptr);
// xi_f, f and the load vector b of B samples (first, level) on mesh n (random forcing)
int forcing_impl(mlmc_ctx* ctx, int n, int level, uint64_t first, int B, double* xif, double* f, double* b);
int qoi_impl(mlmc_ctx* ctx, SolveState& S, int n, int B, const double* u, double* q);
bool mesh_of_config(const mlmc_ctx* ctx, int n);
// Samples per lane batch of a level (the DOF budget of max_batch samples on
// the finest configured mesh, at most kMaxLevelBatch).
int level_cap(const mlmc_ctx* ctx, int level);
// Batch sizes of one level's request (eq. batch read for K lanes; see the
// definition) and the tasks of a round assigned to K lanes finest mesh first
// to the least-loaded lane (Alg. incremental_greedy).
std::vector<int> batch_plan(uint64_t count, int K, int cap, int fill);
// Samples of an n^3 mesh whose fp32 stencil launches reach kFillWaves waves
// (the occupancy from which the engine stops splitting a sample's planes over
// several workgroups)
int fill_batch(int n);
std::vector<Task> plan_round(const mlmc_ctx* ctx, const std::vector<LevelReq>& reqs, int K, const std::vector<int>& caps,
                             bool pack);
// One sampling round: every request's samples drawn, solved on both meshes of
// the pair and reduced to QoIs, the tasks spread over the lanes; with
// `record`, Y = Q_l - Q_{l-1} folded into the levels' device statistics in
// sample order.  Returns the worst status (NONFINITE before NOCONV) after all
// work is done.
int run_round(mlmc_ctx* ctx, std::vector<LevelReq>& reqs, bool record);
// Copy the device statistics of every level into ctx->stats (n, mean, m2).
int read_stats(mlmc_ctx* ctx);
int check_tuning(const mlmc_tuning* t, std::string& why);
mlmc_tuning current_tuning(const mlmc_ctx* ctx);
void apply_tuning(mlmc_ctx* ctx, const mlmc_tuning& t);

}  // namespace eng
}  // namespace mlmc
