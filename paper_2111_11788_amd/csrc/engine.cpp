// Engine of the MLMC library (see engine.hpp).
//
// Whole path of one batch (Sec. 2.2: a level-l sample evaluates the n_l and
// n_{l-1} meshes on one draw and contributes Y_l = Q_l - Q_{l-1}):
//   xi (Philox) -> kappa on each mesh (MFMA KLE) -> GMG-PCG solve per mesh ->
//   QoI -> Y -> running statistics of the level.
// Solver: conjugate gradients preconditioned by one V-cycle (Chebyshev-Jacobi
// smoothing, rediscretised coarse operators down to the 2^3 mesh).  Mixed
// precision runs that PCG in fp32 vectors (fp64 scalars) as the inner solver
// of an fp64 iterative refinement whose residual b - A x is formed in fp64.
#include "engine.hpp"

namespace mlmc {
namespace eng {

hipEvent_t take_event(mlmc_ctx* ctx) {
  if (!ctx->event_pool.empty()) {
    hipEvent_t e = ctx->event_pool.back();
    ctx->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Launch wrapper: optional event timing and algorithmic-byte accounting.

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
  if (c->precision < MLMC_PREC_FP64 || c->precision > MLMC_PREC_MIXED_BF16KLE) { why = "unknown precision"; return MLMC_E_INVALID; }
  if (c->solver != 0 && c->solver != 1) { why = "unknown solver"; return MLMC_E_INVALID; }
  if (c->cheb_degree < 0 || c->cheb_degree > 8) { why = "cheb_degree must be in 0..8"; return MLMC_E_INVALID; }
  if (c->max_batch < 1) { why = "max_batch must be >= 1"; return MLMC_E_INVALID; }
  if (c->forcing != MLMC_FORCING_CONSTANT && c->forcing != MLMC_FORCING_LOGNORMAL) {
    why = "unknown forcing";
    return MLMC_E_INVALID;
  }
  if (c->arena_bytes && !c->arena) { why = "arena_bytes > 0 with a NULL arena"; return MLMC_E_INVALID; }
  if (((uintptr_t)c->arena) % 256) { why = "arena must be 256-byte aligned"; return MLMC_E_INVALID; }
  return MLMC_OK;
}

size_t persistent_bytes(const mlmc_config* c, int K1) {
  Carver cv;
  cv.take<double>(c->n_modes);
  cv.take<int>(3 * (size_t)c->n_modes);
  cv.take<int>((size_t)c->n_modes);
  cv.take<int>((size_t)K1 + 1);
  cv.take<int>(mlmc_ctx::kProfCap);
  cv.take<DevStats>((size_t)c->levels);
  for (int l = 0; l < c->levels; ++l) cv.take<double>((size_t)(c->n0 << l) * K1);
  return cv.top;
}

void drop_work(mlmc_ctx* ctx) {
  ctx->sw.release_graphs();
  ctx->ws_kind = -1;
  for (auto& ln : ctx->lanes) {
    ln->w.sw.release_graphs();
    ln->key = std::make_tuple(-1, -1, -1);
  }
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
  drop_work(ctx);
  ctx->sw = SolveWork{};
  ctx->sw.carve(cv, n, B, ctx->cfg.precision, ctx->cfg.solver);
  HIPCHK(hipMemsetAsync((char*)ctx->cfg.arena + ctx->persistent_top, 0, cv.top - ctx->persistent_top, ctx->st));
  ctx->ws_kind = 0;
  ctx->ws_key = key;
  return MLMC_OK;
}

size_t mesh_work_bytes(const mlmc_config& c, int level, int n, int B) {
  Carver dry;
  MeshWork w;
  w.carve(dry, c, level, n, B);
  return dry.top;
}

int ensure_tables(mlmc_ctx* ctx, int n, double** tab) {
  auto it = ctx->d_tab.find(n);
  if (it == ctx->d_tab.end()) FAIL(MLMC_E_INVALID, "mesh " + std::to_string(n) + " is not a level mesh");
  *tab = it->second;
  return MLMC_OK;
}

bool field_separable(const mlmc_ctx* ctx, int64_t count) {
  (void)count;
  return ctx->field_kernel != 1;   // the launcher falls back to the GEMM when a block does not fit LDS
}

int field_impl(mlmc_ctx* ctx, int n, int B, const double* xi, double* kap, float* kap32, bool exact) {
  double* tab = nullptr;
  if (int rc = ensure_tables(ctx, n, &tab)) return rc;
  const int M = ctx->cfg.n_modes;
  LAUNCH(MLMC_K_FIELD, (double)B * elems(n) * (8.0 + (kap32 ? 4.0 : 0.0)) + (double)B * M * 8.0,
         launch_field(n, M, B, xi, ctx->d_sqrtlam, ctx->d_triples, tab, ctx->K1, kap, kap32, ctx->st, nullptr,
                      !exact && ctx->cfg.precision == MLMC_PREC_MIXED_BF16KLE,
                      field_separable(ctx, B) ? ctx->d_xperm : nullptr, ctx->d_xoff));
  return MLMC_OK;
}

int forcing_impl(mlmc_ctx* ctx, int n, int level, uint64_t first, int B, double* xif, double* f, double* b) {
  const int M = ctx->cfg.n_modes;
  LAUNCH(MLMC_K_XI, (double)B * M * 8, launch_draw_xi(ctx->cfg.seed, level, first, B, M, xif, ctx->st, 2));
  if (int rc = field_impl(ctx, n, B, xif, f, nullptr, true)) return rc;
  LAUNCH(MLMC_K_MISC, (double)B * (elems(n) + grid_stride(n)) * 8, launch_load(n, B, f, b, ctx->st));
  return MLMC_OK;
}

// One V-cycle on levels l.. of L; returns the buffer that holds the result.
// With `dot` the last smoothing step of level l also writes the partial sums
// of b . result (*dot_np per sample).
template <class T>
bool presmooth_level(const mlmc_ctx* ctx, int n, int B) {
  const int f = ctx->fuse;
  const int small = ctx->vsmall_n0[sizeof(T) == 4 ? 1 : 0];
  return (f & MLMC_FUSE_PRESMOOTH) && (f & MLMC_FUSE_PROLONG) && (f & MLMC_FUSE_RESTRICT) && ctx->cheb.degree == 1 &&
         (zv<T>(ctx) & ZVAR_LDS) && !(small && n <= small) && presmooth_usable<T>(n, B);
}

template <class T>
bool zero_step_fusable(const mlmc_ctx* ctx, const std::vector<Level<T>>& L, int B) {
  if (!(ctx->fuse & MLMC_FUSE_UPDATE) || L.size() < 2) return false;
  const int n = L[0].n;
  const int small = ctx->vsmall_n0[sizeof(T) == 4 ? 1 : 0];
  return n >= 4 && n >= ZV<T>::V && !(small && n <= small) && !presmooth_level<T>(ctx, n, B);
}

template <class T>
int vcycle(mlmc_ctx* ctx, std::vector<Level<T>>& L, int l, int B, const T* b, T* x, T* xo, T* t,
           const int* active, T** result, SolveState* dot, uint32_t* dot_np, bool zero_done,
           const RUpdate<T>* ru) {
  const int n = L[l].n;
  const double sz = sizeof(T);
  const double d = dofs(n) * B, e = elems(n) * B;
  hipStream_t st = ctx->st;
  const int var = zv<T>(ctx);
  if (n == 2) {
    LAUNCHM(kid<T>(MLMC_K_COARSEST), B * (8 + 2) * sz, active, B, launch_coarsest<T>(B, L[l].kap, b, x, active, st));
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
    LAUNCHM(kid<T>(MLMC_K_COARSEST), (2 * d + e * 8.0 / 7.0) * sz, active, B,
           launch_vsmall<T>(n, B, ch.degree, ch.c1, ch.c2, kl, b, x, active, st));
    *result = x;
    return MLMC_OK;
  }
  if (!zero_done && L.size() > (size_t)l + 1 && presmooth_level<T>(ctx, n, B)) {
    // one Chebyshev step on each side of the coarse-grid correction, the
    // first (from the zero iterate, c D^-1 b) formed inside both kernels that
    // read it instead of being stored
    Level<T>& nx = L[l + 1];
    const double dc = dofs(n / 2) * B;
    if (ru && dot) {
      // with the PCG residual update of the previous iteration (r -= alpha q,
      // written to the other residual buffer) and the convergence test on it
      uint32_t np = 0;
      LAUNCHM(kid<T>(MLMC_K_RESIDUAL_RESTRICT), ((ru->first ? 1 : 3) * d + e + dc) * sz, active, B,
              launch_residual_restrict_update<T>(n, B, kap, b, ru->r1, ru->q, nx.b, *dot, ch.c2[0], &np, st));
      LAUNCH(MLMC_K_REDUCE, 0, launch_reduce(B, ru->rr_op, ru->tol2, np, *dot, nullptr, st));
    } else {
      LAUNCHM(kid<T>(MLMC_K_RESIDUAL_RESTRICT), (d + e + dc) * sz, active, B,
              launch_residual_restrict<T>(n, B, kap, b, nullptr, nx.b, active, st, true, ch.c2[0]));
    }
    T* xc = nullptr;
    if (int rc = vcycle<T>(ctx, L, l + 1, B, nx.b, nx.x, nx.xo, nx.t, active, &xc)) return rc;
    LAUNCHM(kid<T>(MLMC_K_CHEB_PROLONG), (2 * d + dc + e) * sz, active, B,
            launch_cheb_prolong_presmoothed<T>(n, B, kap, b, xc, x, ch.c2[0], active, st, dot, dot_np,
                                               ru ? (const T*)ru->r1 : nullptr, ru && dot ? dot->pstate : nullptr));
    *result = x;
    return MLMC_OK;
  }
  if (!zero_done)
    LAUNCHM(kid<T>(MLMC_K_CHEB_ZERO), (2 * d + e) * sz, active, B,
            launch_cheb<T>(n, B, kap, b, nullptr, nullptr, x, 0.0, ch.c2[0], true, false, active, st, nullptr,
                           nullptr, var));
  T* cur = x;
  T* oth = xo;
  for (int s = 1; s < ch.degree; ++s) {
    const bool use_xo = s > 1;
    LAUNCHM(kid<T>(use_xo ? MLMC_K_CHEB_XO : MLMC_K_CHEB), ((use_xo ? 4 : 3) * d + e) * sz, active, B,
           launch_cheb<T>(n, B, kap, b, cur, oth, oth, ch.c1[s], ch.c2[s], false, use_xo, active, st, nullptr,
                          nullptr, var));
    std::swap(cur, oth);
  }
  Level<T>& nx = L[l + 1];
  const double dc = dofs(n / 2) * B;
  if ((ctx->fuse & MLMC_FUSE_RESTRICT) && resr_usable<T>(n, B)) {
    // the residual goes straight into the coarse right-hand side
    LAUNCHM(kid<T>(MLMC_K_RESIDUAL_RESTRICT), (2 * d + e + dc) * sz, active, B,
            launch_residual_restrict<T>(n, B, kap, b, cur, nx.b, active, st));
  } else {
    LAUNCHM(kid<T>(MLMC_K_RESIDUAL), (3 * d + e) * sz, active, B,
            launch_residual<T>(n, B, kap, b, cur, t, active, st, var));
    LAUNCHM(kid<T>(MLMC_K_RESTRICT), (d + dc) * sz, active, B, launch_restrict<T>(n, B, t, nx.b, active, st));
  }
  T* xc = nullptr;
  if (int rc = vcycle<T>(ctx, L, l + 1, B, nx.b, nx.x, nx.xo, nx.t, active, &xc)) return rc;
  int s0 = 0;
  if (ctx->fuse & MLMC_FUSE_PROLONG) {
    // first post-smoothing step reads cur + P xc; with more steps to come the
    // corrected iterate is kept in t (free after the restriction) as their
    // previous iterate
    const bool last = ch.degree == 1;
    T* save = last ? nullptr : t;
    LAUNCHM(kid<T>(MLMC_K_CHEB_PROLONG), ((last ? 3 : 4) * d + dc + e) * sz, active, B,
            launch_cheb_prolong<T>(n, B, kap, b, cur, xc, oth, save, ch.c2[0], active, st, last ? dot : nullptr,
                                   last ? dot_np : nullptr, var));
    cur = oth;
    oth = t;
    s0 = 1;
  } else {
    LAUNCHM(kid<T>(MLMC_K_PROLONG), (2 * d + dc) * sz, active, B, launch_prolong_add<T>(n, B, xc, cur, active, st));
  }
  for (int s = s0; s < ch.degree; ++s) {
    const bool use_xo = s > 0;
    const bool last = s == ch.degree - 1;
    LAUNCHM(kid<T>(use_xo ? MLMC_K_CHEB_XO : MLMC_K_CHEB), ((use_xo ? 4 : 3) * d + e) * sz, active, B,
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
                 uint32_t* fused_np, bool zero_done, const RUpdate<T>* ru) {
  const int n = L[0].n;
  *fused_np = 0;
  if (L.size() == 1 || n == 2) {
    if (n == 2) return vcycle<T>(ctx, L, 0, B, r, L[0].x, L[0].xo, L[0].t, S.active, z);
    // Jacobi: z = D^-1 r
    LAUNCHM(kid<T>(MLMC_K_CHEB_ZERO), (2 * dofs(n) + elems(n)) * B * sizeof(T), S.active, B,
           launch_cheb<T>(n, B, L[0].kap, r, nullptr, nullptr, L[0].x, 0.0, 1.0, true, false, S.active, ctx->st,
                          nullptr, nullptr, zv<T>(ctx)));
    *z = L[0].x;
    return MLMC_OK;
  }
  if (ru && !presmooth_level<T>(ctx, n, B)) FAIL(MLMC_E_INVALID, "the fused residual update needs the pre-smoothed level 0");
  return vcycle<T>(ctx, L, 0, B, r, L[0].x, L[0].xo, L[0].t, S.active, z, &S, fused_np, zero_done, ru);
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
                  double tol2, int rr_op, bool count) {
  const int n = L[0].n;
  const double sz = sizeof(T), d = dofs(n) * B, e = elems(n) * B;
  hipStream_t st = ctx->st;
  const int var = zv<T>(ctx);
  uint32_t np = 0;
  T* z = nullptr;
  LAUNCHM(kid<T>(MLMC_K_PCG_APPLY), (2 * d + e) * sz, S.active, B, launch_pcg_apply_dot<T>(n, B, L[0].kap, p, q, S, &np, st, var));
  LAUNCH(MLMC_K_REDUCE, 0, launch_reduce(B, RED_ALPHA, 0.0, np, S, nullptr, st));
  const bool fz = zero_step_fusable<T>(ctx, L, B);
  if (fz)
    LAUNCHM(kid<T>(MLMC_K_PCG_UPDATE_ZERO), (7 * d + e) * sz, S.active, B,
            launch_pcg_update_zero<T>(n, B, L[0].kap, x, p, r, q, L[0].x, ctx->cheb.c2[0], S, &np, st, var));
  else
    LAUNCHM(kid<T>(MLMC_K_PCG_UPDATE), 6 * d * sz, S.active, B, launch_pcg_update<T>(n, B, x, p, r, q, S, &np, st));
  LAUNCH(MLMC_K_REDUCE, 0, launch_reduce(B, rr_op, tol2, np, S, nullptr, st));
  if (int rc = precondition<T>(ctx, L, B, r, &z, S, &np, fz)) return rc;
  if (!np) LAUNCHM(kid<T>(MLMC_K_PCG_DOT), 2 * d * sz, S.active, B, (launch_dot<T>(n, B, r, z, S, &np, st)));
  LAUNCH(MLMC_K_REDUCE, 0, launch_reduce(B, RED_BETA, 0.0, np, S, nullptr, st));
  LAUNCHM(kid<T>(MLMC_K_PCG_DIRECTION), 3 * d * sz, S.active, B, launch_pcg_direction<T>(n, B, z, p, S, st));
  if (count) {
    LAUNCH(MLMC_K_MISC, 0, launch_count_active(B, S, st));
    HIPCHK(hipMemcpyAsync(ctx->h_nactive, S.nactive, sizeof(int), hipMemcpyDeviceToHost, st));
  }
  return MLMC_OK;
}

template <class T>
bool dir_fusable(const mlmc_ctx* ctx, const std::vector<Level<T>>& L, int B) {
  return (ctx->fuse & MLMC_FUSE_DIRECTION) && (zv<T>(ctx) & ZVAR_LDS) && dir_usable<T>(L[0].n, B);
}

template <class T>
bool rupd_fusable(const mlmc_ctx* ctx, const std::vector<Level<T>>& L, int B) {
  return (ctx->fuse & MLMC_FUSE_RUPDATE) && L.size() > 1 && dir_fusable<T>(ctx, L, B) &&
         presmooth_level<T>(ctx, L[0].n, B);
}

template <class T>
int pcg_dir_begin(mlmc_ctx* ctx, std::vector<Level<T>>& L, int B, SolveState& S, const T* r, const int* mask,
                  bool fresh) {
  const int n = L[0].n;
  const double sz = sizeof(T), d = dofs(n) * B, e = elems(n) * B;
  SolveState m = S;
  m.active = const_cast<int*>(mask);
  LAUNCH(MLMC_K_MISC, 0, launch_dir_begin(B, m, fresh, ctx->st));
  if (zero_step_fusable<T>(ctx, L, B))
    LAUNCHM(kid<T>(MLMC_K_CHEB_ZERO), (2 * d + e) * sz, mask, B,
            launch_cheb<T>(n, B, L[0].kap, r, nullptr, nullptr, L[0].x, 0.0, ctx->cheb.c2[0], true, false, mask,
                           ctx->st, nullptr, nullptr, zv<T>(ctx)));
  return MLMC_OK;
}

template <class T>
int pcg_iteration_dir(mlmc_ctx* ctx, std::vector<Level<T>>& L, int B, SolveState& S, T* x, T* r, T* p0, T* p1,
                      T* q, double tol2, int rr_op, bool count, bool first, T* r2) {
  const int n = L[0].n;
  const double sz = sizeof(T), d = dofs(n) * B, e = elems(n) * B;
  hipStream_t st = ctx->st;
  const int var = zv<T>(ctx);
  const bool fz = zero_step_fusable<T>(ctx, L, B);
  // the update r -= alpha q of the previous iteration inside this V-cycle
  const bool fru = r2 && rupd_fusable<T>(ctx, L, B);
  RUpdate<T> ru;
  ru.q = q;
  ru.r1 = r2;
  ru.rr_op = rr_op == RED_RR_INNER ? RED_RR_INNER_UPD : RED_RR_UPD;
  ru.tol2 = tol2;
  ru.first = first;
  uint32_t np = 0;
  T* z = nullptr;
  if (int rc = precondition<T>(ctx, L, B, r, &z, S, &np, fz, fru ? &ru : nullptr)) return rc;
  if (!np) LAUNCHM(kid<T>(MLMC_K_PCG_DOT), 2 * d * sz, S.active, B, (launch_dot<T>(n, B, r, z, S, &np, st)));
  LAUNCH(MLMC_K_REDUCE, 0, launch_reduce(B, RED_BETA_DIR, 0.0, np, S, nullptr, st));
  // reads z, kappa (and p_old, x); writes p, q (and x)
  LAUNCHM(kid<T>(MLMC_K_PCG_APPLY), ((first ? 3 : 6) * d + e) * sz, S.active, B,
          launch_pcg_dir_apply<T>(n, B, L[0].kap, z, x, p0, p1, q, S.pstate, S, &np, st));
  LAUNCH(MLMC_K_REDUCE, 0, launch_reduce(B, RED_ALPHA_DIR, 0.0, np, S, nullptr, st));
  if (!fru) {
    if (fz)
      LAUNCHM(kid<T>(MLMC_K_PCG_UPDATE_ZERO), (4 * d + e) * sz, S.active, B,
              launch_pcg_rupdate_zero<T>(n, B, L[0].kap, r, q, L[0].x, ctx->cheb.c2[0], S, &np, st, var));
    else
      LAUNCHM(kid<T>(MLMC_K_PCG_UPDATE), 3 * d * sz, S.active, B, launch_pcg_rupdate<T>(n, B, r, q, S, &np, st));
    LAUNCH(MLMC_K_REDUCE, 0, launch_reduce(B, rr_op, tol2, np, S, nullptr, st));
  }
  if (count) {
    LAUNCH(MLMC_K_MISC, 0, launch_count_active(B, S, st));
    HIPCHK(hipMemcpyAsync(ctx->h_nactive, S.nactive, sizeof(int), hipMemcpyDeviceToHost, st));
  }
  return MLMC_OK;
}

// PCG on the current iterate x with residual r (both already set, S.active
// and S.bb set).  Stops per sample at ||r|| <= tol ||b|| (recurrence).
// `graph` caches the captured iteration for this work space (may be null).
template <class T>
int pcg(mlmc_ctx* ctx, std::vector<Level<T>>& L, int B, SolveState& S, T* x, T* r, T* p, T* q, double tol,
        int max_iter, int* done_iters, hipGraphExec_t* graph, T* p2, bool fresh, bool defer, T* r2) {
  const int n = L[0].n;
  const double sz = sizeof(T), d = dofs(n) * B;
  hipStream_t st = ctx->st;
  const double tol2 = tol * tol;
  const bool use_graph = graph && ctx->use_graphs && !ctx->profiling;
  if (p2 && dir_fusable<T>(ctx, L, B)) {
    if (int rc = pcg_dir_begin<T>(ctx, L, B, S, r, S.active, fresh)) return rc;
    int it = 0;
    if (max_iter > 0) {
      if (int rc = pcg_iteration_dir<T>(ctx, L, B, S, x, r, p, p2, q, tol2, RED_RR, true, true, r2)) return rc;
      it = 1;
      HIPCHK(hipStreamSynchronize(st));
    }
    if (use_graph && !*graph && it < max_iter && *ctx->h_nactive > 0) {
      hipGraph_t g = nullptr;
      HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
      const int rc = pcg_iteration_dir<T>(ctx, L, B, S, x, r, p, p2, q, tol2, RED_RR, true, false, r2);
      const hipError_t ec = hipStreamEndCapture(st, &g);
      if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
      }
      HIPCHK(ec);
      const hipError_t ei = hipGraphInstantiate(graph, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);   // the instantiated graph does not need it
      HIPCHK(ei);
    }
    while (it < max_iter && *ctx->h_nactive > 0) {
      const int k = use_graph ? std::min(ctx->graph_batch, max_iter - it) : 1;
      for (int j = 0; j < k; ++j) {
        if (use_graph) {
          HIPCHK(hipGraphLaunch(*graph, st));
        } else if (int rc = pcg_iteration_dir<T>(ctx, L, B, S, x, r, p, p2, q, tol2, RED_RR, true, false, r2)) {
          return rc;
        }
      }
      it += k;
      HIPCHK(hipStreamSynchronize(st));
    }
    // the update the last step still owes its iterate (unless its consumer applies it)
    if (!defer)
      LAUNCHM(kid<T>(MLMC_K_PCG_UPDATE), 3 * d * sz, S.began, B, launch_pcg_finish<T>(n, B, x, p, p2, S.began, S, st));
    *done_iters = it;
    return MLMC_OK;
  }
  uint32_t np = 0;
  T* z = nullptr;
  if (int rc = precondition<T>(ctx, L, B, r, &z, S, &np)) return rc;
  if (!np) LAUNCHM(kid<T>(MLMC_K_PCG_DOT), 2 * d * sz, S.active, B, (launch_dot<T>(n, B, r, z, S, &np, st)));
  LAUNCH(MLMC_K_REDUCE, 0, launch_reduce(B, RED_RZ_INIT, 0.0, np, S, nullptr, st));
  LAUNCHM(kid<T>(MLMC_K_PCG_DIRECTION), 2 * d * sz, S.active, B, launch_copy<T>(n, B, z, p, S, st));
  if (use_graph && !*graph) {
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    const int rc = pcg_iteration<T>(ctx, L, B, S, x, r, p, q, tol2);
    const hipError_t ec = hipStreamEndCapture(st, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    HIPCHK(ec);
    const hipError_t ei = hipGraphInstantiate(graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);   // the instantiated graph does not need it
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
int solve_impl(mlmc_ctx* ctx, SolveWork& w, const double* kap, double* u, int32_t* iters_host, int* status,
               bool kap32_ready, const double* bvec) {
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
    if (bvec)
      HIPCHK(hipMemcpyAsync(w.r, bvec, (size_t)B * S0 * sizeof(double), hipMemcpyDeviceToDevice, st));
    else
      LAUNCH(MLMC_K_MISC, d * 8, launch_fill_interior<double>(n, B, w.r, h3, nullptr, st));
    LAUNCH(MLMC_K_PCG_DOT, 2 * d * 8, (launch_dot<double>(n, B, w.r, w.r, O, &np, st)));
    LAUNCH(MLMC_K_REDUCE, 0, launch_reduce(B, RED_BB, 0.0, np, O, nullptr, st));
    for (int round = 0; round < 4 && total_it < ctx->cfg.max_iter; ++round) {
      int it = 0;
      if (int rc = pcg<double>(ctx, L, B, O, u, w.r, w.p, w.q, rtol, ctx->cfg.max_iter - total_it, &it,
                              &w.iter_exec[0], w.p2, false, false, w.r2))
        return rc;
      total_it += it;
      // confirm with the true residual; samples above tolerance continue
      LAUNCH(MLMC_K_MISC, 0, launch_set_active(B, O, 1, st));
      LAUNCHM(MLMC_K_TRUE_RESIDUAL, ((bvec ? 3 : 2) * d + e) * 8, O.active, B,
              launch_true_residual(n, B, kap, h3, u, w.r, O, &np, st, zv<double>(ctx), bvec));
      LAUNCH(MLMC_K_REDUCE, 0, launch_reduce(B, RED_RR, rtol * rtol, np, O, nullptr, st));
      int na = 0;
      if (int rc = count_active(ctx, O, B, &na)) return rc;
      if (na == 0) break;
    }
  } else if ((ctx->fuse & MLMC_FUSE_SOLVE) && ctx->cfg.solver == MLMC_SOLVER_GMG_PCG && (n == 4 || n == 8) &&
             ctx->vsmall_n0[1] >= n) {
    // the whole solve of each sample in one workgroup (all vectors in LDS)
    const ChebCoeffs& ch = ctx->cheb;
    LAUNCH(MLMC_K_SOLVE_SMALL, (e * 8 + d * 8 * (bvec ? 2 : 1)),
           launch_solve_small(n, B, ch.degree, ch.c1, ch.c2, kap, bvec, h3, u, O.active, O.iters, rtol, kInnerRtol,
                              ctx->cfg.max_iter, kMaxOuter, st, O.rr));
  } else {
    auto& L = w.L32;
    SolveState& I = w.inner.s;
    if (!kap32_ready)
      LAUNCH(MLMC_K_MISC, e * 12, (launch_convert<double, float>((size_t)B * elem_count(n), kap, L[0].kap, st)));
    for (size_t l = 1; l < L.size(); ++l)
      LAUNCH(kid<float>(MLMC_K_COARSEN), (elems(L[l - 1].n) + elems(L[l].n)) * B * 4,
             launch_coarsen<float>(L[l - 1].n, B, L[l - 1].kap, L[l].kap, st));
    HIPCHK(hipMemsetAsync(I.iters, 0, B * sizeof(int), st));
    if (ctx->fuse & MLMC_FUSE_REFINE) {
      // Each refinement step writes u + d into the other of two fp64 buffers
      // (its neighbours' u is still being read), the residual of the result
      // demoted to fp32 as the next inner right-hand side, and its fp64 norm;
      // `alt` records which buffer holds each sample's last iterate.
      if (bvec) {   // rin = fp32(b); ||b||^2 from the fp64 b
        LAUNCH(MLMC_K_MISC, d * 12, launch_demote(n, B, bvec, w.rin, O, st));
        LAUNCH(MLMC_K_PCG_DOT, 2 * d * 8, (launch_dot<double>(n, B, bvec, bvec, O, &np, st)));
      } else {
        LAUNCH(MLMC_K_MISC, d * 4, launch_fill_interior<float>(n, B, w.rin, h3, nullptr, st));
        LAUNCH(kid<float>(MLMC_K_PCG_DOT), 2 * d * 4, (launch_dot<float>(n, B, w.rin, w.rin, O, &np, st)));
      }
      LAUNCH(MLMC_K_REDUCE, 0, launch_reduce(B, RED_BB, 0.0, np, O, nullptr, st));
      HIPCHK(hipMemsetAsync(w.alt, 0, B * sizeof(int), st));
      // the buffer written by the expected last step is u, so usually no copy
      // back is needed (steps ~ log(rtol) / log(inner rtol))
      const int expect = std::max(1, (int)std::ceil(std::log(rtol) / std::log(kInnerRtol) - 1e-9));
      double* bufs[2] = {u, w.r64};
      if ((expect - 1) % 2 == 1) std::swap(bufs[0], bufs[1]);
      const double* ucur = nullptr;   // zero iterate
      int next = 0;
      // fused direction: the inner correction starts fresh (no fill), and the
      // update its last step owes is applied by the refinement step
      const bool dir = dir_fusable<float>(ctx, L, B);
      const bool owed = dir && refine_owed_usable(n, B, zv<double>(ctx));
      for (int outer = 0; outer < kMaxOuter && total_it < ctx->cfg.max_iter; ++outer) {
        HIPCHK(hipMemcpyAsync(I.active, O.active, B * sizeof(int), hipMemcpyDeviceToDevice, st));
        // inner ||b||^2 = the sums just reduced for the outer residual
        SolveState Ib = I;
        Ib.partial = O.partial;
        Ib.pstride = O.pstride;
        LAUNCH(MLMC_K_REDUCE, 0, launch_reduce(B, RED_BB, 0.0, np, Ib, nullptr, st));
        if (!dir)
          LAUNCHM(MLMC_K_MISC, d * 4, O.active, B, launch_fill_interior<float>(n, B, w.d, 0.0, O.active, st));
        int it = 0;
        if (int rc = pcg<float>(ctx, L, B, I, w.d, w.rin, w.p32, w.q32, kInnerRtol, ctx->cfg.max_iter - total_it,
                               &it, &w.iter_exec[1], w.p32b, dir, owed, w.rin2))
          return rc;
        total_it += it;
        double* uout = bufs[next];
        const double bb_bytes = bvec ? 8 : 0;
        if (owed)   // reads u, d, p and kappa (and b); writes u + d, rin
          LAUNCHM(MLMC_K_TRUE_RESIDUAL, ((ucur ? 8 : 0) + 4 + 4 + 8 + 4 + bb_bytes) * d + 8 * e, O.active, B,
                  launch_refine_owed(n, B, kap, h3, ucur, w.d, w.p32, w.p32b, I, uout, w.rin, O, &np, st, bvec));
        else
          LAUNCHM(MLMC_K_TRUE_RESIDUAL, ((ucur ? 8 : 0) + 4 + 8 + 4 + bb_bytes) * d + 8 * e, O.active, B,
                  launch_refine(n, B, kap, h3, ucur, w.d, uout, w.rin, O, &np, st, zv<double>(ctx), bvec));
        LAUNCH(MLMC_K_MISC, 0, launch_set_phase_mask(B, O.active, w.alt, uout == w.r64 ? 1 : 0, nullptr, st));
        LAUNCH(MLMC_K_REDUCE, 0, launch_reduce(B, RED_RR, rtol * rtol, np, O, nullptr, st));
        ucur = uout;
        next ^= 1;
        int na = 0;
        if (int rc = count_active(ctx, O, B, &na)) return rc;
        if (na == 0) break;
      }
      SolveState moved = O;
      moved.active = w.alt;
      LAUNCH(MLMC_K_MISC, 0, launch_copy<double>(n, B, w.r64, u, moved, st));
    } else {
      LAUNCH(MLMC_K_MISC, d * 8, launch_fill_interior<double>(n, B, u, 0.0, nullptr, st));
      if (bvec)
        HIPCHK(hipMemcpyAsync(w.r64, bvec, (size_t)B * S0 * sizeof(double), hipMemcpyDeviceToDevice, st));
      else
        LAUNCH(MLMC_K_MISC, d * 8, launch_fill_interior<double>(n, B, w.r64, h3, nullptr, st));
      LAUNCH(MLMC_K_PCG_DOT, 2 * d * 8, (launch_dot<double>(n, B, w.r64, w.r64, O, &np, st)));
      LAUNCH(MLMC_K_REDUCE, 0, launch_reduce(B, RED_BB, 0.0, np, O, nullptr, st));
      for (int outer = 0; outer < kMaxOuter && total_it < ctx->cfg.max_iter; ++outer) {
        LAUNCHM(MLMC_K_MISC, d * 12, O.active, B, launch_demote(n, B, w.r64, w.rin, O, st));
        HIPCHK(hipMemcpyAsync(I.active, O.active, B * sizeof(int), hipMemcpyDeviceToDevice, st));
        const bool dir = dir_fusable<float>(ctx, L, B);   // a fused-direction correction starts fresh
        if (!dir)
          LAUNCHM(MLMC_K_MISC, d * 4, O.active, B, launch_fill_interior<float>(n, B, w.d, 0.0, O.active, st));
        LAUNCHM(kid<float>(MLMC_K_PCG_DOT), 2 * d * 4, I.active, B,
                (launch_dot<float>(n, B, w.rin, w.rin, I, &np, st)));
        LAUNCH(MLMC_K_REDUCE, 0, launch_reduce(B, RED_BB, 0.0, np, I, nullptr, st));
        int it = 0;
        if (int rc = pcg<float>(ctx, L, B, I, w.d, w.rin, w.p32, w.q32, kInnerRtol, ctx->cfg.max_iter - total_it, &it,
                               &w.iter_exec[1], w.p32b, dir, false, w.rin2))
          return rc;
        total_it += it;
        LAUNCHM(MLMC_K_MISC, d * 20, O.active, B, launch_add_correction(n, B, u, w.d, O, st));
        LAUNCHM(MLMC_K_TRUE_RESIDUAL, (2 * d + e) * 8, O.active, B,
                launch_true_residual(n, B, kap, h3, u, w.r64, O, &np, st, zv<double>(ctx), bvec));
        LAUNCH(MLMC_K_REDUCE, 0, launch_reduce(B, RED_RR, rtol * rtol, np, O, nullptr, st));
        int na = 0;
        if (int rc = count_active(ctx, O, B, &na)) return rc;
        if (na == 0) break;
      }
    }
    // report inner iterations as the sample's iteration count
    HIPCHK(hipMemcpyAsync(O.iters, I.iters, B * sizeof(int), hipMemcpyDeviceToDevice, st));
  }
  std::vector<int> act(B);
  std::vector<double> rr(B);
  HIPCHK(hipMemcpyAsync(act.data(), O.active, B * sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(rr.data(), O.rr, B * sizeof(double), hipMemcpyDeviceToHost, st));
  if (iters_host) HIPCHK(hipMemcpyAsync(iters_host, O.iters, B * sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  // the last outer residual tells a NaN / Inf stop from convergence
  int stat = MLMC_OK;
  for (int b = 0; b < B; ++b) {
    if (!std::isfinite(rr[b])) {
      stat = MLMC_E_NONFINITE;
      break;
    }
    if (act[b]) stat = MLMC_E_NOCONV;
  }
  *status = stat;
  return MLMC_OK;
}

int qoi_impl(mlmc_ctx* ctx, SolveState& S, int n, int B, const double* u, double* q) {
  uint32_t np = 0;
  const double m = ctx->cfg.qoi == 1 ? (double)(3 * n / 4 - n / 4 + 1) : 0.0;   // subcube nodes per axis
  LAUNCH(MLMC_K_QOI, (ctx->cfg.qoi == 1 ? m * m * m : dofs(n)) * B * 8,
         launch_qoi_partial(n, B, ctx->cfg.qoi, u, S, &np, ctx->st));
  LAUNCH(MLMC_K_REDUCE, 0, launch_reduce(B, RED_STORE, 0.0, np, S, q, ctx->st));
  return MLMC_OK;
}

bool mesh_of_config(const mlmc_ctx* ctx, int n) { return ctx->d_tab.count(n) > 0; }

// ------------------------------------------------------------ sampling rounds

int level_cap(const mlmc_ctx* ctx, int level) {
  const int top = ctx->cfg.levels - 1;
  auto pair = [&](int l) {
    const int nf = ctx->cfg.n0 << l;
    return dofs(nf) + (l > 0 ? dofs(nf / 2) : 0.0);
  };
  // max_batch samples on the finest configured mesh; a coarser level takes as
  // many samples as cost the same interior DOFs (at most kMaxLevelBatch), so
  // its small meshes are not solved in launch-bound slices
  const double cap = std::min((double)ctx->cfg.max_batch * std::max(1.0, pair(top) / pair(level)),
                              (double)kMaxLevelBatch);
  return std::max(ctx->cfg.max_batch, (int)cap);
}

int fill_batch(int n) {
  const ZGeom g = zgeom<float>(n, 1);
  if (g.G < 1) return kFillWaves;
  const int waves = g.row_blocks * (g.threads / 64);
  return (kFillWaves + waves - 1) / waves;
}

// eq. batch with p|q_l read as the K lanes a level's batches can run on: the
// next batch takes ceil((N - n) / K) of the N - n samples still unassigned,
// between ceil(0.01 ceil(N / K)) and ceil(phi^-1 ceil(N / K)) (phi the golden
// ratio), as the defaults the paper states; the minimum is raised to the
// samples that fill the device (`fill`, at most the capacity: smaller batches
// split their planes over more workgroups and re-read more halos) and every
// batch is capped by the lane capacity.  One lane has no other partition to
// leave work for: its batches are the capacity.
std::vector<int> batch_plan(uint64_t count, int K, int cap, int fill) {
  std::vector<int> out;
  const uint64_t C = (uint64_t)std::max(1, cap);
  if (K <= 1) {
    for (uint64_t n = 0; n < count;) {
      const uint64_t b = std::min(count - n, C);
      out.push_back((int)b);
      n += b;
    }
    return out;
  }
  const uint64_t k = (uint64_t)K;
  const uint64_t per = (count + k - 1) / k;
  const double phi_inv = (std::sqrt(5.0) - 1.0) / 2.0;
  const uint64_t hi = (uint64_t)std::ceil((double)per * phi_inv);
  const uint64_t lo = std::max<uint64_t>((per + 99) / 100, std::min<uint64_t>(C, (uint64_t)std::max(1, fill)));
  for (uint64_t n = 0; n < count;) {
    uint64_t b = (count - n + k - 1) / k;
    b = std::max(lo, std::min(hi, b));
    b = std::min(b, std::min(C, count - n));
    out.push_back((int)b);
    n += b;
  }
  return out;
}

// Tasks of a round (Alg. incremental_greedy on K lanes): every request is cut
// into batches (batch_plan), a batch of a level l > 0 into its fine-mesh and
// coarse-mesh solves.  With `pack`, the solves of two levels on the same mesh
// n (the coarse solves of level l+1 and the fine solves of level l) are paired
// in order, the i-th of one with the i-th of the other, into one task when
// together they fit the lane capacity of the level whose own mesh is n
// (`caps` holds the capacity of every level, indexed by level).  The
// tasks are taken by decreasing mesh (the finest first; on one mesh the
// finer level's first, then sample order) and each goes to the lane with the
// least estimated work so far (interior DOFs x samples; the lowest lane on
// ties).  Without packing a mesh's coarse solves all come before its fine ones.
std::vector<Task> plan_round(const mlmc_ctx* ctx, const std::vector<LevelReq>& reqs, int K,
                             const std::vector<int>& caps, bool pack) {
  std::vector<int> order(reqs.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return reqs[a].level > reqs[b].level; });
  const int n0 = ctx->cfg.n0;
  // solves of each mesh level m (mesh n0 << m): the coarse solves of level m+1, then the fine of level m
  const int nm = ctx->cfg.levels;
  std::vector<std::vector<Part>> coarse(nm), fine(nm);
  for (int r : order) {
    const LevelReq& q = reqs[r];
    uint64_t off = 0;
    for (int b : batch_plan(q.count, K, caps[q.level], fill_batch(n0 << q.level))) {
      Part p;
      p.level = q.level;
      p.req = r;
      p.first = q.first + off;
      p.off = off;
      p.count = b;
      p.which = 0;
      fine[q.level].push_back(p);
      if (q.level > 0) {
        p.which = 1;
        coarse[q.level - 1].push_back(p);
      }
      off += (uint64_t)b;
    }
  }
  std::vector<Task> ts;
  auto add = [&](int m, std::initializer_list<const Part*> ps) {
    Task t;
    t.n = n0 << m;
    for (const Part* p : ps) {
      t.parts.push_back(*p);
      t.count += p->count;
    }
    t.work = (double)t.count * dofs(t.n);
    ts.push_back(t);
  };
  for (int m = nm - 1; m >= 0; --m) {
    const auto& A = coarse[m];
    const auto& F = fine[m];
    const int cap = caps[m];
    if (!pack) {
      for (const Part& p : A) add(m, {&p});
      for (const Part& p : F) add(m, {&p});
      continue;
    }
    const size_t len = std::max(A.size(), F.size());
    for (size_t i = 0; i < len; ++i) {
      const bool ha = i < A.size(), hf = i < F.size();
      if (ha && hf && A[i].count + F[i].count <= cap) {
        add(m, {&A[i], &F[i]});
      } else {
        if (ha) add(m, {&A[i]});
        if (hf) add(m, {&F[i]});
      }
    }
  }
  std::vector<double> load(std::max(1, K), 0.0);
  for (Task& t : ts) {
    int best = 0;
    for (int i = 1; i < K; ++i)
      if (load[i] < load[best]) best = i;
    t.lane = best;
    load[best] += t.work;
  }
  return ts;
}

namespace {

int ensure_lanes(mlmc_ctx* ctx, int K) {
  while ((int)ctx->lanes.size() < K) {
    auto ln = std::make_unique<LaneState>();
    if (!ctx->lanes.empty()) {
      // lanes after the first: an engine view with its own stream (default
      // priority) and pinned counter
      auto sub = std::make_unique<mlmc_ctx>();
      if (hipStreamCreate(&sub->st) != hipSuccess) FAIL(MLMC_E_DEVICE, "cannot create a lane stream");
      sub->own_stream = true;
      if (hipHostMalloc((void**)&sub->h_nactive, sizeof(int), hipHostMallocDefault) != hipSuccess) {
        (void)hipStreamDestroy(sub->st);
        FAIL(MLMC_E_DEVICE, "cannot allocate a lane counter");
      }
      ln->sub = std::move(sub);
    }
    ctx->lanes.push_back(std::move(ln));
  }
  for (size_t i = 1; i < ctx->lanes.size(); ++i) {
    mlmc_ctx* s = ctx->lanes[i]->sub.get();
    s->cfg = ctx->cfg;
    s->K1 = ctx->K1;
    s->d_sqrtlam = ctx->d_sqrtlam;
    s->d_triples = ctx->d_triples;
    s->d_xperm = ctx->d_xperm;
    s->d_xoff = ctx->d_xoff;
    s->field_kernel = ctx->field_kernel;
    s->d_tab = ctx->d_tab;
    s->persistent_top = ctx->persistent_top;
    s->cheb = ctx->cheb;
    s->zvar[0] = ctx->zvar[0];
    s->zvar[1] = ctx->zvar[1];
    s->vsmall_n0[0] = ctx->vsmall_n0[0];
    s->vsmall_n0[1] = ctx->vsmall_n0[1];
    s->use_graphs = ctx->use_graphs;
    s->graph_batch = ctx->graph_batch;
    s->fuse = ctx->fuse;
    s->profiling = false;
  }
  return MLMC_OK;
}

// One task on a lane (ctx: the lane's engine view): draws of every part,
// forcing, field, solve and QoI of the task's samples on its mesh; each
// part's QoIs go to its slice of the round's buffers (dqf: the level's own
// mesh, dqc: the coarse one, offset base[req] + off), the iteration counts of
// the level's own solves to the request's host array.
int run_task(mlmc_ctx* ctx, LaneState& ln, const Task& t, const std::vector<LevelReq>& reqs,
             const std::vector<uint64_t>& base, double* dqf, double* dqc, int* status) {
  const mlmc_config& c = ctx->cfg;
  const int B = t.count;
  const auto key = std::make_tuple(0, t.n, B);
  if (ln.key != key) {
    ln.w.sw.release_graphs();
    ln.w = MeshWork{};
    Carver cv;
    cv.base = (char*)c.arena;
    cv.cap = c.arena_bytes;
    cv.top = ln.offset;
    cv.dry = false;
    ln.w.carve(cv, c, t.parts[0].level, t.n, B);
    // zero boundaries of every grid vector (kernels never write them)
    HIPCHK(hipMemsetAsync((char*)c.arena + ln.offset, 0, cv.top - ln.offset, ctx->st));
    ln.key = key;
  }
  MeshWork& w = ln.w;
  w.level = t.parts[0].level;
  const bool mixed = c.precision != MLMC_PREC_FP64;
  const bool forced = c.forcing == MLMC_FORCING_LOGNORMAL;
  const int M = c.n_modes;
  int o = 0;
  for (const Part& p : t.parts) {
    LAUNCH(MLMC_K_XI, (double)p.count * M * 8,
           launch_draw_xi(c.seed, p.level, p.first, p.count, M, w.xi + (size_t)o * M, ctx->st));
    if (forced)   // xi_f: the forcing's own coefficients (stream 2)
      LAUNCH(MLMC_K_XI, (double)p.count * M * 8,
             launch_draw_xi(c.seed, p.level, p.first, p.count, M, w.xif + (size_t)o * M, ctx->st, 2));
    o += p.count;
  }
  if (forced) {
    if (int rc = field_impl(ctx, t.n, B, w.xif, w.fe, nullptr, true)) return rc;
    LAUNCH(MLMC_K_MISC, (double)B * (elems(t.n) + grid_stride(t.n)) * 8, launch_load(t.n, B, w.fe, w.bvec, ctx->st));
  }
  if (int rc = field_impl(ctx, t.n, B, w.xi, w.kap, mixed ? w.sw.L32[0].kap : nullptr)) return rc;
  std::vector<int32_t> its(B);
  if (int rc = solve_impl(ctx, w.sw, w.kap, w.u, its.data(), status, mixed, forced ? w.bvec : nullptr)) return rc;
  if (int rc = qoi_impl(ctx, w.sw.outer.s, t.n, B, w.u, w.q)) return rc;
  o = 0;
  for (const Part& p : t.parts) {
    double* dq = (p.which ? dqc : dqf) + base[p.req] + p.off;
    HIPCHK(hipMemcpyAsync(dq, w.q + o, (size_t)p.count * sizeof(double), hipMemcpyDeviceToDevice, ctx->st));
    if (p.which == 0 && reqs[p.req].iters)
      std::memcpy(reqs[p.req].iters + p.off, its.data() + o, (size_t)p.count * sizeof(int32_t));
    o += p.count;
  }
  HIPCHK(hipStreamSynchronize(ctx->st));
  return MLMC_OK;
}

int worse(int a, int b) {
  if (a == MLMC_E_NONFINITE || b == MLMC_E_NONFINITE) return MLMC_E_NONFINITE;
  if (a == MLMC_E_NOCONV || b == MLMC_E_NOCONV) return MLMC_E_NOCONV;
  return MLMC_OK;
}

}  // namespace

int read_stats(mlmc_ctx* ctx) {
  const int L = ctx->cfg.levels;
  std::vector<DevStats> rec(L);
  HIPCHK(hipMemcpyAsync(rec.data(), ctx->d_stats, L * sizeof(DevStats), hipMemcpyDeviceToHost, ctx->st));
  HIPCHK(hipStreamSynchronize(ctx->st));
  for (int l = 0; l < L; ++l) {
    double n = rec[l].n, mean = rec[l].mean, m2 = rec[l].m2;
    chan_merge(n, mean, m2, rec[l].pn, rec[l].pmean, rec[l].pm2);
    Running& r = ctx->stats[l];
    r.n = (uint64_t)n;
    r.mean = mean;
    r.m2 = m2;
    r.nonfinite = rec[l].nonfinite;
  }
  return MLMC_OK;
}

int run_round(mlmc_ctx* ctx, std::vector<LevelReq>& reqs, bool record) {
  const mlmc_config& c = ctx->cfg;
  uint64_t total = 0;
  std::vector<uint64_t> base(reqs.size());
  for (size_t i = 0; i < reqs.size(); ++i) {
    for (size_t j = 0; j < i; ++j)
      if (reqs[j].level == reqs[i].level) FAIL(MLMC_E_INVALID, "a round takes each level once");
    base[i] = total;
    total += reqs[i].count;
  }
  if (total == 0) return MLMC_OK;
  if (total > ((uint64_t)1 << 31)) FAIL(MLMC_E_INVALID, "too many samples in one call");
  // the QoIs of every sample on both meshes, at the end of the arena
  const size_t qbytes = 2 * align256(total * sizeof(double));
  // lane capacity of each level, which also bounds a packed task on the level's own mesh
  std::vector<int> caps(c.levels);
  for (int l = 0; l < c.levels; ++l) caps[l] = level_cap(ctx, l);
  int K = ctx->profiling ? 1 : std::max(1, ctx->n_lanes);
  std::vector<Task> ts;
  std::vector<size_t> lane_bytes;
  for (;;) {
    ts = plan_round(ctx, reqs, K, caps, (ctx->fuse & MLMC_FUSE_PACK) != 0);
    lane_bytes.assign(K, 0);
    for (const Task& t : ts)
      lane_bytes[t.lane] = std::max(lane_bytes[t.lane], mesh_work_bytes(c, t.parts[0].level, t.n, t.count));
    size_t need = ctx->persistent_top + qbytes + 256;   // the QoI buffers start at a 256-byte boundary
    for (size_t b : lane_bytes) need += b;
    if (need <= c.arena_bytes) break;
    if (K > 1) {   // fewer lanes
      --K;
      continue;
    }
    bool shrunk = false;   // one lane: halve the batches down to max_batch
    for (int& cp : caps)
      if (cp > c.max_batch) {
        cp = std::max(c.max_batch, cp / 2);
        shrunk = true;
      }
    if (shrunk) continue;
    // still too large: the QoI buffers of a long request crowd out the batch;
    // run the first and second halves of every request as two rounds (the
    // statistics are folded in the same sample order)
    bool splittable = false;
    for (const LevelReq& q : reqs) splittable = splittable || q.count > (uint64_t)c.max_batch;
    if (!splittable)
      FAIL(MLMC_E_NOMEM, "arena too small for a batch of the round: need " + std::to_string(need) + " bytes");
    std::vector<LevelReq> a = reqs, b = reqs;
    for (size_t i = 0; i < reqs.size(); ++i) {
      const uint64_t h = reqs[i].count / 2;
      a[i].count = h;
      b[i].first += h;
      b[i].count -= h;
      if (b[i].y) b[i].y += h;
      if (b[i].qf) b[i].qf += h;
      if (b[i].qc) b[i].qc += h;
      if (b[i].iters) b[i].iters += h;
    }
    a.erase(std::remove_if(a.begin(), a.end(), [](const LevelReq& q) { return q.count == 0; }), a.end());
    const int ra = run_round(ctx, a, record);
    if (ra && ra != MLMC_E_NOCONV && ra != MLMC_E_NONFINITE) return ra;
    const std::string ea = ctx->err;
    const int rb = run_round(ctx, b, record);
    if (rb && rb != MLMC_E_NOCONV && rb != MLMC_E_NONFINITE) return rb;
    const int worst = worse(ra, rb);
    if (worst == ra && ra) ctx->err = ea;
    return worst;
  }
  if (int rc = ensure_lanes(ctx, K)) return rc;
  // the step-level work space shares the arena with the lanes
  ctx->sw.release_graphs();
  ctx->ws_kind = -1;
  size_t off = ctx->persistent_top;
  for (int i = 0; i < K; ++i) {
    LaneState& ln = *ctx->lanes[i];
    if (ln.offset != off || ln.bytes != lane_bytes[i]) {
      ln.w.sw.release_graphs();
      ln.key = std::make_tuple(-1, -1, -1);
      ln.offset = off;
      ln.bytes = lane_bytes[i];
    }
    ln.tasks.clear();
    off += lane_bytes[i];
  }
  for (size_t i = 0; i < ts.size(); ++i) ctx->lanes[ts[i].lane]->tasks.push_back((int)i);
  double* dqf = reinterpret_cast<double*>((char*)c.arena + (c.arena_bytes - qbytes) / 256 * 256);
  double* dqc = dqf + align256(total * sizeof(double)) / sizeof(double);
  // lanes start after the work queued so far on the context's stream
  if (K > 1) {
    hipEvent_t ev = take_event(ctx);
    HIPCHK(hipEventRecord(ev, ctx->st));
    for (int i = 1; i < K; ++i) HIPCHK(hipStreamWaitEvent(ctx->lanes[i]->sub->st, ev, 0));
    ctx->event_pool.push_back(ev);
  }
  std::vector<double> task_s(ts.size(), 0.0);
  auto body = [&](int i) {
    LaneState& ln = *ctx->lanes[i];
    mlmc_ctx* lc = i == 0 ? ctx : ln.sub.get();
    ln.busy = 0.0;
    ln.rc = MLMC_OK;
    ln.status = MLMC_OK;
    for (int ti : ln.tasks) {
      const Task& t = ts[ti];
      const auto t0 = std::chrono::steady_clock::now();
      int st = MLMC_OK;
      const int rc = run_task(lc, ln, t, reqs, base, dqf, dqc, &st);
      task_s[ti] = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      ln.busy += task_s[ti];
      if (rc) {
        ln.rc = rc;
        break;
      }
      ln.status = worse(ln.status, st);
    }
  };
  const auto w0 = std::chrono::steady_clock::now();
  std::vector<std::thread> th;
  for (int i = 1; i < K; ++i) th.emplace_back(body, i);
  body(0);
  for (auto& x : th) x.join();
  const double wall = std::chrono::duration<double>(std::chrono::steady_clock::now() - w0).count();
  ctx->last_plan = ts;
  ctx->last_wall += wall;
  ctx->last_lanes = K;
  int status = MLMC_OK;
  for (int i = 0; i < K; ++i) {
    LaneState& ln = *ctx->lanes[i];
    ctx->last_busy += ln.busy / K;
    if (ln.rc) {
      if (i > 0) ctx->err = ln.sub->err;
      drop_work(ctx);
      return ln.rc;
    }
    status = worse(status, ln.status);
  }
  // host outputs, then the statistics fold in sample order (one workgroup per level)
  for (size_t r = 0; r < reqs.size(); ++r) {
    const LevelReq& q = reqs[r];
    if (q.qf || q.y)
      HIPCHK(hipMemcpyAsync(q.qf ? q.qf : q.y, dqf + base[r], q.count * sizeof(double), hipMemcpyDeviceToHost, ctx->st));
    if (q.level > 0 && q.qc)
      HIPCHK(hipMemcpyAsync(q.qc, dqc + base[r], q.count * sizeof(double), hipMemcpyDeviceToHost, ctx->st));
  }
  if (record) {
    StatsJobs jobs{};
    int nj = 0;
    for (size_t r = 0; r < reqs.size(); ++r) {
      jobs.j[nj++] = StatsJob{dqf + base[r], reqs[r].level > 0 ? dqc + base[r] : nullptr, reqs[r].count,
                              reinterpret_cast<double*>(ctx->d_stats + reqs[r].level)};
      if (nj == kMaxStatsJobs || r + 1 == reqs.size()) {
        LAUNCH(MLMC_K_MISC, 0, launch_level_stats(nj, jobs, ctx->st));
        nj = 0;
      }
    }
  }
  HIPCHK(hipStreamSynchronize(ctx->st));
  for (size_t r = 0; r < reqs.size(); ++r) {
    LevelReq& q = reqs[r];
    if (q.level == 0 && q.qc) std::fill(q.qc, q.qc + q.count, 0.0);
    if (q.y && q.qf)
      for (uint64_t i = 0; i < q.count; ++i) q.y[i] = q.qf[i] - (q.level > 0 && q.qc ? q.qc[i] : 0.0);
    if (q.y && !q.qf && q.level > 0) {
      std::vector<double> qc(q.count);
      HIPCHK(hipMemcpyAsync(qc.data(), dqc + base[r], q.count * sizeof(double), hipMemcpyDeviceToHost, ctx->st));
      HIPCHK(hipStreamSynchronize(ctx->st));
      for (uint64_t i = 0; i < q.count; ++i) q.y[i] -= qc[i];
    }
    if (q.y)
      for (uint64_t i = 0; i < q.count; ++i)
        if (!std::isfinite(q.y[i])) status = MLMC_E_NONFINITE;
  }
  if (record) {
    std::vector<uint64_t> nf0(c.levels);
    for (int l = 0; l < c.levels; ++l) nf0[l] = ctx->stats[l].nonfinite;
    if (int rc = read_stats(ctx)) return rc;
    for (size_t r = 0; r < reqs.size(); ++r) {
      Running& R = ctx->stats[reqs[r].level];
      if (R.nonfinite != nf0[reqs[r].level]) status = MLMC_E_NONFINITE;
      const int nf = c.n0 << reqs[r].level;
      R.cost = dofs(nf) + (reqs[r].level > 0 ? dofs(nf / 2) : 0.0);
      R.timed += reqs[r].count;
      R.next = std::max(R.next, reqs[r].first + reqs[r].count);
    }
    // a task's time is shared by its parts by their samples
    for (size_t i = 0; i < ts.size(); ++i)
      for (const Part& p : ts[i].parts) ctx->stats[p.level].seconds += task_s[i] * p.count / ts[i].count;
  }
  if (status == MLMC_E_NONFINITE) FAIL(MLMC_E_NONFINITE, "a solve or QoI became NaN or Inf");
  if (status == MLMC_E_NOCONV) FAIL(MLMC_E_NOCONV, "some samples did not reach rtol within max_iter");
  return MLMC_OK;
}

int check_tuning(const mlmc_tuning* t, std::string& why) {
  if (!t) { why = "NULL tuning"; return MLMC_E_INVALID; }
  if (t->zvar_fp32 < 0 || t->zvar_fp32 > 7 || t->zvar_fp64 < 0 || t->zvar_fp64 > 7) { why = "zvar bits must be in 0..7"; return MLMC_E_INVALID; }
  auto okv = [](int v, int mx) { return v == 0 || (v >= 4 && v <= mx && (v & (v - 1)) == 0); };
  if (!okv(t->vsmall_fp32, 16) || !okv(t->vsmall_fp64, 8)) { why = "vsmall must be 0 or 4..16 (fp64 4..8), a power of two"; return MLMC_E_INVALID; }
  if (t->cheb_degree < 1 || t->cheb_degree > 8) { why = "cheb_degree must be in 1..8"; return MLMC_E_INVALID; }
  if (t->max_batch < 1) { why = "max_batch must be >= 1"; return MLMC_E_INVALID; }
  if (t->graph_batch < 0 || t->graph_batch > 16) { why = "graph_batch must be in 0..16"; return MLMC_E_INVALID; }
  if (t->field < 0 || t->field > 2) { why = "field must be 0 (auto), 1 (MFMA GEMM) or 2 (separable)"; return MLMC_E_INVALID; }
  if (t->lanes < 1 || t->lanes > 8) { why = "lanes must be in 1..8"; return MLMC_E_INVALID; }
  if (t->fuse & ~(MLMC_FUSE_PROLONG | MLMC_FUSE_UPDATE | MLMC_FUSE_REFINE | MLMC_FUSE_RESTRICT | MLMC_FUSE_PRESMOOTH |
                   MLMC_FUSE_DIRECTION | MLMC_FUSE_RUPDATE | MLMC_FUSE_SOLVE | MLMC_FUSE_PACK)) { why = "unknown fuse bits"; return MLMC_E_INVALID; }
  return MLMC_OK;
}

mlmc_tuning current_tuning(const mlmc_ctx* ctx) {
  mlmc_tuning t{};
  t.zvar_fp64 = ctx->zvar[0];
  t.zvar_fp32 = ctx->zvar[1];
  t.vsmall_fp64 = ctx->vsmall_n0[0];
  t.vsmall_fp32 = ctx->vsmall_n0[1];
  t.cheb_degree = ctx->cheb.degree;
  t.max_batch = ctx->cfg.max_batch;
  t.graph_batch = ctx->use_graphs ? ctx->graph_batch : 0;
  t.fuse = ctx->fuse;
  t.field = ctx->field_kernel;
  t.lanes = ctx->n_lanes;
  t.seconds = 0.0;
  return t;
}

void apply_tuning(mlmc_ctx* ctx, const mlmc_tuning& t) {
  ctx->zvar[0] = t.zvar_fp64;
  ctx->zvar[1] = t.zvar_fp32;
  ctx->vsmall_n0[0] = t.vsmall_fp64;
  ctx->vsmall_n0[1] = t.vsmall_fp32;
  if (t.cheb_degree != ctx->cheb.degree) {
    ctx->cfg.cheb_degree = t.cheb_degree;
    ctx->cheb = cheb_coeffs(t.cheb_degree, kChebHi / kChebRatio, kChebHi);
  }
  ctx->cfg.max_batch = t.max_batch;
  ctx->use_graphs = t.graph_batch > 0;
  ctx->graph_batch = std::max(1, t.graph_batch);
  ctx->fuse = t.fuse;
  ctx->field_kernel = t.field;
  ctx->n_lanes = t.lanes;
  // captured graphs bake in kernel choices: drop them
  drop_work(ctx);
}

template int vcycle<float>(mlmc_ctx*, std::vector<Level<float>>&, int, int, const float*, float*, float*, float*,
                           const int*, float**, SolveState*, uint32_t*, bool, const RUpdate<float>*);
template int vcycle<double>(mlmc_ctx*, std::vector<Level<double>>&, int, int, const double*, double*, double*,
                            double*, const int*, double**, SolveState*, uint32_t*, bool, const RUpdate<double>*);
template int precondition<float>(mlmc_ctx*, std::vector<Level<float>>&, int, const float*, float**, SolveState&,
                                 uint32_t*, bool, const RUpdate<float>*);
template int precondition<double>(mlmc_ctx*, std::vector<Level<double>>&, int, const double*, double**, SolveState&,
                                  uint32_t*, bool, const RUpdate<double>*);
template bool rupd_fusable<float>(const mlmc_ctx*, const std::vector<Level<float>>&, int);
template bool rupd_fusable<double>(const mlmc_ctx*, const std::vector<Level<double>>&, int);
template bool zero_step_fusable<float>(const mlmc_ctx*, const std::vector<Level<float>>&, int);
template bool zero_step_fusable<double>(const mlmc_ctx*, const std::vector<Level<double>>&, int);
template int pcg_iteration<float>(mlmc_ctx*, std::vector<Level<float>>&, int, SolveState&, float*, float*, float*,
                                  float*, double, int, bool);
template int pcg_iteration<double>(mlmc_ctx*, std::vector<Level<double>>&, int, SolveState&, double*, double*,
                                   double*, double*, double, int, bool);
template int pcg<float>(mlmc_ctx*, std::vector<Level<float>>&, int, SolveState&, float*, float*, float*, float*,
                        double, int, int*, hipGraphExec_t*, float*, bool, bool, float*);
template int pcg<double>(mlmc_ctx*, std::vector<Level<double>>&, int, SolveState&, double*, double*, double*,
                         double*, double, int, int*, hipGraphExec_t*, double*, bool, bool, double*);
template bool dir_fusable<float>(const mlmc_ctx*, const std::vector<Level<float>>&, int);
template bool dir_fusable<double>(const mlmc_ctx*, const std::vector<Level<double>>&, int);
template int pcg_dir_begin<float>(mlmc_ctx*, std::vector<Level<float>>&, int, SolveState&, const float*, const int*,
                                  bool);
template int pcg_dir_begin<double>(mlmc_ctx*, std::vector<Level<double>>&, int, SolveState&, const double*,
                                   const int*, bool);
template int pcg_iteration_dir<float>(mlmc_ctx*, std::vector<Level<float>>&, int, SolveState&, float*, float*, float*,
                                      float*, float*, double, int, bool, bool, float*);
template int pcg_iteration_dir<double>(mlmc_ctx*, std::vector<Level<double>>&, int, SolveState&, double*, double*,
                                       double*, double*, double*, double, int, bool, bool, double*);

}  // namespace eng
}  // namespace mlmc
