// C-ABI of the MLMC finite-element library (declared in include/mlmc.h):
// argument checking and the public entry points over the engine.
#include "engine.hpp"

static std::string g_create_error;

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
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->st);
    delete ctx;
    return MLMC_E_NOMEM;
  }
  Carver cv;
  cv.base = (char*)cfg->arena;
  cv.cap = cfg->arena_bytes;
  cv.dry = false;
  ctx->d_sqrtlam = cv.take<double>(cfg->n_modes);
  ctx->d_triples = cv.take<int>(3 * (size_t)cfg->n_modes);
  ctx->d_xperm = cv.take<int>((size_t)cfg->n_modes);
  ctx->d_xoff = cv.take<int>((size_t)ctx->K1 + 1);
  ctx->prof_counts = cv.take<int>(mlmc_ctx::kProfCap);
  ctx->d_stats = cv.take<DevStats>((size_t)cfg->levels);
  std::vector<double> sq(cfg->n_modes);
  for (int m = 0; m < cfg->n_modes; ++m) sq[m] = std::sqrt(ctx->modes.lambda[m]);
  hipError_t e = hipMemcpyAsync(ctx->d_sqrtlam, sq.data(), sq.size() * sizeof(double), hipMemcpyHostToDevice, ctx->st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ctx->d_triples, ctx->modes.triples.data(), ctx->modes.triples.size() * sizeof(int),
                       hipMemcpyHostToDevice, ctx->st);
  // the modes grouped by their x-factor, for the separable evaluation
  std::vector<int> xperm(cfg->n_modes), xoff(ctx->K1 + 1, 0);
  for (int m = 0; m < cfg->n_modes; ++m) xoff[ctx->modes.triples[3 * m] + 1] += 1;
  for (int a = 0; a < ctx->K1; ++a) xoff[a + 1] += xoff[a];
  {
    std::vector<int> fill(xoff.begin(), xoff.end() - 1);
    for (int m = 0; m < cfg->n_modes; ++m) xperm[fill[ctx->modes.triples[3 * m]]++] = m;
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(ctx->d_xperm, xperm.data(), xperm.size() * sizeof(int), hipMemcpyHostToDevice, ctx->st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ctx->d_xoff, xoff.data(), xoff.size() * sizeof(int), hipMemcpyHostToDevice, ctx->st);
  std::vector<std::vector<double>> tabs;
  for (int l = 0; l < cfg->levels && e == hipSuccess; ++l) {
    const int n = cfg->n0 << l;
    tabs.push_back(kl_centroid_table(ctx->modes, n));
    double* d = cv.take<double>((size_t)n * ctx->K1);
    ctx->d_tab[n] = d;
    e = hipMemcpyAsync(d, tabs.back().data(), tabs.back().size() * sizeof(double), hipMemcpyHostToDevice, ctx->st);
  }
  if (e == hipSuccess) e = hipMemsetAsync(ctx->d_stats, 0, (size_t)cfg->levels * sizeof(DevStats), ctx->st);
  if (e == hipSuccess) e = noalloc_scratch_init(&ctx->device, &ctx->scratch);
  if (e == hipSuccess) e = hipHostMalloc((void**)&ctx->h_nactive, sizeof(int), hipHostMallocDefault);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->st);
  if (e != hipSuccess) {
    g_create_error = std::string("HIP error during create: ") + hipGetErrorString(e);
    if (ctx->h_nactive) (void)hipHostFree(ctx->h_nactive);
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->st);
    delete ctx;
    return MLMC_E_DEVICE;
  }
  ctx->persistent_top = cv.top;
  *out = ctx;
  return MLMC_OK;
}

void mlmc_destroy(mlmc_ctx* ctx) {
  if (!ctx) return;
  mlmc_serve_stop(ctx);
  // teardown: errors have nowhere to go
  (void)hipStreamSynchronize(ctx->st);
  for (auto& r : ctx->prof) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto e : ctx->event_pool) (void)hipEventDestroy(e);
  drop_work(ctx);
  for (auto& ln : ctx->lanes)
    if (ln->sub) {
      (void)hipStreamSynchronize(ln->sub->st);
      (void)hipHostFree(ln->sub->h_nactive);
      (void)hipStreamDestroy(ln->sub->st);
    }
  ctx->lanes.clear();
  if (ctx->h_nactive) (void)hipHostFree(ctx->h_nactive);
  if (ctx->own_stream) (void)hipStreamDestroy(ctx->st);
  delete ctx;
}

size_t mlmc_workspace_bytes(const mlmc_config* cfg, int32_t level, int32_t batch) {
  std::string why;
  if (validate(cfg, why) || level < 0 || level >= cfg->levels || batch < 1) return 0;
  const KLModes md = kl_select(cfg->corr_len, cfg->sigma2, cfg->n_modes);
  mlmc_config c = *cfg;
  if (c.cheb_degree == 0) c.cheb_degree = 2;
  // one lane: the larger of the pair's two solves, and the round's QoI buffers
  const int nf = c.n0 << level;
  size_t w = mesh_work_bytes(c, level, nf, batch);
  if (level > 0) w = std::max(w, mesh_work_bytes(c, level, nf / 2, batch));
  return persistent_bytes(&c, (int)md.omega.size()) + w + 2 * align256((size_t)batch * sizeof(double)) + 256;
}

int mlmc_node_map(mlmc_ctx* ctx, int32_t n, int32_t* out) {
  if (!ctx) return MLMC_E_INVALID;
  if (ctx->server) FAIL(MLMC_E_INVALID, "the context is serving");
  if (n < 2 || n > 1024 || !is_pow2(n) || !out) FAIL(MLMC_E_INVALID, "bad node map arguments");
  const size_t S = grid_stride(n);
  if (ctx->persistent_top + align256(S * sizeof(int32_t)) > ctx->cfg.arena_bytes)
    FAIL(MLMC_E_NOMEM, "arena too small for the node map");
  // scratch right after the persistent tables: the cached work space there is
  // dropped and carved (and cleared) again when next needed
  drop_work(ctx);
  int32_t* d = reinterpret_cast<int32_t*>((char*)ctx->cfg.arena + ctx->persistent_top);
  LAUNCH(MLMC_K_MISC, 0, launch_node_map(n, d, ctx->st));
  HIPCHK(hipMemcpyAsync(out, d, S * sizeof(int32_t), hipMemcpyDeviceToHost, ctx->st));
  HIPCHK(hipStreamSynchronize(ctx->st));
  return MLMC_OK;
}

int mlmc_forcing(mlmc_ctx* ctx, int32_t n, int32_t level, uint64_t first, int64_t count, double* f, double* b) {
  if (!ctx) return MLMC_E_INVALID;
  if (ctx->server) FAIL(MLMC_E_INVALID, "the context is serving");
  if (n < 2 || !is_pow2(n) || !mesh_of_config(ctx, n) || level < 0 || count < 0 || count > (1 << 30) ||
      (count > 0 && (!f || !b)))
    FAIL(MLMC_E_INVALID, "bad forcing arguments");
  if (count == 0) return MLMC_OK;
  const size_t xb = align256((size_t)count * ctx->cfg.n_modes * sizeof(double));
  if (ctx->persistent_top + xb > ctx->cfg.arena_bytes) FAIL(MLMC_E_NOMEM, "arena too small for the forcing draw");
  // scratch right after the persistent tables (the cached work space there is
  // dropped and carved again when next needed)
  drop_work(ctx);
  double* xif = reinterpret_cast<double*>((char*)ctx->cfg.arena + ctx->persistent_top);
  if (int rc = forcing_impl(ctx, n, level, first, (int)count, xif, f, b)) return rc;
  HIPCHK(hipStreamSynchronize(ctx->st));
  return MLMC_OK;
}

int mlmc_modes(const mlmc_ctx* ctx, int32_t* triples, double* lambda) {
  if (!ctx) return MLMC_E_INVALID;
  const int M = ctx->cfg.n_modes;
  if (triples) std::memcpy(triples, ctx->modes.triples.data(), 3 * (size_t)M * sizeof(int32_t));
  if (lambda) std::memcpy(lambda, ctx->modes.lambda.data(), (size_t)M * sizeof(double));
  return MLMC_OK;
}

int mlmc_kl_modes(double corr_len, double sigma2, int32_t n_modes, int32_t* triples, double* lambda, double* omega,
                  int32_t max_omega, int32_t* n_omega) {
  if (!(corr_len > 0.0) || !std::isfinite(corr_len) || !(sigma2 >= 0.0) || !std::isfinite(sigma2) || n_modes < 1 ||
      n_modes > 4096 || max_omega < 0 || (max_omega > 0 && !omega))
    return MLMC_E_INVALID;
  const KLModes md = kl_select(corr_len, sigma2, n_modes);
  if (triples) std::memcpy(triples, md.triples.data(), 3 * (size_t)n_modes * sizeof(int32_t));
  if (lambda) std::memcpy(lambda, md.lambda.data(), (size_t)n_modes * sizeof(double));
  const int k1 = (int)md.omega.size();
  if (omega) std::memcpy(omega, md.omega.data(), (size_t)std::min(k1, (int)max_omega) * sizeof(double));
  if (n_omega) *n_omega = k1;
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
         launch_apply<double>(n, (int)count, kappa, u, y, nullptr, ctx->st, zv<double>(ctx)));
  return MLMC_OK;
}

int mlmc_apply_f32(mlmc_ctx* ctx, int32_t n, int64_t count, const float* kappa, const float* u, float* y) {
  if (!ctx) return MLMC_E_INVALID;
  if (n < 2 || !is_pow2(n) || n > 1024 || count < 0 || count > (1 << 30) || (count > 0 && (!kappa || !u || !y)) ||
      (count > 0 && u == y))
    FAIL(MLMC_E_INVALID, "bad apply arguments");
  if (count == 0) return MLMC_OK;
  LAUNCH(kid<float>(MLMC_K_APPLY), (2 * dofs(n) + elems(n)) * count * 4,
         launch_apply<float>(n, (int)count, kappa, u, y, nullptr, ctx->st, zv<float>(ctx)));
  return MLMC_OK;
}

int mlmc_jacobi(mlmc_ctx* ctx, int32_t n, int64_t count, const double* kappa, const double* b, double c,
                double* z) {
  if (!ctx) return MLMC_E_INVALID;
  if (n < 2 || !is_pow2(n) || n > 1024 || count < 0 || count > (1 << 30) || (count > 0 && (!kappa || !b || !z)) ||
      (count > 0 && b == z) || !std::isfinite(c))
    FAIL(MLMC_E_INVALID, "bad jacobi arguments");
  if (count == 0) return MLMC_OK;
  LAUNCH(MLMC_K_CHEB_ZERO, (2 * dofs(n) + elems(n)) * count * 8,
         launch_cheb<double>(n, (int)count, kappa, b, nullptr, nullptr, z, 0.0, c, true, false, nullptr, ctx->st,
                             nullptr, nullptr, zv<double>(ctx)));
  return MLMC_OK;
}

int mlmc_vcycle(mlmc_ctx* ctx, int32_t n, int64_t count, const double* kappa, const double* r, double* z) {
  if (!ctx) return MLMC_E_INVALID;
  if (ctx->server) FAIL(MLMC_E_INVALID, "the context is serving");
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

int mlmc_vcycle_f32(mlmc_ctx* ctx, int32_t n, int64_t count, const float* kappa, const float* r, float* z) {
  if (!ctx) return MLMC_E_INVALID;
  if (ctx->server) FAIL(MLMC_E_INVALID, "the context is serving");
  if (n < 2 || !is_pow2(n) || n > 1024 || count < 1 || count > (1 << 30) || !kappa || !r || !z)
    FAIL(MLMC_E_INVALID, "bad vcycle arguments");
  const int B = (int)count;
  mlmc_config saved = ctx->cfg;
  ctx->cfg.precision = MLMC_PREC_MIXED;
  ctx->cfg.solver = MLMC_SOLVER_GMG_PCG;
  int rc = ensure_solve_work(ctx, n, B);
  ctx->cfg = saved;
  if (rc) return rc;
  auto& L = ctx->sw.L32;
  float* own0 = L[0].kap;
  L[0].kap = const_cast<float*>(kappa);
  hipStream_t st = ctx->st;
  for (size_t l = 1; l < L.size(); ++l)
    LAUNCH(kid<float>(MLMC_K_COARSEN), 0, launch_coarsen<float>(L[l - 1].n, B, L[l - 1].kap, L[l].kap, st));
  SolveState& S = ctx->sw.inner.s;
  LAUNCH(MLMC_K_MISC, 0, launch_set_active(B, S, 1, st));
  float* res = nullptr;
  rc = vcycle<float>(ctx, L, 0, B, r, L[0].x, L[0].xo, L[0].t, S.active, &res);
  L[0].kap = own0;
  if (rc) return rc;
  HIPCHK(hipMemcpyAsync(z, res, (size_t)B * grid_stride(n) * sizeof(float), hipMemcpyDeviceToDevice, st));
  return MLMC_OK;
}

int mlmc_solve(mlmc_ctx* ctx, int32_t n, int64_t count, const double* kappa, double* u, int32_t* iters) {
  if (!ctx) return MLMC_E_INVALID;
  if (ctx->server) FAIL(MLMC_E_INVALID, "the context is serving");
  if (n < 2 || !is_pow2(n) || count < 1 || count > (1 << 30) || !kappa || !u)
    FAIL(MLMC_E_INVALID, "bad solve arguments");
  if (int rc = ensure_solve_work(ctx, n, (int)count)) return rc;
  int status = MLMC_OK;
  if (int rc = solve_impl(ctx, ctx->sw, kappa, u, iters, &status)) return rc;
  if (status == MLMC_E_NONFINITE) FAIL(MLMC_E_NONFINITE, "a residual became NaN or Inf");
  if (status) FAIL(MLMC_E_NOCONV, "some samples did not reach rtol within max_iter");
  return MLMC_OK;
}

int mlmc_qoi(mlmc_ctx* ctx, int32_t n, int64_t count, const double* u, double* q) {
  if (!ctx) return MLMC_E_INVALID;
  if (ctx->server) FAIL(MLMC_E_INVALID, "the context is serving");
  if (n < 2 || !is_pow2(n) || count < 1 || count > (1 << 30) || !u || !q) FAIL(MLMC_E_INVALID, "bad qoi arguments");
  if (ctx->cfg.qoi == 1 && n % 4) FAIL(MLMC_E_INVALID, "subcube QoI needs 4 | n");
  if (int rc = ensure_solve_work(ctx, n, (int)count)) return rc;
  return qoi_impl(ctx, ctx->sw.outer.s, n, (int)count, u, q);
}

}  // extern "C"

extern "C" {

int mlmc_qoi_noalloc(mlmc_ctx* ctx, int32_t n, int64_t count, const double* u, double* q) {
  if (!ctx) return MLMC_E_INVALID;
  if (n < 2 || !is_pow2(n) || n > 1024 || count < 1 || count > (1 << 30) || !u || !q)
    FAIL(MLMC_E_INVALID, "bad qoi arguments");
  if (ctx->cfg.qoi == 1 && n % 4) FAIL(MLMC_E_INVALID, "subcube QoI needs 4 | n");
  if (qoi_scratch_bytes(n, (int)count) > noalloc_scratch_bytes())
    FAIL(MLMC_E_INVALID, "count above the static scratch: at most " +
                             std::to_string(noalloc_scratch_bytes() / qoi_scratch_bytes(n, 1)) + " samples on " +
                             std::to_string(n) + "^3");
  if (!ctx->scratch) FAIL(MLMC_E_DEVICE, "no static scratch on this device");
  const hipError_t e = launch_qoi_scratch(n, (int)count, ctx->cfg.qoi, u, q, ctx->scratch, ctx->st);
  if (e != hipSuccess) FAIL(MLMC_E_DEVICE, std::string("kernel launch failed: ") + hipGetErrorString(e));
  return MLMC_OK;
}

int mlmc_sample_level(mlmc_ctx* ctx, int32_t level, uint64_t first, uint64_t count, double* y, double* q_fine,
                      double* q_coarse, int32_t* iters) {
  if (!ctx) return MLMC_E_INVALID;
  if (ctx->server) FAIL(MLMC_E_INVALID, "the context is serving");
  if (level < 0 || level >= ctx->cfg.levels) FAIL(MLMC_E_INVALID, "level out of range");
  if (count > 0 && (!y || !q_fine || !q_coarse)) FAIL(MLMC_E_INVALID, "NULL output array");
  const int nf = ctx->cfg.n0 << level;
  if (ctx->cfg.qoi == 1 && ((nf % 4) || (level > 0 && (nf / 2) % 4)))
    FAIL(MLMC_E_INVALID, "subcube QoI needs 4 | n on both meshes");
  if (count == 0) return MLMC_OK;
  ctx->last_busy = ctx->last_wall = 0.0;
  std::vector<LevelReq> reqs(1);
  reqs[0].level = level;
  reqs[0].first = first;
  reqs[0].count = count;
  reqs[0].y = y;
  reqs[0].qf = q_fine;
  reqs[0].qc = q_coarse;
  reqs[0].iters = iters;
  return run_round(ctx, reqs, true);
}

int mlmc_get_tuning(const mlmc_ctx* ctx, mlmc_tuning* out) {
  if (!ctx || !out) return MLMC_E_INVALID;
  *out = current_tuning(ctx);
  return MLMC_OK;
}

int mlmc_set_tuning(mlmc_ctx* ctx, const mlmc_tuning* t) {
  if (!ctx) return MLMC_E_INVALID;
  std::string why;
  if (int rc = check_tuning(t, why)) FAIL(rc, why);
  apply_tuning(ctx, *t);
  return MLMC_OK;
}

int mlmc_autotune(mlmc_ctx* ctx, int32_t level, int32_t batch, mlmc_tuning* best_out) {
  if (!ctx) return MLMC_E_INVALID;
  if (ctx->server) FAIL(MLMC_E_INVALID, "the context is serving");
  if (level < 0 || level >= ctx->cfg.levels || batch < 1) FAIL(MLMC_E_INVALID, "bad autotune arguments");
  const uint64_t first = 1ull << 40;   // sample indices far from any estimator run
  std::vector<double> y(batch), qf(batch), qc(batch);
  std::vector<LevelReq> reqs(1);
  reqs[0].level = level;
  reqs[0].first = first;
  reqs[0].count = (uint64_t)batch;
  reqs[0].y = y.data();
  reqs[0].qf = qf.data();
  reqs[0].qc = qc.data();
  auto timed = [&](const mlmc_tuning& t, double* sec) -> int {
    apply_tuning(ctx, t);
    // one untimed run carves work spaces and captures graphs
    int rc = run_round(ctx, reqs, false);
    if (rc && rc != MLMC_E_NOCONV) return rc;
    const auto t0 = std::chrono::steady_clock::now();
    rc = run_round(ctx, reqs, false);
    if (rc && rc != MLMC_E_NOCONV) return rc;
    *sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count() / batch;
    return MLMC_OK;
  };
  mlmc_tuning best = current_tuning(ctx);
  best.max_batch = batch;
  double best_s = 0.0;
  if (int rc = timed(best, &best_s)) return rc;
  auto trial = [&](mlmc_tuning cand) -> int {
    std::string why;
    if (check_tuning(&cand, why)) return MLMC_OK;
    double s = 0.0;
    const int rc = timed(cand, &s);
    if (rc == MLMC_E_NOMEM) return MLMC_OK;   // skip settings the arena cannot hold
    if (rc) return rc;
    if (s < best_s) {
      best_s = s;
      best = cand;
    }
    return MLMC_OK;
  };
  const mlmc_tuning base = best;
  for (int deg : {1, 2, 3}) {
    if (deg == base.cheb_degree) continue;
    mlmc_tuning c = best; c.cheb_degree = deg;
    if (int rc = trial(c)) return rc;
  }
  for (int zv : {0, 1, 2, 6}) {
    if (zv == base.zvar_fp32) continue;
    mlmc_tuning c = best; c.zvar_fp32 = zv; c.zvar_fp64 = zv;
    if (int rc = trial(c)) return rc;
  }
  for (int v : {16, 8, 0}) {
    if (v == best.vsmall_fp32) continue;
    mlmc_tuning c = best; c.vsmall_fp32 = v; c.vsmall_fp64 = std::min(v, 8);
    if (int rc = trial(c)) return rc;
  }
  const int nf = ctx->cfg.n0 << level, nc = level > 0 ? nf / 2 : 0;
  for (int f : {MLMC_FUSE_PROLONG, MLMC_FUSE_UPDATE, MLMC_FUSE_REFINE, MLMC_FUSE_RESTRICT, MLMC_FUSE_PRESMOOTH,
                MLMC_FUSE_DIRECTION, MLMC_FUSE_RUPDATE, MLMC_FUSE_SOLVE, MLMC_FUSE_PACK}) {
    if (f == MLMC_FUSE_SOLVE && nf > 8 && !(nc >= 4 && nc <= 8)) continue;   // no 4^3 or 8^3 solve here
    if (f == MLMC_FUSE_PACK) continue;   // a single level has nothing to pack
    mlmc_tuning c = best; c.fuse ^= f;
    if (int rc = trial(c)) return rc;
  }
  for (int g : {0, 1, 2, 4}) {
    if (g == best.graph_batch) continue;
    mlmc_tuning c = best; c.graph_batch = g;
    if (int rc = trial(c)) return rc;
  }
  for (int div : {2, 4}) {
    if (batch / div < 1) continue;
    mlmc_tuning c = best; c.max_batch = batch / div;
    if (int rc = trial(c)) return rc;
  }
  for (int k : {1, 2, 4}) {
    if (k == best.lanes) continue;
    mlmc_tuning c = best; c.lanes = k;
    if (int rc = trial(c)) return rc;
  }
  best.seconds = best_s;
  apply_tuning(ctx, best);
  if (best_out) *best_out = best;
  return MLMC_OK;
}

namespace {

// (c, r) of vals_l ~ c s^(-r l) over l = 1..lmax (Sec. 2.3: c and alpha
// estimated from the level means, the variance decay likewise): the
// least-squares line through (l, log_s vals_l) from its normal equations,
// whose level sums are exact integers; r is clamped to [lo, hi] and c then
// refitted for the clamped slope.  One level gives no slope: r = dflt
// through that point.
void decay_rate(const std::vector<double>& vals, int lmax, double dflt, double lo, double hi, double s, double* c,
                double* r) {
  const double ls = std::log(s);
  const double n = (double)lmax;
  const double sx = 0.5 * n * (n + 1.0), sxx = n * (n + 1.0) * (2.0 * n + 1.0) / 6.0;
  double sy = 0.0, sxy = 0.0;
  for (int l = 1; l <= lmax; ++l) {
    const double y = std::log(std::max(std::fabs(vals[l]), 1e-300)) / ls;
    sy += y;
    sxy += (double)l * y;
  }
  double rr = dflt;
  if (lmax >= 2) rr = std::min(std::max(-(n * sxy - sx * sy) / (n * sxx - sx * sx), lo), hi);
  *r = rr;
  *c = std::pow(s, (sy + rr * sx) / n);
}

// One sampling round that brings every level 0..L up to target[l] samples
// (continuing each level's sample indices); NOCONV / NONFINITE are merged into
// *status (NONFINITE first) and do not stop the caller's loop.
int sample_to(mlmc_ctx* ctx, const std::vector<uint64_t>& target, int L, int* status) {
  std::vector<LevelReq> reqs;
  for (int l = 0; l <= L; ++l) {
    const uint64_t have = ctx->stats[l].n;
    if (target[l] > have) {
      LevelReq q;
      q.level = l;
      q.first = ctx->stats[l].next;
      q.count = target[l] - have;
      reqs.push_back(q);
    }
  }
  const int rc = run_round(ctx, reqs, true);
  if (rc == MLMC_E_NONFINITE || rc == MLMC_E_NOCONV) {
    if (*status != MLMC_E_NONFINITE) *status = rc;
    return MLMC_OK;
  }
  return rc;
}

}  // namespace

int mlmc_estimate_adaptive(mlmc_ctx* ctx, const mlmc_adaptive_opts* o, uint64_t* n_per_level,
                           mlmc_adaptive_info* info, mlmc_estimate_out* out) {
  if (!ctx) return MLMC_E_INVALID;
  if (ctx->server) FAIL(MLMC_E_INVALID, "the context is serving");
  const int M = ctx->cfg.levels;
  if (!o || !(o->eps > 0.0) || o->l0 < 1 || o->l0 >= M || o->n_pilot < 2 || o->cost_model < 0 ||
      o->cost_model > 1 || o->max_rounds < 0 || !(o->extra_fraction >= 0.0) || o->alpha0 < 0.0 || o->beta0 < 0.0)
    FAIL(MLMC_E_INVALID, "bad adaptive estimate options");
  const double s = 2.0, ls = std::log(s);
  const double alpha0 = o->alpha0 > 0.0 ? o->alpha0 : 2.0, beta0 = o->beta0 > 0.0 ? o->beta0 : 4.0;
  auto dof_cost = [&](int l) {
    const int nf = ctx->cfg.n0 << l;
    return dofs(nf) + (l > 0 ? dofs(nf / 2) : 0.0);
  };
  // measured: seconds per sample; a level not timed yet scales the finest
  // timed level by the DOF ratio
  auto cost_of = [&](int l) {
    if (o->cost_model == 1) return dof_cost(l);
    const Running& r = ctx->stats[l];
    if (r.timed) return r.seconds / (double)r.timed;
    for (int k = M - 1; k >= 0; --k)
      if (ctx->stats[k].timed) return ctx->stats[k].seconds / (double)ctx->stats[k].timed * dof_cost(l) / dof_cost(k);
    return dof_cost(l);
  };
  int L = o->l0;
  int status = MLMC_OK;
  ctx->last_busy = ctx->last_wall = 0.0;
  std::vector<uint64_t> target(M, 0);
  for (int l = 0; l <= L; ++l) target[l] = std::max<uint64_t>(ctx->stats[l].n, (uint64_t)o->n_pilot);
  double alpha = 0.0, beta = 0.0, bias = 0.0, err = 0.0;
  int rounds = 0;
  for (int rnd = 0; rnd <= o->max_rounds; ++rnd) {
    rounds = rnd + 1;
    if (int rc = sample_to(ctx, target, L, &status)) return rc;
    std::vector<double> mean(M), var(M);
    for (int l = 0; l < M; ++l) {
      const Running& r = ctx->stats[l];
      mean[l] = r.mean;
      var[l] = r.n ? r.m2 / (double)r.n : 0.0;
    }
    double cY = 0.0, cV = 0.0;
    decay_rate(mean, L, alpha0, 0.5, 4.0, s, &cY, &alpha);
    decay_rate(var, L, beta0, 0.5, 8.0, s, &cV, &beta);
    const double tail = std::pow(s, alpha) - 1.0;
    bias = cY * std::pow(s, -alpha * L) / tail;
    double vq = 0.0;
    for (int l = 0; l <= L; ++l) vq += var[l] / (double)ctx->stats[l].n;
    err = std::sqrt(bias * bias + vq);
    if (err <= o->eps || rnd == o->max_rounds) break;
    // eq. mlmc_num_levels with c / (s^alpha - 1), L only grows
    const int want_L = (int)std::ceil(std::log(std::sqrt(2.0) * (cY / tail) / o->eps) / ls / alpha);
    const int L_new = std::min(M - 1, std::max(L, want_L));
    std::vector<double> V(L_new + 1), C(L_new + 1);
    for (int l = 0; l <= L_new; ++l) {
      V[l] = l <= L ? var[l] : cV * std::pow(s, -beta * l);
      C[l] = cost_of(l);
    }
    double tot = 0.0;
    for (int l = 0; l <= L_new; ++l) tot += std::sqrt(V[l] * C[l]);
    bool grow = L_new > L;
    for (int l = 0; l <= L_new; ++l) {
      const double nl = 2.0 / (o->eps * o->eps) * std::sqrt(V[l] / C[l]) * tot * (1.0 + o->extra_fraction);
      const uint64_t want = std::max<uint64_t>((uint64_t)std::ceil(nl), (uint64_t)o->n_pilot);
      if (want > target[l]) {
        target[l] = want;
        grow = true;
      }
    }
    L = L_new;
    if (!grow) break;
  }
  for (int l = 0; l < M; ++l) {
    if (l <= L) ctx->stats[l].cost = cost_of(l);
    if (n_per_level) n_per_level[l] = l <= L ? ctx->stats[l].n : 0;
  }
  if (info) {
    info->L = L;
    info->rounds = rounds;
    info->alpha = alpha;
    info->beta = beta;
    info->bias = bias;
    info->err = err;
  }
  if (out) mlmc_get_estimate(ctx, out);
  if (status == MLMC_E_NONFINITE) FAIL(status, "some samples were NaN or Inf (kept out of the statistics)");
  if (status == MLMC_E_NOCONV) FAIL(status, "some samples did not reach rtol within max_iter");
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
    o.nonfinite = r.nonfinite;
    out->qtilde += r.mean;
    if (r.n) out->var_qtilde += o.var / (double)r.n;
  }
  out->lanes = ctx->last_lanes;
  out->active_ratio = ctx->last_wall > 0.0 ? ctx->last_busy / ctx->last_wall : 0.0;
  return MLMC_OK;
}

int mlmc_estimate(mlmc_ctx* ctx, const mlmc_estimate_opts* o, uint64_t* n_per_level, mlmc_estimate_out* out) {
  if (!ctx) return MLMC_E_INVALID;
  if (ctx->server) FAIL(MLMC_E_INVALID, "the context is serving");
  if (!o || (!o->n_fixed && !(o->eps > 0.0)) || o->n_pilot < 2 || o->cost_model < 0 || o->cost_model > 1 ||
      !(o->extra_fraction >= 0.0) || o->max_rounds < 1)
    FAIL(MLMC_E_INVALID, "bad estimate options");
  const int L = ctx->cfg.levels;
  int status = MLMC_OK;
  ctx->last_busy = ctx->last_wall = 0.0;
  auto cost_of = [&](int l) {
    const Running& r = ctx->stats[l];
    if (o->cost_model == 1 || r.timed == 0) {
      const int nf = ctx->cfg.n0 << l;
      return dofs(nf) + (l > 0 ? dofs(nf / 2) : 0.0);
    }
    return r.seconds / (double)r.timed;
  };
  std::vector<uint64_t> target(L, 0);
  // pilot (or the caller's fixed N_l)
  for (int l = 0; l < L; ++l) {
    const uint64_t have = ctx->stats[l].n;
    target[l] = std::max<uint64_t>(have, o->n_fixed ? o->n_fixed[l] : (uint64_t)o->n_pilot);
  }
  for (int round = 0; round <= o->max_rounds; ++round) {
    bool more = false;
    for (int l = 0; l < L; ++l) more = more || target[l] > ctx->stats[l].n;
    if (int rc = sample_to(ctx, target, L - 1, &status)) return rc;
    if ((!more && round > 0) || round == o->max_rounds || o->n_fixed) break;
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
  if (out) mlmc_get_estimate(ctx, out);
  if (status == MLMC_E_NONFINITE) FAIL(status, "some samples were NaN or Inf (kept out of the statistics)");
  if (status == MLMC_E_NOCONV) FAIL(status, "some samples did not reach rtol within max_iter");
  return MLMC_OK;
}

int mlmc_reset_stats(mlmc_ctx* ctx) {
  if (!ctx) return MLMC_E_INVALID;
  if (ctx->server) FAIL(MLMC_E_INVALID, "the context is serving");
  ctx->stats.assign(ctx->cfg.levels, Running{});
  HIPCHK(hipMemsetAsync(ctx->d_stats, 0, (size_t)ctx->cfg.levels * sizeof(DevStats), ctx->st));
  HIPCHK(hipStreamSynchronize(ctx->st));
  return MLMC_OK;
}

int mlmc_fold_stats(mlmc_ctx* ctx, int32_t level, const double* y, uint64_t count) {
  if (!ctx) return MLMC_E_INVALID;
  if (ctx->server) FAIL(MLMC_E_INVALID, "the context is serving");
  if (level < 0 || level >= ctx->cfg.levels || (count > 0 && !y)) FAIL(MLMC_E_INVALID, "bad fold arguments");
  if (count == 0) return MLMC_OK;
  const uint64_t nf0 = ctx->stats[level].nonfinite;
  StatsJobs jobs{};
  jobs.j[0] = StatsJob{y, nullptr, count, reinterpret_cast<double*>(ctx->d_stats + level)};
  LAUNCH(MLMC_K_MISC, 0, launch_level_stats(1, jobs, ctx->st));
  if (int rc = read_stats(ctx)) return rc;
  if (ctx->stats[level].nonfinite != nf0) FAIL(MLMC_E_NONFINITE, "some values were NaN or Inf");
  return MLMC_OK;
}

int mlmc_last_plan(const mlmc_ctx* ctx, mlmc_plan_task* out, int32_t max, int32_t* n) {
  if (!ctx || !n || max < 0 || (max > 0 && !out)) return MLMC_E_INVALID;
  int32_t k = 0;
  for (size_t i = 0; i < ctx->last_plan.size(); ++i) {
    const Task& t = ctx->last_plan[i];
    for (const Part& p : t.parts) {
      if (k < max) out[k] = mlmc_plan_task{p.level, t.n, p.first, p.count, t.lane, (int32_t)i};
      ++k;
    }
  }
  *n = k;
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
  ctx->prof_used = 0;
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
  std::vector<int> cnt(ctx->prof_used);
  if (ctx->prof_used)
    HIPCHK(hipMemcpy(cnt.data(), ctx->prof_counts, cnt.size() * sizeof(int), hipMemcpyDeviceToHost));
  ctx->prof_used = 0;
  for (auto& r : ctx->prof) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, r.a, r.b));
    ctx->k_launch[r.id] += 1;
    ctx->k_ms[r.id] += ms;
    // masked launches: only the active samples' bytes move
    ctx->k_bytes[r.id] += r.cnt >= 0 && r.B > 0 ? r.bytes * cnt[r.cnt] / r.B : r.bytes;
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

