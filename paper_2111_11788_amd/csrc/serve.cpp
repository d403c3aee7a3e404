// Serving: a persistent request loop with step-level continuous batching.
//
// A request is one MLMC sample (level l, sample index i); it needs the FE
// solve of the n_l mesh and, for l > 0, of the n_{l-1} mesh on the same draw
// (Sec. 2.2).  Each mesh has a resident pool of S slots carved from the
// context's arena (the HBM budget): every slot keeps its kappa, its whole
// fp32 multigrid hierarchy and its solver vectors on the device until the
// solve finishes.  A host thread and a stream per pool run steps; each step
//   admits queued jobs into free slots (draw xi, KLE field, coarse kappa,
//   x = 0, r = b), restarts the fp32 inner PCG of slots that need it, runs one
//   inner PCG iteration for every slot in its inner phase, applies the fp64
//   refinement (x += d, r = b - A x) for slots whose inner solve converged,
//   and computes the QoI of slots whose true residual reached rtol.
// So requests join a batch that is already iterating as soon as a slot is
// free (continuous batching), pools of different meshes run concurrently, and
// each slot's arithmetic is exactly that of a slot solved alone: every
// reduction is per slot with a geometry fixed by the pool size.
#include "engine.hpp"

#include <atomic>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>

namespace {

using Clock = std::chrono::steady_clock;
constexpr double kInnerTol = 1e-4;   // relative tolerance of each fp32 inner solve

struct Job {
  uint64_t ticket;
  int level;
  uint64_t sample;
  bool fine;
};

struct Request {
  int level = 0;
  uint64_t sample = 0;
  double t_submit = 0, t_admit = -1, t_done = 0;
  int pending = 0;
  double qf = 0, qc = 0;
  int iters = 0;
  int status = MLMC_OK;
  bool done = false;
};

struct Pool {
  int m = 0, n = 0, S = 0;
  double busy_slot_s = 0.0;     // sum over steps of occupied slots x step seconds (server mutex)
  size_t slot_bytes = 0;        // arena bytes of one slot
  mlmc_ctx sub;                 // engine view: shared tables, own stream and pinned counter
  SolveWork w;
  double *kap64 = nullptr, *u = nullptr, *xi = nullptr, *q = nullptr;
  uint64_t* d_ids = nullptr;
  int *d_lv = nullptr, *d_slots = nullptr;
  int *phase = nullptr, *m_trans = nullptr, *m_restart = nullptr, *m_done = nullptr, *m_new = nullptr;
  uint64_t* h_ids = nullptr;
  int *h_lv = nullptr, *h_slots = nullptr, *h_phase = nullptr, *h_iters = nullptr;
  double* h_q = nullptr;
  std::vector<int> busy;
  std::vector<Job> job;
  std::deque<Job> queue;        // guarded by the server mutex
  int occupied = 0;
  std::thread th;
  // Lending (all guarded by the server mutex).  A main pool owns an arena
  // region; while it is idle its region may hold a guest pool of another
  // mesh with the same slot count as that mesh's own pool, which serves that
  // pool's queue.
  size_t region_off = 0, region_bytes = 0;   // a main pool's region
  Pool* owner = nullptr;        // a guest: the main pool whose queue it serves
  Pool* helper = nullptr;       // a main pool: its guest running in another region
  std::unique_ptr<Pool> guest;  // a main pool: the guest in its region (it is lent)
  bool closing = false;         // a guest: admit nothing more, end when its slots are empty
  bool exited = false;          // a guest: its thread has ended

  void carve(Carver& cv, const mlmc_config& c, int m_, int S_) {
    m = m_;
    n = c.n0 << m_;
    S = S_;
    w.carve(cv, n, S, MLMC_PREC_MIXED, MLMC_SOLVER_GMG_PCG);
    kap64 = cv.take<double>((size_t)S * elem_count(n));
    u = cv.take<double>((size_t)S * grid_stride(n));
    xi = cv.take<double>((size_t)S * c.n_modes);
    q = cv.take<double>(S);
    d_ids = cv.take<uint64_t>(S);
    d_lv = cv.take<int>(S);
    d_slots = cv.take<int>(S);
    phase = cv.take<int>(S);
    m_trans = cv.take<int>(S);
    m_restart = cv.take<int>(S);
    m_done = cv.take<int>(S);
    m_new = cv.take<int>(S);
  }
};

size_t pool_bytes(const mlmc_config& c, int m, int S) {
  Carver dry;
  Pool p;
  p.carve(dry, c, m, S);
  return dry.top;
}

}  // namespace

struct mlmc_server {
  mlmc_ctx* ctx = nullptr;
  std::vector<std::unique_ptr<Pool>> pools;   // by mesh level
  std::mutex mu;
  std::condition_variable cv;
  std::unordered_map<uint64_t, Request> reqs;
  std::deque<uint64_t> finished;               // completion order, not yet drained
  std::condition_variable done_cv;
  uint64_t next_ticket = 1;
  bool stopping = false;
  int error = MLMC_OK;
  std::string error_msg;
  Clock::time_point t0 = Clock::now();
  uint64_t completed = 0;
  uint64_t lends = 0, reclaims = 0;
  double dofs_done = 0.0;
  double first_submit = -1.0, last_done = 0.0;

  double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
};

namespace {

#define SRV_LAUNCH(call)                                                   \
  do {                                                                     \
    const hipError_t e_ = (call);                                          \
    if (e_ != hipSuccess) {                                                \
      ctx->err = std::string("serving kernel failed: ") + hipGetErrorString(e_); \
      return MLMC_E_DEVICE;                                                \
    }                                                                      \
  } while (0)

SolveState view(SolveState s, int* active, int* phase) {
  s.active = active;
  s.phase = phase;
  return s;
}

// Admit `c` new jobs whose slots are in p.h_slots[0..c): draw, field, hierarchy, x = 0, r = b.
int setup_slots(Pool& p, int c) {
  mlmc_ctx* ctx = &p.sub;
  hipStream_t st = ctx->st;
  const int S = p.S, n = p.n;
  const double h = 1.0 / n;
  HIPCHK(hipMemcpyAsync(p.d_ids, p.h_ids, c * sizeof(uint64_t), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(p.d_lv, p.h_lv, c * sizeof(int), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(p.d_slots, p.h_slots, c * sizeof(int), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemsetAsync(p.m_new, 0, S * sizeof(int), st));
  SRV_LAUNCH(launch_set_phase_list(c, p.d_slots, p.m_new, 1, st));
  SRV_LAUNCH(launch_draw_xi_rows(ctx->cfg.seed, c, ctx->cfg.n_modes, p.d_ids, p.d_lv, p.d_slots, p.xi, st));
  double* tab = nullptr;
  if (int rc = ensure_tables(ctx, n, &tab)) return rc;
  auto& L = p.w.L32;
  SRV_LAUNCH(launch_field(n, ctx->cfg.n_modes, c, p.xi, ctx->d_sqrtlam, ctx->d_triples, tab, ctx->K1, p.kap64,
                          L[0].kap, st, p.d_slots, ctx->cfg.precision == MLMC_PREC_MIXED_BF16KLE,
                          field_separable(ctx, c) ? ctx->d_xperm : nullptr, ctx->d_xoff));
  for (size_t l = 1; l < L.size(); ++l)
    SRV_LAUNCH(launch_coarsen<float>(L[l - 1].n, S, L[l - 1].kap, L[l].kap, st, p.m_new));
  SRV_LAUNCH(launch_fill_interior<double>(n, S, p.u, 0.0, p.m_new, st));
  SRV_LAUNCH(launch_fill_interior<double>(n, S, p.w.r64, h * h * h, p.m_new, st));
  SolveState on = view(p.w.outer.s, p.m_new, p.phase);
  uint32_t np = 0;
  SRV_LAUNCH(launch_dot<double>(n, S, p.w.r64, p.w.r64, on, &np, st));
  SRV_LAUNCH(launch_reduce(S, RED_BB, 0.0, np, on, nullptr, st));
  SRV_LAUNCH(launch_set_phase_mask(S, p.m_new, p.phase, PHASE_RESTART, p.w.inner.s.iters, st));
  return MLMC_OK;
}

int masks(Pool& p) {
  mlmc_ctx* ctx = &p.sub;
  SRV_LAUNCH(launch_phase_masks(p.S, p.phase, p.w.inner.s.active, p.m_trans, p.m_restart, p.m_done, ctx->st));
  return MLMC_OK;
}

// One step of every occupied slot (see the file comment).
int step(Pool& p) {
  mlmc_ctx* ctx = &p.sub;
  hipStream_t st = ctx->st;
  const int S = p.S, n = p.n;
  const double h = 1.0 / n;
  auto& L = p.w.L32;
  uint32_t np = 0;
  const bool dir = dir_fusable<float>(ctx, L, S);
  // restart the inner solve: rin = (float) r64, d = 0, z = M^-1 rin, p = z
  // (with the fused direction, the first iteration forms z and p)
  if (int rc = masks(p)) return rc;
  {
    SolveState ir = view(p.w.inner.s, p.m_restart, p.phase);
    SolveState orr = view(p.w.outer.s, p.m_restart, p.phase);
    SRV_LAUNCH(launch_demote(n, S, p.w.r64, p.w.rin, orr, st));
    if (!dir)   // a fused-direction correction starts fresh
      SRV_LAUNCH(launch_fill_interior<float>(n, S, p.w.d, 0.0, p.m_restart, st));
    SRV_LAUNCH(launch_dot<float>(n, S, p.w.rin, p.w.rin, ir, &np, st));
    SRV_LAUNCH(launch_reduce(S, RED_BB, 0.0, np, ir, nullptr, st));
    if (dir) {
      // the first iteration preconditions rin itself
      if (int rc = pcg_dir_begin<float>(ctx, L, S, ir, p.w.rin, p.m_restart, true)) return rc;
    } else {
      float* z = nullptr;
      np = 0;
      if (int rc = precondition<float>(ctx, L, S, p.w.rin, &z, ir, &np)) return rc;
      if (!np) SRV_LAUNCH(launch_dot<float>(n, S, p.w.rin, z, ir, &np, st));
      SRV_LAUNCH(launch_reduce(S, RED_RZ_INIT, 0.0, np, ir, nullptr, st));
      SRV_LAUNCH(launch_copy<float>(n, S, z, p.w.p32, ir, st));
    }
    SRV_LAUNCH(launch_set_phase_mask(S, p.m_restart, p.phase, PHASE_INNER, nullptr, st));
  }
  // one inner iteration
  if (int rc = masks(p)) return rc;
  {
    SolveState ii = view(p.w.inner.s, p.w.inner.s.active, p.phase);
    const double tol2 = kInnerTol * kInnerTol;
    if (dir) {
      if (int rc = pcg_iteration_dir<float>(ctx, L, S, ii, p.w.d, p.w.rin, p.w.p32, p.w.p32b, p.w.q32, tol2,
                                            RED_RR_INNER, false, false, p.w.rin2))
        return rc;
    } else if (int rc = pcg_iteration<float>(ctx, L, S, ii, p.w.d, p.w.rin, p.w.p32, p.w.q32, tol2, RED_RR_INNER,
                                             false)) {
      return rc;
    }
  }
  // fp64 refinement of converged inner solves
  if (int rc = masks(p)) return rc;
  {
    SolveState ot = view(p.w.outer.s, p.m_trans, p.phase);
    if (dir)   // the update the inner solve's last step still owes d
      SRV_LAUNCH(launch_pcg_finish<float>(n, S, p.w.d, p.w.p32, p.w.p32b, p.m_trans, p.w.inner.s, st));
    SRV_LAUNCH(launch_add_correction(n, S, p.u, p.w.d, ot, st));
    SRV_LAUNCH(launch_true_residual(n, S, p.kap64, h * h * h, p.u, p.w.r64, ot, &np, st, zv<double>(ctx)));
    SRV_LAUNCH(launch_reduce(S, RED_RR_OUTER, ctx->cfg.rtol * ctx->cfg.rtol, np, ot, nullptr, st));
  }
  // QoI of finished slots
  if (int rc = masks(p)) return rc;
  {
    SolveState dn = view(p.w.outer.s, p.m_done, p.phase);
    SRV_LAUNCH(launch_qoi_partial(n, S, ctx->cfg.qoi, p.u, dn, &np, st, true));
    SRV_LAUNCH(launch_reduce(S, RED_STORE, 0.0, np, dn, p.q, st));
  }
  HIPCHK(hipMemcpyAsync(p.h_phase, p.phase, S * sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(p.h_q, p.q, S * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(p.h_iters, p.w.inner.s.iters, S * sizeof(int), hipMemcpyDeviceToHost, st));
  SRV_LAUNCH(launch_set_phase_mask(S, p.m_done, p.phase, PHASE_FREE, nullptr, st));
  HIPCHK(hipStreamSynchronize(st));
  return MLMC_OK;
}

// Pool set-up: carve its buffers from `off` in the arena, its engine view
// (shared tables, own stream and pinned counter), pinned host arrays, and the
// region cleared (zero boundaries, every slot free).
int init_pool(mlmc_ctx* ctx, Pool& p, size_t off, int m, int S) {
  Carver cv;
  cv.base = (char*)ctx->cfg.arena;
  cv.cap = ctx->cfg.arena_bytes;
  cv.top = off;
  cv.dry = false;
  p.carve(cv, ctx->cfg, m, S);
  p.slot_bytes = pool_bytes(ctx->cfg, m, 1);
  p.sub.cfg = ctx->cfg;
  p.sub.modes = ctx->modes;
  p.sub.K1 = ctx->K1;
  p.sub.d_sqrtlam = ctx->d_sqrtlam;
  p.sub.d_triples = ctx->d_triples;
  p.sub.d_xperm = ctx->d_xperm;
  p.sub.d_xoff = ctx->d_xoff;
  p.sub.d_tab = ctx->d_tab;
  p.sub.cheb = ctx->cheb;
  p.sub.zvar[0] = ctx->zvar[0];
  p.sub.zvar[1] = ctx->zvar[1];
  p.sub.vsmall_n0[0] = ctx->vsmall_n0[0];
  p.sub.vsmall_n0[1] = ctx->vsmall_n0[1];
  p.sub.fuse = ctx->fuse;
  p.sub.use_graphs = false;
  p.busy.assign(S, 0);
  p.job.assign(S, Job{});
  if (hipStreamCreate(&p.sub.st) != hipSuccess) return MLMC_E_DEVICE;
  p.sub.own_stream = true;
  if (hipHostMalloc((void**)&p.h_ids, S * sizeof(uint64_t), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&p.h_lv, S * sizeof(int), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&p.h_slots, S * sizeof(int), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&p.h_phase, S * sizeof(int), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&p.h_iters, S * sizeof(int), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&p.h_q, S * sizeof(double), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&p.sub.h_nactive, sizeof(int), hipHostMallocDefault) != hipSuccess)
    return MLMC_E_DEVICE;
  if (hipMemsetAsync((char*)ctx->cfg.arena + off, 0, cv.top - off, p.sub.st) != hipSuccess ||
      hipStreamSynchronize(p.sub.st) != hipSuccess)
    return MLMC_E_DEVICE;
  return MLMC_OK;
}

// The pool's stream and pinned host arrays (idempotent).
void free_pool(Pool& p) {
  if (p.sub.st) {
    (void)hipStreamSynchronize(p.sub.st);   // teardown: nothing to report to
    (void)hipStreamDestroy(p.sub.st);
    p.sub.st = nullptr;
  }
  for (void** h : {(void**)&p.h_ids, (void**)&p.h_lv, (void**)&p.h_slots, (void**)&p.h_phase, (void**)&p.h_iters,
                   (void**)&p.h_q, (void**)&p.sub.h_nactive})
    if (*h) {
      (void)hipHostFree(*h);
      *h = nullptr;
    }
}

void pool_loop(mlmc_server* srv, Pool* p);

// Called by main pool P after its step, server mutex held: when P's queue
// holds more jobs than its free slots, and another main pool is idle with a region that
// holds a pool of P's mesh and slot count, that region takes a guest pool for
// P (the same slot count, so each slot's arithmetic is that of P's own
// slots).  The guest's set-up runs under the mutex (a stream, pinned arrays
// and one clear of the region).
void maybe_lend(mlmc_server* srv, Pool* P) {
  // more queued than P's free slots take at its next admission
  if (srv->stopping || P->helper || P->S == 0 || (int64_t)P->queue.size() <= (int64_t)(P->S - P->occupied)) return;
  mlmc_ctx* ctx = srv->ctx;
  const size_t need = pool_bytes(ctx->cfg, P->m, P->S);
  for (auto& lp : srv->pools) {
    Pool* L = lp.get();
    if (L == P || L->S == 0 || L->guest || L->helper || L->occupied > 0 || !L->queue.empty() || L->region_bytes < need)
      continue;
    std::unique_ptr<Pool> g(new Pool());
    if (init_pool(ctx, *g, L->region_off, P->m, P->S) != MLMC_OK) {
      free_pool(*g);
      return;
    }
    g->owner = P;
    P->helper = g.get();
    L->guest = std::move(g);
    srv->lends++;
    L->guest->th = std::thread(pool_loop, srv, L->guest.get());
    return;
  }
}

// Called by lent main pool L whose own queue has work, server mutex held
// through lk: the guest stops admitting and finishes its slots, then L's
// region is cleared and L serves again.  False when the server stops (or
// the clear fails) meanwhile.
bool reclaim(mlmc_server* srv, Pool* L, std::unique_lock<std::mutex>& lk) {
  Pool* g = L->guest.get();
  g->closing = true;
  srv->cv.notify_all();
  srv->cv.wait(lk, [&] { return srv->stopping || g->exited; });
  if (srv->stopping) return false;   // serve_stop joins and frees the guest
  lk.unlock();
  if (g->th.joinable()) g->th.join();
  free_pool(*g);
  const bool ok = hipMemsetAsync((char*)srv->ctx->cfg.arena + L->region_off, 0, L->region_bytes, L->sub.st) == hipSuccess &&
                  hipStreamSynchronize(L->sub.st) == hipSuccess;
  lk.lock();
  g->owner->helper = nullptr;
  L->guest.reset();
  srv->reclaims++;
  if (!ok) {
    srv->error = MLMC_E_DEVICE;
    srv->error_msg = "clearing a returned pool region failed";
    srv->stopping = true;
    srv->cv.notify_all();
    return false;
  }
  return true;
}

void pool_loop(mlmc_server* srv, Pool* p) {
  const int max_iter = srv->ctx->cfg.max_iter;
  std::vector<int> steps(p->S, 0);
  Pool* src = p->owner ? p->owner : p;   // the pool whose queue feeds these slots
  for (;;) {
    int c = 0;
    {
      std::unique_lock<std::mutex> lk(srv->mu);
      srv->cv.wait(lk, [&] {
        if (srv->stopping) return true;
        if (p->owner) return p->occupied > 0 || p->closing || (!src->queue.empty() && p->occupied < p->S);
        if (p->guest) return !p->queue.empty();   // lent: wake to take the region back
        return p->occupied > 0 || (!p->queue.empty() && p->occupied < p->S);
      });
      if (srv->stopping || (p->owner && p->closing && p->occupied == 0)) {
        if (p->owner) p->exited = true;
        srv->cv.notify_all();
        return;
      }
      if (p->guest) {
        if (!reclaim(srv, p, lk)) return;
        continue;
      }
      for (int s = 0; s < p->S && !src->queue.empty() && !p->closing; ++s) {
        if (p->busy[s]) continue;
        const Job j = src->queue.front();
        src->queue.pop_front();
        p->busy[s] = 1;
        p->job[s] = j;
        steps[s] = 0;
        p->occupied++;
        p->h_ids[c] = j.sample;
        p->h_lv[c] = j.level;
        p->h_slots[c] = s;
        ++c;
        auto it = srv->reqs.find(j.ticket);
        if (it != srv->reqs.end() && it->second.t_admit < 0) it->second.t_admit = srv->now();
      }
    }
    const double t_step = srv->now();
    int rc = c ? setup_slots(*p, c) : MLMC_OK;
    if (!rc) rc = step(*p);
    std::lock_guard<std::mutex> lk(srv->mu);
    src->busy_slot_s += (double)p->occupied * (srv->now() - t_step);   // a guest's slots count for its mesh
    if (rc) {
      srv->error = rc;
      srv->error_msg = p->sub.err;
      srv->stopping = true;
      if (p->owner) p->exited = true;
      srv->cv.notify_all();
      return;
    }
    const double t = srv->now();
    for (int s = 0; s < p->S; ++s) {
      if (!p->busy[s]) continue;
      steps[s]++;
      const bool done = p->h_phase[s] == PHASE_DONE;
      const bool stuck = !done && steps[s] > 4 * max_iter;   // safety net: never converging
      if (!done && !stuck) continue;
      const Job& j = p->job[s];
      auto it = srv->reqs.find(j.ticket);
      if (it != srv->reqs.end()) {
        Request& r = it->second;
        const double qv = p->h_q[s];
        if (j.fine) {
          r.qf = qv;
          r.iters = p->h_iters[s];
        } else {
          r.qc = qv;
        }
        if (stuck) r.status = MLMC_E_NOCONV;
        if (!std::isfinite(qv)) r.status = MLMC_E_NONFINITE;
        srv->dofs_done += (double)(p->n - 1) * (p->n - 1) * (p->n - 1);
        if (--r.pending == 0) {
          r.done = true;
          r.t_done = t;
          srv->completed++;
          srv->last_done = t;
          srv->finished.push_back(j.ticket);
        }
      }
      if (stuck) {
        // the slot's device phase is reset with the next admission of the slot
        p->h_phase[s] = PHASE_FREE;
      }
      p->busy[s] = 0;
      p->occupied--;
    }
    if (!p->owner) maybe_lend(srv, p);
    srv->cv.notify_all();
    srv->done_cv.notify_all();
  }
}

void fill_result(const Request& r, uint64_t ticket, mlmc_sample_result* out) {
  out->ticket = ticket;
  out->status = r.status;
  out->level = r.level;
  out->sample = r.sample;
  out->q_fine = r.qf;
  out->q_coarse = r.level > 0 ? r.qc : 0.0;
  out->y = out->q_fine - out->q_coarse;
  out->iters = r.iters;
  out->latency_s = r.t_done - r.t_submit;
  out->queue_s = (r.t_admit >= 0 ? r.t_admit : r.t_done) - r.t_submit;
}

}  // namespace

extern "C" {

int mlmc_serve_start(mlmc_ctx* ctx, const int32_t* slots_per_mesh) {
  if (!ctx) return MLMC_E_INVALID;
  if (ctx->server) FAIL(MLMC_E_INVALID, "already serving");
  if (ctx->cfg.solver != MLMC_SOLVER_GMG_PCG) FAIL(MLMC_E_INVALID, "serving runs the GMG-PCG solver");
  if (ctx->cfg.forcing != MLMC_FORCING_CONSTANT) FAIL(MLMC_E_INVALID, "serving solves with f = 1");
  const int L = ctx->cfg.levels;
  std::vector<int> S(L, 0);
  const size_t avail = ctx->cfg.arena_bytes - ctx->persistent_top;
  if (slots_per_mesh) {
    for (int m = 0; m < L; ++m) {
      if (slots_per_mesh[m] < 0) FAIL(MLMC_E_INVALID, "negative slot count");
      S[m] = slots_per_mesh[m];
    }
  } else {
    // equal share of the budget per mesh, at most 4096 slots each
    for (int m = 0; m < L; ++m) {
      const size_t per = pool_bytes(ctx->cfg, m, 1);
      const size_t share = (size_t)(0.95 * (double)avail / L);
      S[m] = (int)std::min<size_t>(4096, share / per);
    }
  }
  // each mesh's region: its pool, or with the default split its whole share
  // (so that an idle region can take a guest pool of another mesh)
  std::vector<size_t> region(L, 0);
  size_t need = ctx->persistent_top;
  for (int m = 0; m < L; ++m) {
    if (S[m] == 0) continue;
    region[m] = align256(slots_per_mesh ? pool_bytes(ctx->cfg, m, S[m])
                                        : std::max(pool_bytes(ctx->cfg, m, S[m]),
                                                   (size_t)(0.95 * (double)avail / L)));
    need += region[m];
  }
  if (need > ctx->cfg.arena_bytes)
    FAIL(MLMC_E_NOMEM, "arena too small for the serving pools: need " + std::to_string(need) + " bytes");
  // the pools take over the arena after the persistent tables
  drop_work(ctx);
  auto* srv = new mlmc_server();
  srv->ctx = ctx;
  ctx->server = srv;
  size_t off = ctx->persistent_top;
  int rc = MLMC_OK;
  for (int m = 0; m < L; ++m) {
    srv->pools.emplace_back(new Pool());
    Pool& p = *srv->pools.back();
    p.m = m;
    p.n = ctx->cfg.n0 << m;
    if (S[m] == 0 || rc) continue;
    p.region_off = off;
    p.region_bytes = region[m];
    off += region[m];
    rc = init_pool(ctx, p, p.region_off, m, S[m]);
  }
  if (rc) {
    mlmc_serve_stop(ctx);
    FAIL(rc, "serving set-up failed");
  }
  for (auto& p : srv->pools)
    if (p->S > 0) p->th = std::thread(pool_loop, srv, p.get());
  return MLMC_OK;
}

int mlmc_serve_stop(mlmc_ctx* ctx) {
  if (!ctx) return MLMC_E_INVALID;
  mlmc_server* srv = ctx->server;
  if (!srv) return MLMC_OK;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stopping = true;
  }
  srv->cv.notify_all();
  srv->done_cv.notify_all();
  // main pools first (a lent pool's thread may be taking its region back),
  // then the guests still in a region
  for (auto& p : srv->pools)
    if (p->th.joinable()) p->th.join();
  for (auto& p : srv->pools)
    if (p->guest) {
      if (p->guest->th.joinable()) p->guest->th.join();
      free_pool(*p->guest);
      p->guest.reset();
    }
  for (auto& p : srv->pools) free_pool(*p);
  ctx->server = nullptr;
  delete srv;
  return MLMC_OK;
}

int mlmc_submit_batch(mlmc_ctx* ctx, int32_t count, const int32_t* levels, const uint64_t* samples,
                      uint64_t* tickets) {
  if (!ctx || count < 0 || (count > 0 && (!levels || !samples || !tickets))) return MLMC_E_INVALID;
  mlmc_server* srv = ctx->server;
  if (!srv) return MLMC_E_INVALID;
  std::lock_guard<std::mutex> lk(srv->mu);
  if (srv->error) return srv->error;
  if (srv->stopping) return MLMC_E_INVALID;
  for (int i = 0; i < count; ++i) {
    const int level = levels[i];
    if (level < 0 || level >= ctx->cfg.levels) return MLMC_E_INVALID;
    if (srv->pools[level]->S == 0 || (level > 0 && srv->pools[level - 1]->S == 0)) return MLMC_E_BUDGET;
  }
  const double now = srv->now();
  for (int i = 0; i < count; ++i) {
    const int level = levels[i];
    const uint64_t t = srv->next_ticket++;
    Request r;
    r.level = level;
    r.sample = samples[i];
    r.t_submit = now;
    r.pending = level > 0 ? 2 : 1;
    srv->reqs.emplace(t, r);
    srv->pools[level]->queue.push_back(Job{t, level, samples[i], true});
    if (level > 0) srv->pools[level - 1]->queue.push_back(Job{t, level, samples[i], false});
    tickets[i] = t;
  }
  if (count && srv->first_submit < 0) srv->first_submit = now;
  srv->cv.notify_all();
  return MLMC_OK;
}

int mlmc_submit(mlmc_ctx* ctx, int32_t level, uint64_t sample_id, uint64_t* ticket) {
  if (!ticket) return MLMC_E_INVALID;
  return mlmc_submit_batch(ctx, 1, &level, &sample_id, ticket);
}

int mlmc_poll(mlmc_ctx* ctx, uint64_t ticket, mlmc_sample_result* out) {
  if (!ctx || !out) return MLMC_E_INVALID;
  mlmc_server* srv = ctx->server;
  if (!srv) return MLMC_E_INVALID;
  std::lock_guard<std::mutex> lk(srv->mu);
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end()) return srv->error ? srv->error : MLMC_E_INVALID;
  const Request& r = it->second;
  if (!r.done) return srv->error ? srv->error : MLMC_PENDING;
  fill_result(r, ticket, out);
  srv->reqs.erase(it);
  return MLMC_OK;
}

int mlmc_drain(mlmc_ctx* ctx, mlmc_sample_result* out, int32_t max, int32_t* n, double timeout_s) {
  if (!ctx || !out || !n || max < 1) return MLMC_E_INVALID;
  *n = 0;
  mlmc_server* srv = ctx->server;
  if (!srv) return MLMC_E_INVALID;
  std::unique_lock<std::mutex> lk(srv->mu);
  srv->done_cv.wait_for(lk, std::chrono::duration<double>(std::max(0.0, timeout_s)),
                        [&] { return !srv->finished.empty() || srv->error || srv->stopping; });
  int k = 0;
  while (k < max && !srv->finished.empty()) {
    const uint64_t t = srv->finished.front();
    srv->finished.pop_front();
    auto it = srv->reqs.find(t);
    if (it == srv->reqs.end()) continue;   // already taken by mlmc_poll
    fill_result(it->second, t, out + k);
    srv->reqs.erase(it);
    ++k;
  }
  *n = k;
  return srv->error;
}

int mlmc_serve_stats(mlmc_ctx* ctx, mlmc_serve_stats_out* out) {
  if (!ctx || !out) return MLMC_E_INVALID;
  mlmc_server* srv = ctx->server;
  if (!srv) return MLMC_E_INVALID;
  std::lock_guard<std::mutex> lk(srv->mu);
  out->completed = srv->completed;
  out->sample_dofs = srv->dofs_done;
  out->busy_seconds = srv->first_submit >= 0 ? srv->last_done - srv->first_submit : 0.0;
  int q = 0, occ = 0;
  for (int m = 0; m < (int)srv->pools.size() && m < 16; ++m) {
    const Pool& p = *srv->pools[m];
    // a mesh's slots: its own pool unless lent out, plus its guest elsewhere
    const int gs = p.helper ? p.helper->S : 0, go = p.helper ? p.helper->occupied : 0;
    out->slots[m] = (p.guest ? 0 : p.S) + gs;
    out->occupied[m] = p.occupied + go;
    out->slot_busy_s[m] = p.busy_slot_s;
    out->slot_bytes[m] = (double)p.slot_bytes;
    q += (int)p.queue.size();
    occ += p.occupied + go;
  }
  out->lends = srv->lends;
  out->reclaims = srv->reclaims;
  out->queued = q;
  out->running = occ;
  out->uptime_s = srv->now();
  return srv->error;
}

}  // extern "C"
