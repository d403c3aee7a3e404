// Pause-model stress of the scheduler (Sec. 5.1, "A benchmarking example"):
// host side.  The model of a sample only waits, so the run measures the
// scheduling through the active ratio A(p) = a(p) / (p t_w(p)) of
// eq. active_ratio.  Durations are drawn on the device (Philox, see
// k_pause_draw) and counted in ticks of the device wall clock; the schedule is
// a host loop of steps, one device launch each:
//   * tasks (batch consecutive samples of one level, the batch sampling of
//     Sec. 4.2) are queued finest level first, in sample order (the
//     finest-first rule of Alg. incremental_greedy);
//   * at a step boundary every queued task that fits the free workgroup
//     slots is admitted, in queue order (tasks of a level have one width, so
//     this is a count per level);
//   * the step lasts max(min_step, least remaining time of a running task);
//     each running task's workgroups wait min(remaining, step) and tasks whose
//     time is used up finish at the end of the step.
// Every decision is integer arithmetic on the tick counts, so the schedule is
// reproducible from the durations alone.
#pragma clang fp contract(off)

#include "engine.hpp"

#include <chrono>
#include <cmath>

namespace {

struct PauseTask {
  int level = 0;
  int width = 0;
  int64_t first = 0;     // index of the task's first sample in the level-major sample list
  int64_t n = 0;         // samples in the task
  uint64_t rem = 0;      // ticks still to wait
};

}  // namespace

extern "C" int mlmc_pause_model(mlmc_ctx* ctx, const mlmc_pause_opts* o, int64_t* ticks, int64_t* done_step,
                                mlmc_pause_out* out) {
  if (!ctx) return MLMC_E_INVALID;
  if (ctx->server) FAIL(MLMC_E_INVALID, "the context is serving");
  if (!o || !out || o->n_levels < 1 || o->n_levels > 16 || !o->counts || !o->widths)
    FAIL(MLMC_E_INVALID, "bad pause-model arguments");
  if (!(o->capacity >= 1 && o->capacity <= 8192) || o->batch < 1)
    FAIL(MLMC_E_INVALID, "pause model: capacity must be 1..8192 and batch >= 1");
  const double s3 = std::sqrt(3.0) * o->sigma_us;
  if (!(o->mu_us > 0.0) || !(o->sigma_us >= 0.0) || !(o->mu_us - s3 >= 0.0) || !(o->min_step_us >= 0.0))
    FAIL(MLMC_E_INVALID, "pause model: need mu > 0 and 0 <= sigma <= mu / sqrt(3), min_step >= 0");
  int64_t total = 0;
  for (int l = 0; l < o->n_levels; ++l) {
    if (o->counts[l] < 0 || o->widths[l] < 1 || o->widths[l] > o->capacity)
      FAIL(MLMC_E_INVALID, "pause model: counts >= 0 and widths in 1..capacity");
    total += o->counts[l];
    if (total > (int64_t)1 << 24) FAIL(MLMC_E_INVALID, "pause model: at most 2^24 samples");
  }
  int khz = 0;
  HIPCHK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, 0));
  if (khz <= 0) FAIL(MLMC_E_DEVICE, "no device wall clock rate");
  const double f = khz / 1000.0;   // ticks per microsecond
  const double a = o->mu_us - s3, w = 2.0 * s3;
  // a step waits at most max(min_step, longest task) ticks in a 32-bit count
  const double longest = (a + w) * (double)o->batch * f, minstep = o->min_step_us * f;
  if (longest > 2147483647.0 || minstep > 2147483647.0)
    FAIL(MLMC_E_INVALID, "pause model: a task or the shortest step exceeds 2^31 clock ticks");

  // device scratch right after the persistent tables (the cached work space
  // there is dropped and carved again when next needed)
  const int P = o->capacity;
  const size_t dur_b = align256((size_t)(total > 0 ? total : 1) * sizeof(double));
  const size_t spin_b = align256((size_t)P * sizeof(uint32_t)), meas_b = align256((size_t)P * sizeof(uint64_t));
  if (ctx->persistent_top + dur_b + spin_b + meas_b > ctx->cfg.arena_bytes)
    FAIL(MLMC_E_NOMEM, "arena too small for the pause-model draws");
  drop_work(ctx);
  char* base = (char*)ctx->cfg.arena + ctx->persistent_top;
  double* d_dur = reinterpret_cast<double*>(base);
  uint32_t* d_spin = reinterpret_cast<uint32_t*>(base + dur_b);
  uint64_t* d_meas = reinterpret_cast<uint64_t*>(base + dur_b + spin_b);

  // durations, level-major, as ticks
  std::vector<int64_t> off(o->n_levels + 1, 0);
  for (int l = 0; l < o->n_levels; ++l) off[l + 1] = off[l] + o->counts[l];
  for (int l = 0; l < o->n_levels; ++l)
    LAUNCH(MLMC_K_MISC, 0, launch_pause_draw(ctx->cfg.seed, l, o->counts[l], a, w, d_dur + off[l], ctx->st));
  std::vector<double> dur((size_t)total);
  if (total > 0) HIPCHK(hipMemcpyAsync(dur.data(), d_dur, (size_t)total * sizeof(double), hipMemcpyDeviceToHost, ctx->st));
  HIPCHK(hipMemsetAsync(d_meas, 0, (size_t)P * sizeof(uint64_t), ctx->st));
  HIPCHK(hipStreamSynchronize(ctx->st));
  std::vector<uint64_t> tk((size_t)total);
  for (int64_t s = 0; s < total; ++s) {
    const double x = dur[(size_t)s] * f;
    tk[(size_t)s] = (uint64_t)std::floor(x + 0.5);
  }
  if (ticks)
    for (int64_t s = 0; s < total; ++s) ticks[s] = (int64_t)tk[(size_t)s];

  // tasks, finest level first
  std::vector<PauseTask> tasks;
  std::vector<int64_t> lv_first(o->n_levels, 0), lv_end(o->n_levels, 0);   // task ranges per level
  for (int l = o->n_levels - 1; l >= 0; --l) {
    lv_first[l] = (int64_t)tasks.size();
    for (int64_t i = 0; i < o->counts[l]; i += o->batch) {
      PauseTask t;
      t.level = l;
      t.width = o->widths[l];
      t.first = off[l] + i;
      t.n = std::min<int64_t>(o->batch, o->counts[l] - i);
      for (int64_t q = 0; q < t.n; ++q) t.rem += tk[(size_t)(t.first + q)];
      tasks.push_back(t);
    }
    lv_end[l] = (int64_t)tasks.size();
  }
  double active_ticks = 0.0;
  for (const PauseTask& t : tasks) active_ticks += (double)t.width * (double)t.rem;

  uint32_t* h_spin = nullptr;
  HIPCHK(hipHostMalloc((void**)&h_spin, (size_t)P * sizeof(uint32_t), hipHostMallocDefault));
  std::vector<int64_t> next(lv_first);   // next queued task of each level
  std::vector<int64_t> running;
  int free_slots = P;
  int64_t steps = 0;
  double ideal_ticks = 0.0;
  int rc = MLMC_OK;
  const auto t0 = std::chrono::steady_clock::now();
  while (true) {
    // admission, queue order: finest level first
    for (int l = o->n_levels - 1; l >= 0 && free_slots > 0; --l) {
      const int wl = o->widths[l];
      int64_t k = std::min<int64_t>(lv_end[l] - next[l], free_slots / wl);
      for (; k > 0; --k) {
        running.push_back(next[l]++);
        free_slots -= wl;
      }
    }
    if (running.empty()) break;
    uint64_t step = UINT64_MAX;
    for (int64_t id : running) step = std::min(step, tasks[(size_t)id].rem);
    step = std::max<uint64_t>(step, (uint64_t)std::floor(minstep + 0.5));
    int nwg = 0;
    for (int64_t id : running) {
      const PauseTask& t = tasks[(size_t)id];
      const uint32_t s = (uint32_t)std::min(t.rem, step);
      for (int q = 0; q < t.width; ++q) h_spin[nwg++] = s;
    }
    hipError_t e = hipMemcpyAsync(d_spin, h_spin, (size_t)nwg * sizeof(uint32_t), hipMemcpyHostToDevice, ctx->st);
    if (e == hipSuccess) e = launch_pause_spin(d_spin, d_meas, nwg, ctx->st);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->st);
    if (e != hipSuccess) {
      ctx->err = std::string("HIP error in the pause-model step: ") + hipGetErrorString(e);
      rc = MLMC_E_DEVICE;
      break;
    }
    ideal_ticks += (double)step;
    size_t keep = 0;
    for (size_t r = 0; r < running.size(); ++r) {
      PauseTask& t = tasks[(size_t)running[r]];
      t.rem -= std::min(t.rem, step);
      if (t.rem == 0) {
        free_slots += t.width;
        if (done_step)
          for (int64_t q = 0; q < t.n; ++q) done_step[t.first + q] = steps;
      } else {
        running[keep++] = running[r];
      }
    }
    running.resize(keep);
    ++steps;
  }
  const double wall = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  hipHostFree(h_spin);
  if (rc) return rc;
  std::vector<uint64_t> meas((size_t)P);
  HIPCHK(hipMemcpyAsync(meas.data(), d_meas, (size_t)P * sizeof(uint64_t), hipMemcpyDeviceToHost, ctx->st));
  HIPCHK(hipStreamSynchronize(ctx->st));
  double meas_ticks = 0.0;
  for (uint64_t m : meas) meas_ticks += (double)m;

  const double us = 1e-6;
  out->tasks = (int64_t)tasks.size();
  out->steps = steps;
  out->clock_mhz = f;
  out->wall_s = steps > 0 ? wall : 0.0;
  out->active_slot_s = active_ticks / f * us;
  out->ratio = out->wall_s > 0.0 ? out->active_slot_s / ((double)P * out->wall_s) : 0.0;
  out->ideal_ratio = ideal_ticks > 0.0 ? active_ticks / ((double)P * ideal_ticks) : 0.0;
  out->measured_slot_s = meas_ticks / f * us;
  return MLMC_OK;
}
