// Serving under concurrent clients, for an AddressSanitizer build of the
// library's host code: three client threads submit and poll requests of
// both levels while a fourth reads the server's counters, then the main
// thread stops the server and destroys the context.  Exit status 0 when
// every request finished with MLMC_OK and the counters add up;
// AddressSanitizer reports invalid or freed-memory accesses of the request
// map, queues and pools on stderr and fails the run.
#include <hip/hip_runtime_api.h>

#include <atomic>
#include <cstdio>
#include <cstring>
#include <thread>
#include <vector>

#include "mlmc.h"

namespace {

constexpr int kClients = 3, kPerClient = 12;

int fail(const char* what, int rc, mlmc_ctx* ctx) {
  std::fprintf(stderr, "%s: rc %d (%s)\n", what, rc, mlmc_last_error(ctx));
  return 1;
}

}  // namespace

int main() {
  void* arena = nullptr;
  const size_t bytes = (size_t)1 << 30;
  int ndev = 0;
  const hipError_t ec = hipGetDeviceCount(&ndev);
  const hipError_t em = ec == hipSuccess && ndev > 0 ? hipMalloc(&arena, bytes) : ec;
  if (em != hipSuccess || ndev < 1) {
    std::fprintf(stderr, "no device memory: %s (devices %d)\n", hipGetErrorString(em), ndev);
    return 2;
  }
  mlmc_config c;
  std::memset(&c, 0, sizeof c);
  c.n0 = 8;
  c.levels = 2;
  c.sigma2 = 1.0;
  c.corr_len = 0.5;
  c.n_modes = 8;
  c.seed = 7;
  c.qoi = MLMC_QOI_DOMAIN_AVERAGE;
  c.rtol = 1e-8;
  c.max_iter = 400;
  c.precision = MLMC_PREC_MIXED;
  c.solver = MLMC_SOLVER_GMG_PCG;
  c.max_batch = 8;
  c.arena = arena;
  c.arena_bytes = bytes;
  mlmc_ctx* ctx = nullptr;
  if (int rc = mlmc_create(&c, &ctx)) return fail("create", rc, nullptr);
  const int32_t slots[2] = {6, 4};
  if (int rc = mlmc_serve_start(ctx, slots)) return fail("serve_start", rc, ctx);

  std::atomic<int> bad{0}, done{0};
  std::atomic<bool> clients_done{false};
  std::vector<std::thread> th;
  for (int t = 0; t < kClients; ++t) {
    th.emplace_back([&, t] {
      std::vector<uint64_t> tickets;
      for (int i = 0; i < kPerClient; ++i) {
        uint64_t tk = 0;
        if (mlmc_submit(ctx, (t + i) % 2, (uint64_t)(100 * t + i), &tk) != MLMC_OK) {
          ++bad;
          return;
        }
        tickets.push_back(tk);
      }
      for (uint64_t tk : tickets) {
        mlmc_sample_result r;
        for (;;) {
          const int rc = mlmc_poll(ctx, tk, &r);
          if (rc == MLMC_PENDING) {
            std::this_thread::yield();
            continue;
          }
          if (rc != MLMC_OK || r.status != MLMC_OK) ++bad;
          ++done;
          break;
        }
      }
    });
  }
  std::thread watcher([&] {
    mlmc_serve_stats_out s;
    while (!clients_done.load()) {
      if (mlmc_serve_stats(ctx, &s) != MLMC_OK) ++bad;
      std::this_thread::yield();
    }
  });
  for (auto& x : th) x.join();
  clients_done = true;
  watcher.join();
  mlmc_serve_stats_out s;
  if (int rc = mlmc_serve_stats(ctx, &s)) return fail("serve_stats", rc, ctx);
  if (int rc = mlmc_serve_stop(ctx)) return fail("serve_stop", rc, ctx);
  mlmc_destroy(ctx);
  hipFree(arena);
  const int want = kClients * kPerClient;
  std::printf("requests %d done %d bad %d completed %llu\n", want, done.load(), bad.load(),
              (unsigned long long)s.completed);
  return (bad.load() == 0 && done.load() == want && s.completed == (uint64_t)want) ? 0 : 1;
}
