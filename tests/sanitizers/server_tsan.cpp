// The serving loop under a host sanitizer (ThreadSanitizer, or AddressSanitizer
// with UndefinedBehaviorSanitizer; host code only): two caller threads
// submit requests and poll their tickets while a third reads the server's
// statistics, against the server's own worker thread that forms batches,
// launches them on its streams and completes them.  Exits nonzero if a
// request fails; ThreadSanitizer reports data races on stderr.
//
// Build (from the repository root) and run: tests/sanitizers/run_tsan.sh
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdio>
#include <random>
#include <thread>
#include <vector>

#include "dmx.h"

int main() {
  // one free sphere (radius 0.1 m, 1 kg) over a plane, the six free-joint
  // dofs controlled
  const int32_t parent[1] = {-1}, iner_type[1] = {DMX_GEOM_SPHERE}, jb[1] = {0}, jt[1] = {DMX_JOINT_FREE};
  const double bpos[3] = {0, 0, 0}, bquat[4] = {1, 0, 0, 0}, isize[3] = {0.1, 0, 0}, iquat[4] = {1, 0, 0, 0};
  const double mass[1] = {1.0}, jaxis[3] = {0, 0, 1}, jpos[3] = {0, 0, 0};
  const int32_t gbody[2] = {-1, 0}, gtype[2] = {DMX_GEOM_PLANE, DMX_GEOM_SPHERE};
  const double gsize[6] = {0, 0, 0, 0.1, 0, 0}, gpos[6] = {0, 0, 0, 0, 0, 0}, gquat[8] = {1, 0, 0, 0, 1, 0, 0, 0};
  const int32_t g1[1] = {0}, g2[1] = {1};
  const double mu[1] = {1.0}, solref[2] = {0.002, 1.0}, solimp[5] = {0.9, 0.95, 0.001, 0.5, 2.0};
  const double cfd[5] = {0.0, 0.9, 0.01, 1.0, 4.0};
  const int32_t ctrl[6] = {0, 1, 2, 3, 4, 5};
  dmx_model_desc d{};
  d.nbody = 1; d.njnt = 1; d.ngeom = 2; d.npair = 1; d.nu = 6;
  d.body_parent = parent; d.body_pos = bpos; d.body_quat = bquat; d.body_iner_type = iner_type;
  d.body_iner_size = isize; d.body_iner_quat = iquat; d.body_mass = mass;
  d.jnt_body = jb; d.jnt_type = jt; d.jnt_axis = jaxis; d.jnt_pos = jpos;
  d.geom_body = gbody; d.geom_type = gtype; d.geom_size = gsize; d.geom_pos = gpos; d.geom_quat = gquat;
  d.pair_g1 = g1; d.pair_g2 = g2; d.pair_mu = mu; d.pair_solref = solref; d.pair_solimp = solimp; d.pair_cfd = cfd;
  d.ctrl_dof = ctrl;
  d.gravity[2] = -9.81;
  dmx_model* m = nullptr;
  if (dmx_model_create(&d, &m) != DMX_OK) { std::fprintf(stderr, "model: %s\n", dmx_last_error()); return 2; }
  dmx_server_opts so;
  dmx_default_server_opts(&so);
  so.hbm_budget_bytes = 1ll << 30;
  so.n_streams = 4;
  so.max_inflight = 4;
  dmx_server* sv = nullptr;
  if (dmx_server_create(&so, &sv) != DMX_OK) { std::fprintf(stderr, "server: %s\n", dmx_last_error()); return 2; }
  std::atomic<int> failed{0}, done{0};
  std::atomic<bool> stop{false};
  auto caller = [&](int seed) {
    std::mt19937_64 rng(seed);
    std::uniform_real_distribution<double> U(-1.0, 1.0);
    for (int it = 0; it < 12; ++it) {
      const int N = 8 + (int)(rng() % 24), H = 3 + (int)(rng() % 8);
      std::vector<double> x0(13, 0.0), u((size_t)N * H * 6), cost(N), grad((size_t)N * H * 6);
      std::vector<int32_t> st(N);
      x0[2] = 0.3; x0[3] = 1.0;
      for (double& v : u) v = U(rng);
      dmx_request q{};
      q.model = m; q.n_worlds = N; q.n_intervals = H; q.interval_dt = 0.01; q.x0 = x0.data(); q.u = u.data();
      q.target[2] = 0.2; q.ctrl_weight = 1e-3; q.want_grad = 1;
      uint64_t t = 0;
      if (dmx_submit(sv, &q, &t) != DMX_OK) { failed++; continue; }
      dmx_result r{};
      r.cost = cost.data(); r.grad_u = grad.data(); r.world_status = st.data();
      dmx_status s;
      while ((s = dmx_poll(sv, t, &r)) == DMX_PENDING) std::this_thread::yield();
      if (s != DMX_OK) { failed++; continue; }
      for (int w = 0; w < N; ++w) if (st[w] != 0) failed++;
      done++;
    }
  };
  std::thread watcher([&] {
    while (!stop.load()) {
      int32_t qd = 0, inf = 0;
      int64_t bytes = 0;
      (void)dmx_server_stats(sv, &qd, &inf, &bytes);
      std::this_thread::yield();
    }
  });
  std::thread a(caller, 1), b(caller, 2);
  a.join();
  b.join();
  stop.store(true);
  watcher.join();
  dmx_server_destroy(sv);
  dmx_model_destroy(m);
  std::printf("server under the host sanitizer: %d requests done, %d failures\n", done.load(), failed.load());
  return failed.load() ? 1 : 0;
}
