// Launch wrappers of the batched kernels and the table entries that name
// them.  Each kernel family is instantiated in its own translation unit
// (kern_free*.hip, kern_tree.hip), which exports its entry table; the host
// library (dmx_lib.hip) dispatches through the tables.
#pragma once
#include <hip/hip_runtime.h>

#include "dmx_free.hpp"
#include "dmx_rk.hpp"

namespace dmx_host {

using FwdFn = void (*)(const void*, const dmx::FwdArgs&, hipStream_t, int);
using AdjFn = void (*)(const void*, const dmx::AdjArgs&, hipStream_t, int);

// Batched form: one launch, one team of lanes per world.  Plain form
// (plain != 0): one launch per world with the same kernel, serialized on the
// stream (the baseline of the benchmark).
// Teams of a kernel the device holds at once (occupancy x compute units).
template <class K>
long long resident_teams(K kernel, int team) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 64, 0) != hipSuccess) return 0;
  return (long long)cus * per_cu * (64 / team);
}

// Grid of a batched launch: one team per world, or with a work queue as many
// teams as the device holds at once (at most one per world).
template <class P, class K>
int grid_blocks(K kernel, int W, bool queue) {
  long long teams = W;
  if (queue) {
    const long long r = resident_teams(kernel, P::TEAM);
    if (r > 0 && r < teams) teams = r;
  }
  return (int)((teams * P::TEAM + 63) / 64);
}

template <class P>
long long fwd_resident_teams() {
  static long long r = resident_teams(dmx::fwd_kernel<P>, P::TEAM);
  return r;
}

template <class P>
void launch_fwd(const void* model, const dmx::FwdArgs& a, hipStream_t s, int plain) {
  if (!plain) {
    const int blocks = grid_blocks<P>(dmx::fwd_kernel<P>, a.W, a.g.queue != nullptr);
    if (a.g.queue) hipLaunchKernelGGL(dmx::reset_queue, dim3(1), dim3(64), 0, s, a.g.queue);
    hipLaunchKernelGGL(dmx::fwd_kernel<P>, dim3(blocks), dim3(64), 0, s, (const typename P::Model*)model, a);
    return;
  }
  constexpr int NX = P::NQ + P::NV;
  for (int w = 0; w < a.W; ++w) {
    dmx::FwdArgs b = a;
    b.W = 1;
    b.x0 = a.x0 + (size_t)w * NX;
    b.u = a.u ? a.u + (size_t)w * a.n_int * a.nu : nullptr;
    b.xout = a.xout + (size_t)w * NX;
    b.status = a.status + w;
    b.n_acc = a.n_acc ? a.n_acc + w : nullptr;
    b.n_rej = a.n_rej ? a.n_rej + w : nullptr;
    b.counters = a.counters ? a.counters + (size_t)w * dmx::kFwdCounters : nullptr;
    b.tape = a.tape ? a.tape + (size_t)w * a.cap * a.rec : nullptr;
    b.forced = a.forced ? a.forced + (size_t)w * a.forced_cap * 2 : nullptr;
    b.forced_n = a.forced_n ? a.forced_n + w : nullptr;
    b.steplog = a.steplog ? a.steplog + (size_t)w * a.log_cap * 4 : nullptr;
    b.log_n = a.log_n ? a.log_n + w : nullptr;
    b.fail_state = a.fail_state ? a.fail_state + (size_t)w * (NX + P::NV) : nullptr;
    hipLaunchKernelGGL(dmx::fwd_kernel<P>, dim3(1), dim3(64), 0, s, (const typename P::Model*)model, b);
  }
}
template <class P>
void launch_adj(const void* model, const dmx::AdjArgs& a, hipStream_t s, int plain) {
  constexpr int NXS = P::NQ + P::NV + 3;
  const bool recompute = a.rec < NXS + 6 * P::NV;  // checkpoint-only tape
  auto kernel = recompute ? (a.hbar ? dmx::adj_kernel<P, true, true> : dmx::adj_kernel<P, true, false>)
                          : (a.hbar ? dmx::adj_kernel<P, false, true> : dmx::adj_kernel<P, false, false>);
  if (!plain) {
    const int blocks = grid_blocks<P>(kernel, a.W, a.g.queue != nullptr);
    if (a.g.queue) hipLaunchKernelGGL(dmx::reset_queue, dim3(1), dim3(64), 0, s, a.g.queue);
    hipLaunchKernelGGL(kernel, dim3(blocks), dim3(64), 0, s, (const typename P::Model*)model, a);
    return;
  }
  constexpr int NX = P::NQ + P::NV;
  const size_t nut = (size_t)a.n_int * a.nu;
  for (int w = 0; w < a.W; ++w) {
    dmx::AdjArgs b = a;
    b.W = 1;
    b.tape = a.tape + (size_t)w * a.cap * a.rec;
    b.n_acc = a.n_acc + w;
    b.status = a.status + w;
    b.u = a.u ? a.u + (size_t)w * nut : nullptr;
    b.xbar = a.xbar + (size_t)w * NX;
    b.x0bar = a.x0bar + (size_t)w * NX;
    b.ubar = a.ubar ? a.ubar + (size_t)w * nut : nullptr;
    b.counters = a.counters ? a.counters + (size_t)w * dmx::kAdjCounters : nullptr;
    b.hbar = a.hbar ? a.hbar + (size_t)w * a.npar : nullptr;
    hipLaunchKernelGGL(kernel, dim3(1), dim3(64), 0, s, (const typename P::Model*)model, b);
  }
}

// optimize-then-discretize adjoint: one launch, one team per world (the
// plain form launches world by world)
template <class P>
void launch_otd(const void* model, const dmx::AdjArgs& a, hipStream_t s, int plain) {
  auto kernel = a.hbar ? dmx::otd_kernel<P, true> : dmx::otd_kernel<P, false>;
  if (!plain) {
    const int blocks = grid_blocks<P>(kernel, a.W, a.g.queue != nullptr);
    if (a.g.queue) hipLaunchKernelGGL(dmx::reset_queue, dim3(1), dim3(64), 0, s, a.g.queue);
    hipLaunchKernelGGL(kernel, dim3(blocks), dim3(64), 0, s, (const typename P::Model*)model, a);
    return;
  }
  constexpr int NX = P::NQ + P::NV;
  const size_t nut = (size_t)a.n_int * a.nu;
  for (int w = 0; w < a.W; ++w) {
    dmx::AdjArgs b = a;
    b.W = 1;
    b.tape = a.tape + (size_t)w * a.cap * a.rec;
    b.n_acc = a.n_acc + w;
    b.status = a.status + w;
    b.u = a.u ? a.u + (size_t)w * nut : nullptr;
    b.xbar = a.xbar + (size_t)w * NX;
    b.x0bar = a.x0bar + (size_t)w * NX;
    b.ubar = a.ubar ? a.ubar + (size_t)w * nut : nullptr;
    b.counters = a.counters ? a.counters + (size_t)w * dmx::kAdjCounters : nullptr;
    b.hbar = a.hbar ? a.hbar + (size_t)w * a.npar : nullptr;
    hipLaunchKernelGGL(kernel, dim3(1), dim3(64), 0, s, (const typename P::Model*)model, b);
  }
}

using AccFn = void (*)(const void*, int, const double*, const double*, int, const dmx::SolverOpts&, double*, int*,
                       hipStream_t);

template <class P>
void launch_acc(const void* model, int n, const double* x, const double* tau, int cfd, const dmx::SolverOpts& o,
                double* acc, int* status, hipStream_t s) {
  const long long threads = (long long)n * P::TEAM;
  const int blocks = (int)((threads + 63) / 64);
  hipLaunchKernelGGL(dmx::accel_kernel<P>, dim3(blocks), dim3(64), 0, s, (const typename P::Model*)model, n, x, tau,
                     cfd, o.beta, o.newton_maxit, acc, status);
}

struct KernelEntry {
  int kind, nc, team, nv, nb;
  FwdFn fwd;
  AdjFn adj;
  AccFn acc;
  AdjFn otd;
  long long (*resident)();
};

#define FREE_ENTRY(NC, L) \
  {0, NC, L, 6, 1, &launch_fwd<dmx::FreePhys<NC, L>>, &launch_adj<dmx::FreePhys<NC, L>>, \
   &launch_acc<dmx::FreePhys<NC, L>>, &launch_otd<dmx::FreePhys<NC, L>>, &fwd_resident_teams<dmx::FreePhys<NC, L>>}
#define TREE_ENTRY(NV, NB, NC, L) \
  {1, NC, L, NV, NB, &launch_fwd<dmx::TreePhys<NV, NB, NC, L>>, &launch_adj<dmx::TreePhys<NV, NB, NC, L>>, \
   &launch_acc<dmx::TreePhys<NV, NB, NC, L>>, &launch_otd<dmx::TreePhys<NV, NB, NC, L>>, \
   &fwd_resident_teams<dmx::TreePhys<NV, NB, NC, L>>}


struct KernelTable {
  const KernelEntry* entries;
  int n;
};
// entry tables of the kernel translation units
KernelTable free_kernels_small();
KernelTable free_kernels();
KernelTable free_kernels_wide();
KernelTable tree_kernels();

}  // namespace dmx_host
