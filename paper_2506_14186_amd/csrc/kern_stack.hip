// Cube-stack kernels (forward, reverse, accelerations) and their launchers.
#include "dmx_stack_rk.hpp"
#include "dmx_stack_adj.hpp"
#include "dmx_stack_host.hpp"

namespace dmx_host {

long long stack_resident() {
  static long long r = [] {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0ll;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0ll;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, dmx::stack_fwd_kernel, 64, 0) != hipSuccess) return 0ll;
    return (long long)cus * per_cu;
  }();
  return r;
}

static int stack_grid(const dmx::StackArgs& a) {
  long long n = a.W;
  if (a.queue) {
    const long long r = stack_resident();
    if (r > 0 && r < n) n = r;
  }
  return (int)n;
}

void stack_fwd(const dmx::StackArgs& a, hipStream_t s, int plain) {
  if (!plain) {
    if (a.queue) hipLaunchKernelGGL(dmx::reset_queue, dim3(1), dim3(64), 0, s, a.queue);
    hipLaunchKernelGGL(dmx::stack_fwd_kernel, dim3(stack_grid(a)), dim3(64), 0, s, a);
    return;
  }
  for (int w = 0; w < a.W; ++w) {  // one world per launch, serialized on the stream
    dmx::StackArgs b = a;
    b.queue = nullptr;
    b.order = nullptr;
    b.w0 = w;
    b.W = w + 1;
    hipLaunchKernelGGL(dmx::stack_fwd_kernel, dim3(1), dim3(64), 0, s, b);
  }
}

void stack_adj(const dmx::StackArgs& a, hipStream_t s, int plain) {
  auto kernel = a.stages ? dmx::stack_adj_kernel<false> : dmx::stack_adj_kernel<true>;
  if (!plain) {
    if (a.queue) hipLaunchKernelGGL(dmx::reset_queue, dim3(1), dim3(64), 0, s, a.queue);
    hipLaunchKernelGGL(kernel, dim3(stack_grid(a)), dim3(64), 0, s, a);
    return;
  }
  for (int w = 0; w < a.W; ++w) {
    dmx::StackArgs b = a;
    b.queue = nullptr;
    b.order = nullptr;
    b.w0 = w;
    b.W = w + 1;
    hipLaunchKernelGGL(kernel, dim3(1), dim3(64), 0, s, b);
  }
}

void stack_accel(const dmx::StackModel* model, int n, const double* x, const double* tau, int cfd,
                 const dmx::SolverOpts& o, double* acc, int* status, hipStream_t s) {
  hipLaunchKernelGGL(dmx::stack_acc_kernel, dim3(n), dim3(64), 0, s, model, n, x, tau, cfd, o.beta, o.newton_maxit,
                     acc, status);
}

}  // namespace dmx_host
