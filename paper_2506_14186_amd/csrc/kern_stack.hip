// Cube-stack kernels (forward, reverse, accelerations) and their launchers.
#include "dmx_stack_rk.hpp"
#include "dmx_stack_adj.hpp"
#include "dmx_stack_host.hpp"

namespace dmx_host {

template <typename K>
static long long resident_of(K kernel) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0ll;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0ll;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 64, 0) != hipSuccess) return 0ll;
  return (long long)cus * per_cu;
}

long long stack_resident() {
  static long long r = resident_of(dmx::stack_fwd_kernel);
  return r;
}

// a persistent launch fills the device (work queue) or takes one world per
// workgroup; the plain form launches one world at a time, serialized on the
// stream
template <typename K>
static void launch_worlds(K kernel, long long resident, const dmx::StackArgs& a, hipStream_t s, int plain) {
  if (!plain) {
    long long n = a.W;
    if (a.queue) {
      hipLaunchKernelGGL(dmx::reset_queue, dim3(1), dim3(64), 0, s, a.queue);
      if (resident > 0 && resident < n) n = resident;
    }
    hipLaunchKernelGGL(kernel, dim3((int)n), dim3(64), 0, s, a);
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

void stack_fwd(const dmx::StackArgs& a, hipStream_t s, int plain) {
  launch_worlds(dmx::stack_fwd_kernel, stack_resident(), a, s, plain);
}

void stack_adj(const dmx::StackArgs& a, hipStream_t s, int plain) {
  static const long long r0 = resident_of(dmx::stack_adj_kernel<false>);
  static const long long r1 = resident_of(dmx::stack_adj_kernel<true>);
  if (a.stages) launch_worlds(dmx::stack_adj_kernel<false>, r0, a, s, plain);
  else launch_worlds(dmx::stack_adj_kernel<true>, r1, a, s, plain);
}

void stack_grad(const dmx::StackArgs& a, hipStream_t s, int plain) {
  static const long long r0 = resident_of(dmx::stack_grad_kernel<false>);
  static const long long r1 = resident_of(dmx::stack_grad_kernel<true>);
  if (a.stages) launch_worlds(dmx::stack_grad_kernel<false>, r0, a, s, plain);
  else launch_worlds(dmx::stack_grad_kernel<true>, r1, a, s, plain);
}

void stack_accel(const dmx::StackModel* model, int n, const double* x, const double* tau, int cfd,
                 const dmx::SolverOpts& o, double* acc, int* status, hipStream_t s) {
  hipLaunchKernelGGL(dmx::stack_acc_kernel, dim3(n), dim3(64), 0, s, model, n, x, tau, cfd, o.beta, o.newton_maxit,
                     acc, status);
}

}  // namespace dmx_host
