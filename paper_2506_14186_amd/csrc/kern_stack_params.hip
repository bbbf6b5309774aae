// Reverse sweep of cube-stack rollouts with the model parameters' cotangents
// (kept apart from kern_stack.hip, whose kernels it leaves as they are).
#define DMX_STACK_KERNELS_ELSEWHERE
#include "dmx_stack_rk.hpp"
#include "dmx_stack_adj.hpp"
#include "dmx_stack_host.hpp"

namespace dmx_host {

template <typename K>
static long long resident_params(K kernel) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0ll;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0ll;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 64, 0) != hipSuccess) return 0ll;
  return (long long)cus * per_cu;
}

// the launch shapes of kern_stack.hip: a persistent launch over the work queue
// (or one world per workgroup), or one world per launch in the plain form
template <typename K>
static void launch_params(K kernel, long long resident, const dmx::StackArgs& a, hipStream_t s, int plain) {
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

void stack_adj_params(const dmx::StackArgs& a, hipStream_t s, int plain) {
  static const long long r0 = resident_params(dmx::stack_adj_kernel<false, true>);
  static const long long r1 = resident_params(dmx::stack_adj_kernel<true, true>);
  if (a.stages) launch_params(dmx::stack_adj_kernel<false, true>, r0, a, s, plain);
  else launch_params(dmx::stack_adj_kernel<true, true>, r1, a, s, plain);
}

}  // namespace dmx_host
