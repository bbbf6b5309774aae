// Host entry points of the cube-stack kernels (kern_stack.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "dmx_stack.hpp"

namespace dmx_host {
// worlds the device holds at once (one wavefront each)
long long stack_resident();
// forward rollouts / reverse sweep of a batch of stack worlds: one persistent
// launch (work queue when a.queue is set), or one launch per world (plain)
void stack_fwd(const dmx::StackArgs& a, hipStream_t s, int plain);
void stack_adj(const dmx::StackArgs& a, hipStream_t s, int plain);
// reverse sweep that also accumulates the model parameters' cotangents into
// a.pbar (kern_stack_params.hip)
void stack_adj_params(const dmx::StackArgs& a, hipStream_t s, int plain);
// forward rollout then reverse sweep of each world in one launch (a.xbar given)
void stack_grad(const dmx::StackArgs& a, hipStream_t s, int plain);
// accelerations at n independent states of one model
void stack_accel(const dmx::StackModel* model, int n, const double* x, const double* tau, int cfd,
                 const dmx::SolverOpts& o, double* acc, int* status, hipStream_t s);
}  // namespace dmx_host
