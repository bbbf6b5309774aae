// Serving loop: request queue, budgeted device arena, concurrent streams.
// Included by dmx_lib.hip (uses its model/kernel tables).
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

namespace srv {

// ---------------------------------------------------------------- kernels
__global__ void broadcast_x0(double* x0s, const double* x0, int W, int nx) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < (long long)W * nx;
       i += (long long)gridDim.x * blockDim.x)
    x0s[i] = x0[i % nx];
}

// cost = |q_T[0:3] - target|^2 + cw * dt * sum |u|^2; cotangent of the final
// state for the gradient; NaN cost for failed worlds.
__global__ void cost_kernel(const double* xout, const int* status, const double* u, int W, int nx, int nq, int H,
                            int nu, double dt, double cw, double t0, double t1, double t2, double* cost,
                            double* xbar) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= W) return;
  const double tg[3] = {t0, t1, t2};
  const double* x = xout + (size_t)w * nx;
  double c = 0.0;
  for (int i = 0; i < nx; ++i) xbar[(size_t)w * nx + i] = 0.0;
  const int np = nq < 3 ? nq : 3;
  for (int i = 0; i < np; ++i) {
    const double d = x[i] - tg[i];
    c += d * d;
    xbar[(size_t)w * nx + i] = 2.0 * d;
  }
  double cu = 0.0;
  const double* uw = u + (size_t)w * H * nu;
  for (int i = 0; i < H * nu; ++i) cu += uw[i] * uw[i];
  c += cw * dt * cu;
  cost[w] = status[w] ? __longlong_as_double(0x7ff8000000000000ll) : c;
}

__global__ void ctrl_grad_kernel(double* ubar, const double* u, long long n, double coef) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    ubar[i] += coef * u[i];
}

// ---------------------------------------------------------------- arena
struct Arena {
  char* base = nullptr;
  size_t size = 0, used = 0;
  std::map<size_t, size_t> free_;  // offset -> length, coalesced

  bool alloc(size_t n, size_t* off) {
    n = (n + 255) & ~size_t(255);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        *off = it->first;
        const size_t rest = it->second - n, o = it->first;
        free_.erase(it);
        if (rest) free_[o + n] = rest;
        used += n;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t n) {
    n = (n + 255) & ~size_t(255);
    used -= n;
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) { it->second += nx->second; free_.erase(nx); }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) { pv->second += it->second; free_.erase(it); }
    }
  }
};

// pinned host buffers recycled by size class (hipHostFree is not called while serving)
struct PinnedPool {
  std::multimap<size_t, void*> free_;
  std::vector<void*> all;
  void* get(size_t n) {
    size_t cls = 4096;
    while (cls < n) cls *= 2;
    auto it = free_.find(cls);
    if (it != free_.end()) { void* p = it->second; free_.erase(it); return p; }
    void* p = nullptr;
    if (hipHostMalloc(&p, cls, hipHostMallocDefault) != hipSuccess) return nullptr;
    all.push_back(p);
    return p;
  }
  void put(void* p, size_t n) {
    size_t cls = 4096;
    while (cls < n) cls *= 2;
    free_.emplace(cls, p);
  }
  ~PinnedPool() { for (void* p : all) (void)hipHostFree(p); }
};

}  // namespace srv
