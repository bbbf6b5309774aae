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
// Per-world cost of a batch: |p_T - target_w|^2 + cw_w * dt * sum |u|^2 over
// the world's own intervals, p_T the 3 coordinates of the world's final
// state (x_off[w], nx[w] doubles) from index pos[w] (the controlled body's
// position; npos <= 3 coordinates for models with fewer), and the
// final-state cotangent for the gradient; NaN cost for failed worlds.
__global__ void cost_kernel(const double* xout, const int* status, const double* u, int W, const long long* x_off,
                            const int* nx, const int* pos, int npos, int nu, const int* n_int_w, const long long* u_off,
                            const double* target, const double* cw, double dt, double* cost, double* xbar) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= W) return;
  const double* x = xout + x_off[w];
  double* xb = xbar + x_off[w];
  double c = 0.0;
  for (int i = 0; i < nx[w]; ++i) xb[i] = 0.0;
  const int p = pos[w];
  for (int i = 0; i < npos; ++i) {
    const double d = x[p + i] - target[3 * w + i];
    c += d * d;
    xb[p + i] = 2.0 * d;
  }
  double cu = 0.0;
  if (nu > 0) {
    const double* uw = u + u_off[w];
    const int n = n_int_w[w] * nu;
    for (int i = 0; i < n; ++i) cu += uw[i] * uw[i];
  }
  c += cw[w] * dt * cu;
  cost[w] = status[w] ? __longlong_as_double(0x7ff8000000000000ll) : c;
}

// u_bar += 2 cw_w dt u over each world's own intervals (one block per world)
__global__ void ctrl_grad_kernel(double* ubar, const double* u, int nu, const int* n_int_w, const long long* u_off,
                                 const double* cw, double dt) {
  const int w = blockIdx.x;
  const long long off = u_off[w], n = (long long)n_int_w[w] * nu;
  const double coef = 2.0 * cw[w] * dt;
  for (long long i = threadIdx.x; i < n; i += blockDim.x) ubar[off + i] += coef * u[off + i];
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
  size_t largest_free() const {
    size_t m = 0;
    for (const auto& kv : free_) m = kv.second > m ? kv.second : m;
    return m;
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
