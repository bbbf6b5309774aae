// Adaptive Dormand-Prince 5(4) rollouts of cube-stack worlds (Sec. 3.1,
// App. C.2), one world per wavefront, with the state spread over the dof
// lanes (lane 2b: body b's position and linear velocity, lane 2b + 1: its
// quaternion and angular velocity).  Stage combinations, the (+) map and the
// tape writes are lane-local; the error norm is a wave sum.  Worlds of
// different sizes (cube counts) and horizons share one persistent launch
// through a device work queue (App. D, "Parallelizing DiffMJX simulations").
#pragma once
#include "dmx_stack.hpp"

namespace dmx {


DMX_DEV int stack_rec(int k, int stages) { return 3 + 13 * k + (stages ? 36 * k : 0); }

// indices of this dof lane's q entries (3 or 4) and v/acc entries (3)
DMX_DEV int q_index(const StackRole& ro, int j) { return 7 * ro.b + 3 * ro.half + j; }
DMX_DEV int v_index(const StackModel& m, const StackRole& ro, int j) { return 7 * m.k + 6 * ro.b + 3 * ro.half + j; }
DMX_DEV int a_index(const StackRole& ro, int j) { return 6 * ro.b + 3 * ro.half + j; }
DMX_DEV int nq_lane(const StackRole& ro) { return ro.half ? 4 : 3; }

DMX_DEV void load_state(const StackModel& m, const StackRole& ro, const double* x, double* yq, double* yv) {
  // lanes without a body hold an identity quaternion at rest (their stage
  // states stay finite; they write nothing)
#pragma unroll
  for (int j = 0; j < 4; ++j) yq[j] = (ro.half == 1 && j == 0) ? 1.0 : 0.0;
#pragma unroll
  for (int j = 0; j < 3; ++j) yv[j] = 0.0;
  if (!ro.dof) return;
  const int nq = nq_lane(ro);
#pragma unroll
  for (int j = 0; j < 4; ++j) if (j < nq) yq[j] = x[q_index(ro, j)];
#pragma unroll
  for (int j = 0; j < 3; ++j) yv[j] = x[v_index(m, ro, j)];
}
DMX_DEV void store_state(const StackModel& m, const StackRole& ro, double* x, const double* yq, const double* yv) {
  if (!ro.dof) return;
  const int nq = nq_lane(ro);
#pragma unroll
  for (int j = 0; j < 4; ++j) if (j < nq) x[q_index(ro, j)] = yq[j];
#pragma unroll
  for (int j = 0; j < 3; ++j) x[v_index(m, ro, j)] = yv[j];
}

// generalized forces of this lane's dofs in interval kk
DMX_DEV void stack_tau(const StackModel& m, const StackRole& ro, const double* uw, int kk, double* tau) {
#pragma unroll
  for (int j = 0; j < 3; ++j) tau[j] = 0.0;
  if (!ro.dof || !uw) return;
  for (int i = 0; i < m.nu; ++i) {
    const int d = m.ctrl[i] - 6 * ro.b - 3 * ro.half;
    if (d >= 0 && d < 3) {
      const double ui = uw[(size_t)kk * m.nu + i];
#pragma unroll
      for (int j = 0; j < 3; ++j) if (j == d) tau[j] += ui;
    }
  }
}

// (+) on this lane: position += dq, or quat <- normalize(quat exp(dq / 2))
DMX_DEV void stack_qplus(const StackRole& ro, const double* yq, const double* dq, double* Yq) {
  if (ro.half == 0) {
#pragma unroll
    for (int j = 0; j < 3; ++j) Yq[j] = yq[j] + dq[j];
    Yq[3] = 0.0;
  } else {
    const Q4 e = qexp_half(mk3(dq[0], dq[1], dq[2]), nullptr, nullptr, nullptr, nullptr);
    const Q4 r = qnormalize(qmul(mkq(yq[0], yq[1], yq[2], yq[3]), e), nullptr);
    Yq[0] = r.w; Yq[1] = r.x; Yq[2] = r.y; Yq[3] = r.z;
  }
}

// stage state i >= 1 of this lane from y and the stage accelerations A[l]
DMX_DEV void stack_stage(const StackRole& ro, const double* yq, const double* yv, const double (*A)[3], int i,
                         double h, double* Yq, double* Yv, double* dq) {
  const StageCoef k = stage_coef(i);
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    double sv = 0.0, sq = 0.0;
#pragma unroll
    for (int l = 0; l < 6; ++l) {
      const double a = l < i ? A[l][j] : 0.0;
      sv += k.a[l] * a;
      sq += k.a2[l] * a;
    }
    Yv[j] = yv[j] + h * sv;
    dq[j] = h * (k.c * yv[j] + h * sq);
  }
  stack_qplus(ro, yq, dq, Yq);
}

template <bool DUMMY = false>
DMX_DEV void stack_fwd_world(const StackModel& m, StackLds& S, const StackArgs& a, int w) {
  const StackRole ro = stack_role(m);
  const SolverOpts& o = a.o;
  const int n_int = a.n_int_w ? a.n_int_w[w] : a.n_int;
  const double* uw = (a.u && m.nu) ? a.u + st_uoff(a, w) : nullptr;
  const int rec = stack_rec(m.k, a.stages);
  double* tape_w = a.tape ? a.tape + st_toff(a, w) : nullptr;
  const long long cap = st_cap(a, w);
  const double* x0 = a.x0 + st_xoff(a, w);
  double yq[4], yv[3];
  load_state(m, ro, x0, yq, yv);
  StackStat st{};
  {
    bool fin = true;
#pragma unroll
    for (int j = 0; j < 4; ++j) fin = fin && isfinite(yq[j]);
#pragma unroll
    for (int j = 0; j < 3; ++j) fin = fin && isfinite(yv[j]);
    if (!wave_all(fin || !ro.dof)) st.status |= 4;
  }
  double A[7][3];
#pragma unroll
  for (int i = 0; i < 7; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) A[i][j] = 0.0;
  double t = 0.0, hprop = quantize_step(fmin(o.h0, a.dt), o.h_levels), eprev_pow = 1.0;
  long long attempts = 0;
  int nacc = 0, nrej = 0, fi = 0, nlog = 0;
  const int nforced = a.forced ? min(a.forced_n[w], a.forced_cap) : 0;
  const int NX = 13 * m.k;
  const int fatal_bits = ~kStOverflow;
  bool replay_done = false, have_prev = false;
  double tau[3];
  for (int kk = 0; kk < n_int && (st.status & fatal_bits) == 0 && !replay_done; ++kk) {
    stack_tau(m, ro, uw, kk, tau);
    const double tend = (double)(kk + 1) * a.dt;
    bool have_k1 = false;
    while (t < tend) {
      double h;
      bool landing;
      if (a.forced) {
        if (fi >= nforced) { replay_done = true; break; }
        h = a.forced[((size_t)w * a.forced_cap + fi) * 2 + 1];
        landing = t + h >= tend - 0.005 * h;
        ++fi;
      } else {
        landing = t + 1.01 * hprop >= tend;
        h = landing ? tend - t : hprop;
      }
      if (attempts >= o.max_attempts) { st.status |= 1; break; }
      ++attempts;
      if (ro.lane == 0) st.u_att++;
      double Yq[4], Yv[3], dq[3];
      const int status_before = st.status;
      bool fatal = false;
#pragma unroll 1
      for (int i = 0; i < 7; ++i) {
        if (i == 0 && have_k1) continue;
        if (i == 0) {
#pragma unroll
          for (int j = 0; j < 4; ++j) Yq[j] = yq[j];
#pragma unroll
          for (int j = 0; j < 3; ++j) Yv[j] = yv[j];
        } else {
          stack_stage(ro, yq, yv, A, i, h, Yq, Yv, dq);
        }
        double xw[3], ai[3];
        const int prev = i > 0 ? i - 1 : 0;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          double v = A[0][j];
#pragma unroll
          for (int l = 1; l < 6; ++l) v = (l == prev) ? A[l][j] : v;
          xw[j] = v;
        }
        const bool warm = i > 0 || have_prev;
        stack_acc(m, S, ro, Yq, Yv, tau, false, o.beta, o.newton_maxit, warm ? xw : nullptr, ai, st);
        have_prev = true;
#pragma unroll
        for (int l = 0; l < 7; ++l)
#pragma unroll
          for (int j = 0; j < 3; ++j) A[l][j] = (l == i) ? ai[j] : A[l][j];
        if (i == 0) {
          have_k1 = true;
          if (st.status & (12 | kStGraph)) { fatal = true; break; }
        }
        // a trial stage that the solver cannot take (non-neighbour contact)
        // fails like a failed solve: the attempt is rejected (below)
        if (st.status & kStGraph) break;
      }
      if (fatal) break;
      // error estimate: v: h sum e_i a_i; position: h^2 sum (e a)_i a_i;
      // quaternion: difference of the 5th- and 4th-order (+)-integrated values
      double acc2 = 0.0;
      if (ro.dof) {
        double ev[3], dqh[3], eq[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          double s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
          for (int l = 0; l < 7; ++l) { s1 += kTab.e[l] * A[l][j]; s2 += kTab.bhA[l] * A[l][j]; s3 += kTab.eA[l] * A[l][j]; }
          ev[j] = h * s1;
          dqh[j] = h * (kTab.bh_sum * yv[j] + h * s2);
          eq[j] = h * h * s3;
        }
        if (ro.half == 0) {
#pragma unroll
          for (int j = 0; j < 3; ++j) {
            const double r = eq[j] * rcp_nr(o.atol + o.rtol * fmax(fabs(yq[j]), fabs(Yq[j])));
            acc2 += r * r;
          }
        } else {
          double qh[4];
          stack_qplus(ro, yq, dqh, qh);
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const double r = (Yq[j] - qh[j]) * rcp_nr(o.atol + o.rtol * fmax(fabs(yq[j]), fabs(Yq[j])));
            acc2 += r * r;
          }
        }
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          const double r = ev[j] * rcp_nr(o.atol + o.rtol * fmax(fabs(yv[j]), fabs(Yv[j])));
          acc2 += r * r;
        }
      }
      double e2[1] = {acc2};
      wave_sum<1>(e2);
      double err = sqrt(e2[0] / NX);
      if ((st.status & (12 | kStGraph)) && !a.forced) {
        st.status = status_before;
        err = __longlong_as_double(0x7ff0000000000000ll);
      }
      const bool accept = a.forced ? true : (err <= 1.0);
      const double et = isfinite(err) ? fmax(err, o.err_floor) : 1e300;
      double fac = o.safety * pow(et, -(o.kP + o.kI) / o.err_order) * eprev_pow;
      fac = fmin(o.facmax, fmax(o.facmin, fac));
      if (a.steplog && nlog < a.log_cap && ro.lane == 0) {
        double* lg = a.steplog + ((size_t)w * a.log_cap + nlog) * 4;
        lg[0] = t; lg[1] = h; lg[2] = err; lg[3] = accept ? 1.0 : 0.0;
      }
      if (a.steplog) ++nlog;
      if (accept) {
        if (tape_w) {
          if (nacc >= cap) { st.status |= 32; break; }
          double* r = tape_w + (size_t)nacc * rec;
          if (ro.lane == 0) { r[0] = t; r[1] = h; r[2] = (double)kk; }
          store_state(m, ro, r + 3, yq, yv);
          if (a.stages && ro.dof) {
#pragma unroll
            for (int l = 0; l < 6; ++l)
#pragma unroll
              for (int j = 0; j < 3; ++j) r[3 + NX + 6 * m.k * l + a_index(ro, j)] = A[l][j];
          }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) yq[j] = Yq[j];
#pragma unroll
        for (int j = 0; j < 3; ++j) { yv[j] = Yv[j]; A[0][j] = A[6][j]; }
        t = landing ? tend : t + h;
        eprev_pow = pow(et, o.kP / o.err_order);
        hprop = quantize_step(fac * h, o.h_levels);
        ++nacc;
        bool fin = true;
#pragma unroll
        for (int j = 0; j < 4; ++j) fin = fin && isfinite(yq[j]);
#pragma unroll
        for (int j = 0; j < 3; ++j) fin = fin && isfinite(yv[j]);
        if (!wave_all(fin || !ro.dof)) { st.status |= 4; break; }
      } else {
        hprop = quantize_step(fmin(1.0, fac) * h, o.h_levels);
        ++nrej;
      }
      if (!a.forced && hprop < 1e-12 * fmax(1.0, fabs(t))) { st.status |= 2; break; }
      if (st.status & (12 | kStGraph)) break;
    }
  }
  store_state(m, ro, a.xout + st_xoff(a, w), yq, yv);
  if (a.counters) {
    double c[kFwdCounters] = {(double)st.u_att, (double)st.u_rhs, (double)st.u_con, (double)st.u_nit,
                              (double)st.u_ncon, (double)st.u_nedge, (double)st.u_ls, (double)st.u_con2,
                              (double)st.u_ncon2};
    wave_sum<kFwdCounters>(c);
    if (ro.lane == 0)
      for (int i = 0; i < kFwdCounters; ++i) a.counters[(size_t)w * kFwdCounters + i] = (long long)c[i];
  }
  if (ro.lane == 0) {
    a.status[w] = st.status;
    if (a.n_acc) a.n_acc[w] = nacc;
    if (a.n_rej) a.n_rej[w] = nrej;
    if (a.log_n) a.log_n[w] = nlog;
  }
}

DMX_DEV int stack_take(const StackArgs& a, int* next_static, bool first) {
  int idx;
  if (a.queue) {
    int v = 0;
    if ((threadIdx.x & 63) == 0) v = atomicAdd(a.queue, 1);
    idx = __shfl(v, 0, 64);
  } else {
    idx = first ? a.w0 + (int)blockIdx.x : a.W;
  }
  (void)next_static;
  if (idx >= a.W) return -1;
  return a.order ? a.order[idx] : idx;
}

// The two plain (non-template) kernels below are defined in one translation
// unit only (kern_stack.hip); other units that use these headers define
// DMX_STACK_KERNELS_ELSEWHERE.
#ifndef DMX_STACK_KERNELS_ELSEWHERE
__global__ void __launch_bounds__(64) stack_fwd_kernel(StackArgs a) {
  __shared__ StackLds S;
  for (bool first = true;; first = false) {
    const int w = stack_take(a, nullptr, first);
    if (w < 0) break;
    const StackModel& m = st_model(a, w);
    stack_fwd_world(m, S, a, w);
  }
}

// Accelerations at independent states of one model (one wavefront each).
__global__ void __launch_bounds__(64) stack_acc_kernel(const StackModel* __restrict__ model, int n,
                                                       const double* x, const double* tau_in, int cfd, double beta,
                                                       int maxit, double* acc_out, int* status) {
  __shared__ StackLds S;
  const int w = blockIdx.x;
  if (w >= n) return;
  const StackModel& m = *model;
  const StackRole ro = stack_role(m);
  const int NX = 13 * m.k, NV = 6 * m.k;
  double yq[4], yv[3], tau[3] = {0.0, 0.0, 0.0}, acc[3];
  load_state(m, ro, x + (size_t)w * NX, yq, yv);
  if (tau_in && ro.dof) {
#pragma unroll
    for (int j = 0; j < 3; ++j) tau[j] = tau_in[(size_t)w * NV + a_index(ro, j)];
  }
  StackStat st{};
  stack_acc(m, S, ro, yq, yv, tau, cfd != 0, beta, maxit, nullptr, acc, st);
  if (ro.dof) {
#pragma unroll
    for (int j = 0; j < 3; ++j) acc_out[(size_t)w * NV + a_index(ro, j)] = acc[j];
  }
  if (ro.lane == 0) status[w] = st.status;
}
#endif  // DMX_STACK_KERNELS_ELSEWHERE

}  // namespace dmx
