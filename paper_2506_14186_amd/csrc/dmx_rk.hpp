// Adaptive Dormand-Prince 5(4) rollouts and their discrete adjoint, one team
// of lanes per world, for any physics policy P providing:
//   NQ, NV, TEAM, Model, acc(), acc_vjp(), qplus(), qplus_vjp(), q_is_linear().
//
// Forward (Sec. 3.1, App. C.2): stage states Y_i = (q_n (+) h sum_j a_ij v_j,
// v_n + h sum_j a_ij a_j) with v_j the velocity part of Y_j; FSAL; an
// embedded error estimate, accept iff err <= 1, PI step-size control with the
// controller coefficients of App. E.1.  Every accepted step is written to the
// tape with its stage accelerations, so the reverse sweep rebuilds each stage
// state bit for bit without re-solving the contact problem.
//
// Reverse (discretize-then-optimize, App. C.2): step sizes and the accepted
// sequence are constants; each step is differentiated through its stage
// combinations, the (+) map and the acceleration map (acc_vjp).
#pragma once
#include "dmx_common.hpp"

namespace dmx {

// ------------------------------------------------------------ tableau
struct Tableau {
  double a[7][7];   // a[i][j], stage i uses stages j < i; row 6 = b (FSAL)
  double a2[7][7];  // (a a)[i][l] = sum_j a[i][j] a[j][l]
  double c[7];
  double e[7];      // b - bh
  double bhA[7];    // sum_j bh[j] a[j][l]
  double eA[7];     // sum_j e[j] a[j][l]
  double bh_sum;
};

// the derived coefficients of a pair from its A (row 6 = b, FSAL) and b-hat
constexpr Tableau tableau_from(const double (&A)[7][7], const double (&BH)[7]) {
  Tableau t{};
  for (int i = 0; i < 7; ++i) {
    double s = 0.0;
    for (int j = 0; j < 7; ++j) { t.a[i][j] = A[i][j]; s += A[i][j]; }
    t.c[i] = s;
  }
  for (int i = 0; i < 7; ++i)
    for (int l = 0; l < 7; ++l) {
      double s = 0.0;
      for (int j = 0; j < 7; ++j) s += A[i][j] * A[j][l];
      t.a2[i][l] = s;
    }
  t.bh_sum = 0.0;
  for (int j = 0; j < 7; ++j) { t.e[j] = (j < 6 ? A[6][j] : 0.0) - BH[j]; t.bh_sum += BH[j]; }
  for (int l = 0; l < 7; ++l) {
    double s1 = 0.0, s2 = 0.0;
    for (int j = 0; j < 7; ++j) { s1 += BH[j] * A[j][l]; s2 += t.e[j] * A[j][l]; }
    t.bhA[l] = s1; t.eA[l] = s2;
  }
  return t;
}

// Dormand-Prince 5(4)
constexpr Tableau make_tableau() {
  const double A[7][7] = {
      {0, 0, 0, 0, 0, 0, 0},
      {1.0 / 5.0, 0, 0, 0, 0, 0, 0},
      {3.0 / 40.0, 9.0 / 40.0, 0, 0, 0, 0, 0},
      {44.0 / 45.0, -56.0 / 15.0, 32.0 / 9.0, 0, 0, 0, 0},
      {19372.0 / 6561.0, -25360.0 / 2187.0, 64448.0 / 6561.0, -212.0 / 729.0, 0, 0, 0},
      {9017.0 / 3168.0, -355.0 / 33.0, 46732.0 / 5247.0, 49.0 / 176.0, -5103.0 / 18656.0, 0, 0},
      {35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0, -2187.0 / 6784.0, 11.0 / 84.0, 0}};
  const double BH[7] = {5179.0 / 57600.0, 0.0, 7571.0 / 16695.0, 393.0 / 640.0, -92097.0 / 339200.0,
                        187.0 / 2100.0, 1.0 / 40.0};
  return tableau_from(A, BH);
}

// Tsitouras 5(4) (Tsit5, the solver of the paper's experiments, App. E.1):
// the FSAL pair of Tsitouras (2011); b-hat = b - btilde, btilde the published
// error weights
constexpr Tableau make_tableau_tsit5() {
  const double A[7][7] = {
      {0, 0, 0, 0, 0, 0, 0},
      {0.161, 0, 0, 0, 0, 0, 0},
      {-0.008480655492356989, 0.335480655492357, 0, 0, 0, 0, 0},
      {2.897153057105493, -6.359448489975075, 4.3622954328695815, 0, 0, 0, 0},
      {5.325864828439257, -11.748883564062828, 7.4955393428898365, -0.09249506636175525, 0, 0, 0},
      {5.86145544294642, -12.92096931784711, 8.159367898576159, -0.071584973281401, -0.028269050394068383, 0, 0},
      {0.09646076681806523, 0.01, 0.4798896504144996, 1.379008574103742, -3.290069515436081, 2.324710524099774, 0}};
  const double BT[7] = {-0.00178001105222577714, -0.0008164344596567469, 0.007880878010261995,
                        -0.1447110071732629, 0.5823571654525552, -0.45808210592918697, 0.015151515151515152};
  double BH[7] = {};
  for (int j = 0; j < 7; ++j) BH[j] = (j < 6 ? A[6][j] : 0.0) - BT[j];
  return tableau_from(A, BH);
}
// compile-time tableau: stage-specialized code reads it with constant
// indices, so every coefficient is an immediate operand
constexpr Tableau kTab = make_tableau();
constexpr Tableau kTab5 = make_tableau_tsit5();

struct SolverOpts {
  double rtol, atol, h0, safety, facmin, facmax, kP, kI, err_order, err_floor, beta;
  long long max_attempts;
  int newton_maxit, cfd, h_levels;
  int tableau;  // 0: Dormand-Prince 5(4), 1: Tsitouras 5(4)
};

// Proposed steps rounded down to h_levels mantissa values per octave (exact
// binary arithmetic), so that step sequences are insensitive to rounding-level
// differences of the error estimate.
DMX_DEV double quantize_step(double h, int levels) {
  if (levels <= 0 || !(h > 0.0) || !isfinite(h)) return h;
  int e;
  const double m = frexp(h, &e);
  const double k = floor(m * (2.0 * levels));
  return ldexp(k / (2.0 * levels), e);
}

// attempts, rhs, contacts, newton its, newton contacts, edges, line search,
// then contacts and newton contacts between two bodies (stacks)
constexpr int kFwdCounters = 9;
constexpr int kAdjCounters = 4;  // steps, vjps, vjp contacts, vjp edges

// Per-world layout of a batch and its work distribution.  Null arrays mean
// the uniform layout: n_int intervals per world, controls u[w][n_int][nu],
// tape records [w][cap], worlds processed once each in index order.
struct Ragged {
  const int* n_int_w;         // [W] intervals of world w
  const long long* u_off;     // [W] first element of world w's controls in u (and u_bar)
  const long long* tape_off;  // [W] first tape record of world w
  const int* cap_w;           // [W] tape records available to world w
  const int* order;           // [W] processing order (longest first)
  int* queue;                 // work counter, zero at launch (null: one world per team)
};

DMX_DEV int world_intervals(const Ragged& g, int n_int, int w) { return g.n_int_w ? g.n_int_w[w] : n_int; }
DMX_DEV size_t world_u(const Ragged& g, int n_int, int nu, int w) {
  return g.u_off ? (size_t)g.u_off[w] : (size_t)w * n_int * nu;
}
DMX_DEV size_t world_tape(const Ragged& g, long long cap, int w) {
  return g.tape_off ? (size_t)g.tape_off[w] : (size_t)w * cap;
}
DMX_DEV long long world_cap(const Ragged& g, long long cap, int w) { return g.cap_w ? g.cap_w[w] : cap; }

// Next world of a team: without a queue the team's own index once; with a
// queue its leader lane takes the next position from the shared counter and
// broadcasts it.  Every team leaves once the counter has passed W.
template <int L>
DMX_DEV int take_world(const Ragged& g, int W, int team, bool first) {
  int idx;
  if (g.queue) {
    int v = 0;
    if ((threadIdx.x & (L - 1)) == 0) v = atomicAdd(g.queue, 1);
    idx = __shfl(v, (int)(threadIdx.x & 63) & ~(L - 1), 64);
  } else {
    idx = first ? team : W;
  }
  if (idx >= W) return -1;
  return g.order ? g.order[idx] : idx;
}

static __global__ void reset_queue(int* q) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *q = 0;
}

struct FwdArgs {
  int W, n_int, nu;
  double dt;
  long long* counters;  // [W][kFwdCounters] or null
  const double* x0;
  const double* u;
  double* xout;
  int* status;
  int* n_acc;
  int* n_rej;
  long long* n_newton;
  double* tape;
  long long cap;
  int rec;
  const double* forced;
  const int* forced_n;
  int forced_cap;
  double* steplog;
  int* log_n;
  int log_cap;
  double* fail_state;
  Ragged g;
  SolverOpts o;
};

struct AdjArgs {
  int W, n_int, nu;
  double dt;            // control interval length (the optimize-then-discretize adjoint's grid)
  double* hbar;         // [W][npar] model-parameter cotangents (the first npar of kParams), or null
  int npar;             // 3 (box half sizes) or kParams
  long long* counters;  // [W][kAdjCounters] or null
  const double* tape;
  long long cap;
  int rec;
  const int* n_acc;
  const int* status;
  const double* u;
  const double* xbar;
  double* x0bar;
  double* ubar;
  Ragged g;
  SolverOpts o;
};

// generalized force of interval k: tau[ctrl[i]] += u[w][k][i] (unrolled over
// dofs so that tau stays in registers)
template <class P>
DMX_DEV void load_tau(const typename P::Model& m, const double* uw, int k, int nu, double* tau) {
#pragma unroll
  for (int d = 0; d < P::NV; ++d) tau[d] = 0.0;
  for (int i = 0; i < nu; ++i) {
    const double ui = uw[(size_t)k * nu + i];
    const int c = m.ctrl[i];
#pragma unroll
    for (int d = 0; d < P::NV; ++d)
      if (c == d) tau[d] += ui;
  }
}

template <class P>
DMX_DEV void store_ubar(const typename P::Model& m, const double* tb, double* dst, int nu) {
  for (int i = 0; i < nu; ++i) {
    const int c = m.ctrl[i];
    double g = 0.0;
#pragma unroll
    for (int d = 0; d < P::NV; ++d)
      if (c == d) g = tb[d];
    dst[i] = g;
  }
}

// dst[i] = src[i] for a team-replicated array: every lane of the team stores
// every element (the lanes hold bitwise-equal values, and one store
// instruction writes each address once), so no per-element lane selection
template <int N, int L>
DMX_DEV void team_store(double* dst, const double* src, int tl) {
  (void)tl;
#pragma unroll
  for (int i = 0; i < N; ++i) dst[i] = src[i];
}

// Coefficients of stage i (a[i][l], (A A)[i][l], c[i]), selected by a
// switch on the (uniform) stage index so that they are immediate operands.
struct StageCoef {
  double a[6], a2[6], c;
};
template <int I, int T>
DMX_DEV StageCoef stage_coef_c() {
  constexpr const Tableau& tb = T ? kTab5 : kTab;
  StageCoef k;
#pragma unroll
  for (int l = 0; l < 6; ++l) { k.a[l] = tb.a[I][l]; k.a2[l] = tb.a2[I][l]; }
  k.c = tb.c[I];
  return k;
}
template <int T>
DMX_DEV StageCoef stage_coef_t(int i) {
  switch (i) {
    case 1: return stage_coef_c<1, T>();
    case 2: return stage_coef_c<2, T>();
    case 3: return stage_coef_c<3, T>();
    case 4: return stage_coef_c<4, T>();
    case 5: return stage_coef_c<5, T>();
    default: return stage_coef_c<6, T>();
  }
}
// tab: 0 Dormand-Prince, 1 Tsitouras (uniform across the wavefront)
DMX_DEV StageCoef stage_coef(int i, int tab = 0) { return tab ? stage_coef_t<1>(i) : stage_coef_t<0>(i); }

// Teams of at least four lanes split per-component work of the tableau
// combinations over their lanes (component d on lane d mod L) and share the
// results through LDS; smaller teams compute every component on each lane.
template <class P>
constexpr bool kSplitDofs = P::TEAM >= 4;

// sums over the earlier stages for component d: sv = sum a[i][l] A[l][d],
// sq = sum (A A)[i][l] A[l][d]; entries of later stages (stale, possibly
// non-finite after a failed trial) are masked, not branched over; the six LDS
// reads are issued together
template <class P>
DMX_DEV void stage_sums(const double (*A)[P::NV], int i, const StageCoef& k, int d, double* sv_out, double* sq_out) {
  double av[6];
#pragma unroll
  for (int l = 0; l < 6; ++l) av[l] = A[l][d];
  double sv = 0.0, sq = 0.0;
#pragma unroll
  for (int l = 0; l < 6; ++l) {
    const double x = l < i ? av[l] : 0.0;
    sv += k.a[l] * x;
    sq += k.a2[l] * x;
  }
  *sv_out = sv;
  *sq_out = sq;
}

// stage state Y_i from y_n and the stage accelerations A[0..i-1] (i >= 1);
// with keep, the (+) map's exponential coefficients for its VJP
template <class P>
DMX_DEV void stage_state(const double* y, const double (*A)[P::NV], int i, double h, double* Y, double* dq,
                         typename P::QPlusKeep* keep = nullptr, int tab = 0) {
  constexpr int NQ = P::NQ, NV = P::NV, L = P::TEAM;
  const StageCoef k = stage_coef(i, tab);
  double sv[NV], sq[NV];
  if constexpr (kSplitDofs<P>) {
    double* buf = lds_dof_area<L, 3 * NV>();
    const int tl = threadIdx.x & (L - 1);
#pragma unroll
    for (int r = 0; r < (NV + L - 1) / L; ++r) {
      const int d = tl + r * L;
      if (d < NV) stage_sums<P>(A, i, k, d, &buf[d], &buf[NV + d]);
    }
    wave_fence();
#pragma unroll
    for (int d = 0; d < NV; ++d) { sv[d] = buf[d]; sq[d] = buf[NV + d]; }
    wave_fence();
  } else {
#pragma unroll
    for (int d = 0; d < NV; ++d) stage_sums<P>(A, i, k, d, &sv[d], &sq[d]);
  }
#pragma unroll
  for (int d = 0; d < NV; ++d) {
    Y[NQ + d] = y[NQ + d] + h * sv[d];
    dq[d] = h * (k.c * y[NQ + d] + h * sq[d]);
  }
  if (keep) P::qplus_keep(y, dq, Y, keep);
  else P::qplus(y, dq, Y);
}

// cotangents of stage i's combination: v_bar from its velocity part and the
// (+) increment's velocity term, A_bar[l] for the earlier stages
template <class P>
DMX_DEV void stage_distribute(int i, const double* Ybar, const double* dqb, double h, double* vb, double (*Ab)[P::NV],
                              int tab = 0) {
  constexpr int NQ = P::NQ, NV = P::NV, L = P::TEAM;
  const StageCoef k = stage_coef(i, tab);
#pragma unroll
  for (int d = 0; d < NV; ++d) vb[d] += Ybar[NQ + d] + h * k.c * dqb[d];
  // a[i][l] = (A A)[i][l] = 0 for l >= i (explicit tableau): every entry is
  // updated, without branches (the cotangents are finite); component d's
  // column is updated by lane d mod L (by every lane for small teams)
  auto column = [&](int d, double ybd, double qbd) {
    double ab[6];
#pragma unroll
    for (int l = 0; l < 6; ++l) ab[l] = Ab[l][d];
#pragma unroll
    for (int l = 0; l < 6; ++l) Ab[l][d] = ab[l] + (h * k.a[l] * ybd + h * h * k.a2[l] * qbd);
  };
  if constexpr (kSplitDofs<P>) {
    const int tl = threadIdx.x & (L - 1);
#pragma unroll
    for (int r = 0; r < (NV + L - 1) / L; ++r) {
      const int d = tl + r * L;
      if (d < NV) column(d, pick<NV>(Ybar + NQ, d), pick<NV>(dqb, d));
    }
    wave_fence();
  } else {
#pragma unroll
    for (int d = 0; d < NV; ++d) column(d, Ybar[NQ + d], dqb[d]);
  }
}

template <class P>
DMX_DEV void capture_failure(double* dst, int w, const double* Y, const double* tau, int tl) {
  constexpr int NX = P::NQ + P::NV, L = P::TEAM;
  double* d = dst + (size_t)w * (NX + P::NV);
  team_store<NX, L>(d, Y, tl);
  team_store<P::NV, L>(d + NX, tau, tl);
}

// Accelerations at independent states (one team per state).
template <class P>
__global__ void __launch_bounds__(64) accel_kernel(const typename P::Model* __restrict__ model, int n,
                                                   const double* x, const double* tau_in, int cfd, double beta,
                                                   int maxit, double* acc_out, int* status) {
  constexpr int L = P::TEAM, NQ = P::NQ, NV = P::NV, NX = NQ + NV;
  const int gt = blockIdx.x * blockDim.x + threadIdx.x;
  const int w = gt / L;
  const int tl = gt & (L - 1);
  stage_pairs(*model);
  if (w >= n) return;
  double y[NX], tau[NV], acc[NV];
#pragma unroll
  for (int i = 0; i < NX; ++i) y[i] = x[(size_t)w * NX + i];
#pragma unroll
  for (int i = 0; i < NV; ++i) tau[i] = tau_in ? tau_in[(size_t)w * NV + i] : 0.0;
  Stat st{};
  P::acc(*model, y, tau, cfd != 0, beta, maxit, nullptr, acc, st);
  team_store<NV, L>(acc_out + (size_t)w * NV, acc, tl);
  if (tl == 0) status[w] = st.status;
}

// One world's forward rollout by its team; A: the team's stage accelerations
// in LDS (every team lane writes the same replicated values).
template <class P>
DMX_DEV void fwd_world(const typename P::Model& m, const FwdArgs& a, int w, int tl, double (*A)[P::NV]) {
  constexpr int L = P::TEAM, NQ = P::NQ, NV = P::NV, NX = NQ + NV;
  const SolverOpts& o = a.o;
  const int n_int = world_intervals(a.g, a.n_int, w);
  const double* uw = a.u ? a.u + world_u(a.g, a.n_int, a.nu, w) : nullptr;
  double* tape_w = a.tape ? a.tape + world_tape(a.g, a.cap, w) * a.rec : nullptr;
  const long long cap = world_cap(a.g, a.cap, w);
  double y[NX];
#pragma unroll
  for (int i = 0; i < NX; ++i) y[i] = a.x0[(size_t)w * NX + i];
  double tau[NV];
  Stat st{};
  double t = 0.0, hprop = quantize_step(fmin(o.h0, a.dt), o.h_levels), eprev = 1.0;
  // eprev^(kP / order), updated with eprev (one pow per accepted step)
  double eprev_pow = 1.0;
  long long attempts = 0;
  int nacc = 0, nrej = 0, fi = 0, nlog = 0;
  const int nforced = a.forced ? min(a.forced_n[w], a.forced_cap) : 0;
#pragma unroll
  for (int i = 0; i < NX; ++i)
    if (!isfinite(y[i])) st.status |= 4;
  bool replay_done = false, have_prev = false;
  for (int kk = 0; kk < n_int && st.status == 0 && !replay_done; ++kk) {
    load_tau<P>(m, uw, kk, a.nu, tau);
    const double tend = (double)(kk + 1) * a.dt;
    bool have_k1 = false;
    while (t < tend) {
      double h;
      bool landing;
      if (a.forced) {
        if (fi >= nforced) { replay_done = true; break; }  // replay ends with its list
        h = a.forced[((size_t)w * a.forced_cap + fi) * 2 + 1];
        landing = t + h >= tend - 0.005 * h;
        ++fi;
      } else {
        landing = t + 1.01 * hprop >= tend;
        h = landing ? tend - t : hprop;
      }
      if (attempts >= o.max_attempts) { st.status |= 1; break; }
      ++attempts;
      if (tl == 0) st.u_att++;
      // stages: 0 (only after an accepted step's interval end or at the
      // start, FSAL otherwise) and 1..6; one call site of the acceleration
      // map.  The stage index runs from 0 for every team, so that it is
      // uniform across the wavefront (tableau reads stay scalar).
      double Y[NX], dq[NV];
      const int status_before = st.status;
      bool fatal = false;
#pragma unroll 1
      for (int i = 0; i < 7; ++i) {
        if (i == 0 && have_k1) continue;
        if (i == 0) {
#pragma unroll
          for (int j = 0; j < NX; ++j) Y[j] = y[j];
        } else {
          stage_state<P>(y, A, i, h, Y, dq, nullptr, o.tableau);
        }
        double ai[NV];
        const int before = st.status;
        // warm start from the previous stage (stage 0: the last accepted
        // step's final stage, at the same state)
        const double* xw = i > 0 ? A[i - 1] : (have_prev ? A[0] : nullptr);
        P::acc(m, Y, tau, false, o.beta, o.newton_maxit, xw, ai, st);
        have_prev = true;
        if ((st.status & 12) && !(before & 12) && a.fail_state) capture_failure<P>(a.fail_state, w, Y, tau, tl);
#pragma unroll
        for (int d = 0; d < NV; ++d) A[i][d] = ai[d];
        if (i == 0) {
          have_k1 = true;
          if (st.status & 12) { fatal = true; break; }  // a failed solve at an accepted state ends the world
        }
      }
      if (fatal) break;
      // Y holds y_new (stage 7).  Error estimate in the ambient coordinates:
      // v: h sum e_i a_i; linear q: h sum e_i v_i; quaternions: difference of
      // the 5th- and 4th-order (+)-integrated values.
      double err = 0.0;
      {
        double dqh[NV], ev[NV], eq[NV], s1[NV], s2[NV], s3[NV];
        const bool t5 = o.tableau != 0;
        auto comb = [&](int d, double* s1d, double* s2d, double* s3d) {
          double a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll
          for (int l = 0; l < 7; ++l) {
            const double ce = t5 ? kTab5.e[l] : kTab.e[l], cb = t5 ? kTab5.bhA[l] : kTab.bhA[l];
            const double cea = t5 ? kTab5.eA[l] : kTab.eA[l];
            a1 += ce * A[l][d]; a2 += cb * A[l][d]; a3 += cea * A[l][d];
          }
          *s1d = a1; *s2d = a2; *s3d = a3;
        };
        if constexpr (kSplitDofs<P>) {  // component d on lane d mod L, shared through LDS
          double* buf = lds_dof_area<L, 3 * NV>();
#pragma unroll
          for (int r = 0; r < (NV + L - 1) / L; ++r) {
            const int d = tl + r * L;
            if (d < NV) comb(d, &buf[d], &buf[NV + d], &buf[2 * NV + d]);
          }
          wave_fence();
#pragma unroll
          for (int d = 0; d < NV; ++d) { s1[d] = buf[d]; s2[d] = buf[NV + d]; s3[d] = buf[2 * NV + d]; }
          wave_fence();
        } else {
#pragma unroll
          for (int d = 0; d < NV; ++d) comb(d, &s1[d], &s2[d], &s3[d]);
        }
#pragma unroll
        for (int d = 0; d < NV; ++d) {
          ev[d] = h * s1[d];
          dqh[d] = h * ((t5 ? kTab5.bh_sum : kTab.bh_sum) * y[NQ + d] + h * s2[d]);
          eq[d] = h * h * s3[d];
        }
        double qh[NQ];
        P::qplus(y, dqh, qh);
        double acc2 = 0.0;
#pragma unroll
        for (int i = 0; i < NQ; ++i) {
          double e = P::q_is_linear(i) ? eq[P::q_dof(i)] : Y[i] - qh[i];
          const double r = e * rcp_nr(o.atol + o.rtol * fmax(fabs(y[i]), fabs(Y[i])));
          acc2 += r * r;
        }
#pragma unroll
        for (int d = 0; d < NV; ++d) {
          const double r = ev[d] * rcp_nr(o.atol + o.rtol * fmax(fabs(y[NQ + d]), fabs(Y[NQ + d])));
          acc2 += r * r;
        }
        err = sqrt(acc2 / NX);
      }
      // a contact solve that failed at a trial stage rejects the attempt
      // (the step shrinks); only a failure at an accepted state is fatal
      if ((st.status & 12) && !a.forced) {
        st.status = status_before;
        err = __longlong_as_double(0x7ff0000000000000ll);
      }
      const bool accept = a.forced ? true : (err <= 1.0);
      const double et = isfinite(err) ? fmax(err, o.err_floor) : 1e300;
      double fac = o.safety * pow(et, -(o.kP + o.kI) / o.err_order) * eprev_pow;
      fac = fmin(o.facmax, fmax(o.facmin, fac));
      if (a.steplog && nlog < a.log_cap && tl == 0) {
        double* lg = a.steplog + ((size_t)w * a.log_cap + nlog) * 4;
        lg[0] = t; lg[1] = h; lg[2] = err; lg[3] = accept ? 1.0 : 0.0;
      }
      if (a.steplog) ++nlog;
      if (accept) {
        if (tape_w) {
          if (nacc >= cap) { st.status |= 32; break; }
          double* rec = tape_w + (size_t)nacc * a.rec;
          if (tl == 0) { rec[0] = t; rec[1] = h; rec[2] = (double)kk; }
          team_store<NX, L>(rec + 3, y, tl);
          if (a.rec >= 3 + NX + 6 * NV) {  // stage accelerations (else a checkpoint-only tape)
            // from LDS, entry j by lane j mod L
            const double* Af = &A[0][0];
#pragma unroll
            for (int r = 0; r < (6 * NV + L - 1) / L; ++r) {
              const int j = tl + r * L;
              if (j < 6 * NV) rec[3 + NX + j] = Af[j];
            }
          }
        }
#pragma unroll
        for (int i = 0; i < NX; ++i) y[i] = Y[i];
#pragma unroll
        for (int d = 0; d < NV; ++d) A[0][d] = A[6][d];
        t = landing ? tend : t + h;
        eprev = et;
        eprev_pow = pow(et, o.kP / o.err_order);
        hprop = quantize_step(fac * h, o.h_levels);
        ++nacc;
        bool fin = true;
#pragma unroll
        for (int i = 0; i < NX; ++i) fin = fin && isfinite(y[i]);
        if (!fin) { st.status |= 4; break; }
      } else {
        hprop = quantize_step(fmin(1.0, fac) * h, o.h_levels);
        ++nrej;
      }
      if (!a.forced && hprop < 1e-12 * fmax(1.0, fabs(t))) { st.status |= 2; break; }
      if (st.status & 12) break;
    }
  }
  team_store<NX, L>(a.xout + (size_t)w * NX, y, tl);
  if (a.counters) {
    double c[kFwdCounters] = {(double)st.u_att, (double)st.u_rhs, (double)st.u_con, (double)st.u_nit,
                              (double)st.u_ncon, (double)st.u_nedge, (double)st.u_ls, 0.0, 0.0};
    team_sum_arr<L, kFwdCounters>(c);
    if (tl == 0)
      for (int i = 0; i < kFwdCounters; ++i) a.counters[(size_t)w * kFwdCounters + i] = (long long)c[i];
  }
  if (tl == 0) {
    a.status[w] = st.status;
    if (a.n_acc) a.n_acc[w] = nacc;
    if (a.n_rej) a.n_rej[w] = nrej;
    if (a.n_newton) a.n_newton[w] = st.newton_it;
    if (a.log_n) a.log_n[w] = nlog;
  }
}

template <class P>
__global__ void __launch_bounds__(64) fwd_kernel(const typename P::Model* __restrict__ model, FwdArgs a) {
  constexpr int L = P::TEAM, NV = P::NV;
  const int gt = blockIdx.x * blockDim.x + threadIdx.x;
  const int team = gt / L, tl = gt & (L - 1);
  __shared__ double sA[64 / L][7][NV];
  double (*A)[NV] = sA[(threadIdx.x & 63) / L];
  stage_pairs(*model);
  for (bool first = true;; first = false) {
    const int w = take_world<L>(a.g, a.W, team, first);
    if (w < 0) break;
    fwd_world<P>(*model, a, w, tl, A);
  }
}

// RECOMPUTE: the tape holds only the accepted steps' start states
// (checkpoints); each step's stage accelerations are solved again, in the
// forward's order and with its warm starts, before the step is reversed.
// the first a.npar model-parameter cotangents of world w
template <int L>
DMX_DEV void store_params(const AdjArgs& a, int w, const double* hb, int tl) {
  if (a.npar == kParams) team_store<kParams, L>(a.hbar + (size_t)w * kParams, hb, tl);
  else team_store<3, L>(a.hbar + (size_t)w * 3, hb, tl);
}

// HB: the model parameters' cotangent is accumulated (a.hbar set); a template
// flag, so that the plain reverse sweep carries none of its registers
template <class P, bool RECOMPUTE, bool HB = false>
DMX_DEV void adj_world(const typename P::Model& m, const AdjArgs& a, int w, int tl, double (*A)[P::NV],
                       double (*Ab)[P::NV]) {
  constexpr int L = P::TEAM, NQ = P::NQ, NV = P::NV, NX = NQ + NV;
  const SolverOpts& o = a.o;
  const int nsteps = a.n_acc[w];
  // u_bar entries of this world: its own intervals in a packed layout, the
  // whole dense row otherwise (intervals beyond the world's count get 0)
  const size_t nut = (size_t)(a.g.u_off ? world_intervals(a.g, a.n_int, w) : a.n_int) * a.nu;
  const size_t uoff = world_u(a.g, a.n_int, a.nu, w);
  const double* uw = a.u ? a.u + uoff : nullptr;
  double* ubw = a.ubar ? a.ubar + uoff : nullptr;
  const double* tape_w = a.tape + world_tape(a.g, a.cap, w) * a.rec;
  if (a.status[w] != 0) {
    const double nan = __longlong_as_double(0x7ff8000000000000ll);
    for (int i = tl; i < NX; i += L) a.x0bar[(size_t)w * NX + i] = nan;
    for (size_t i = tl; i < nut; i += L) ubw[i] = nan;
    if (HB) for (int i = tl; i < a.npar; i += L) a.hbar[(size_t)w * a.npar + i] = nan;
    return;
  }
  for (size_t i = tl; i < nut; i += L) ubw[i] = 0.0;
  // the model parameters' cotangent: every stage's acceleration map uses the
  // same parameters, so their cotangents add up over all stages and steps
  double hb[HB ? kParams : 1];
#pragma unroll
  for (int i = 0; i < (HB ? kParams : 1); ++i) hb[i] = 0.0;
  double yb[NX];
#pragma unroll
  for (int i = 0; i < NX; ++i) yb[i] = a.xbar[(size_t)w * NX + i];
  double tau[NV], tb_acc[NV];
  int cur_k = -1;
  Stat st{};
  for (int s = nsteps - 1; s >= 0; --s) {
    const double* rec = tape_w + (size_t)s * a.rec;
    const double h = rec[1];
    const int kk = (int)rec[2];
    // touch the previous record's cache lines (one word per 128 bytes, one
    // lane each) so that the next step's loads find them in L2; the word is
    // consumed at the end of this step, long after it arrived
    float warm = 0.0f;
    {
      const int line = min(tl * 16, a.rec - 1);  // 16 doubles per 128-byte line; the last word too
      if (s > 0 && tl * 16 < a.rec + 16) warm = *(const float*)(rec - a.rec + line);
    }
    if (tl == 0) st.u_step++;
    if (kk != cur_k) {
      if (cur_k >= 0 && tl == 0) store_ubar<P>(m, tb_acc, ubw + (size_t)cur_k * a.nu, a.nu);
      cur_k = kk;
      load_tau<P>(m, uw, kk, a.nu, tau);
#pragma unroll
      for (int i = 0; i < NV; ++i) tb_acc[i] = 0.0;
    }
    double y[NX];
#pragma unroll
    for (int i = 0; i < NX; ++i) y[i] = rec[3 + i];
#pragma unroll
    for (int j = 0; j < 6; ++j)
#pragma unroll
      for (int d = 0; d < NV; ++d) Ab[j][d] = 0.0;
    if constexpr (RECOMPUTE) {
#pragma unroll 1
      for (int i = 0; i < 6; ++i) {
        double Y[NX], dq[NV], ai[NV];
        if (i == 0) {
#pragma unroll
          for (int j = 0; j < NX; ++j) Y[j] = y[j];
        } else {
          stage_state<P>(y, A, i, h, Y, dq, nullptr, o.tableau);
        }
        P::acc(m, Y, tau, false, o.beta, o.newton_maxit, i > 0 ? A[i - 1] : nullptr, ai, st);
#pragma unroll
        for (int d = 0; d < NV; ++d) A[i][d] = ai[d];
      }
    } else {  // stage accelerations into LDS, entry j by lane j mod L
      double* Af = &A[0][0];
#pragma unroll
      for (int r = 0; r < (6 * NV + L - 1) / L; ++r) {
        const int j = tl + r * L;
        if (j < 6 * NV) Af[j] = rec[3 + NX + j];
      }
      wave_fence();
    }
#pragma unroll
    for (int d = 0; d < NV; ++d) A[6][d] = 0.0;
    double qb[NQ], vb[NV];
#pragma unroll
    for (int i = 0; i < NQ; ++i) qb[i] = 0.0;
#pragma unroll
    for (int d = 0; d < NV; ++d) vb[d] = 0.0;
    double Ybar[NX];
#pragma unroll
    for (int i = 0; i < NX; ++i) Ybar[i] = yb[i];
#pragma unroll 1
    for (int i = 6; i >= 0; --i) {
      double Y[NX], dq[NV];
      typename P::QPlusKeep qk;
      if (i < 6) {
        if (i > 0) {
          stage_state<P>(y, A, i, h, Y, dq, &qk, o.tableau);
        } else {  // stage 0 is the step's start state
#pragma unroll
          for (int j = 0; j < NX; ++j) Y[j] = y[j];
        }
        double tb[NV], xs[NV], ab[NV];
#pragma unroll
        for (int d = 0; d < NV; ++d) { xs[d] = A[i][d]; ab[d] = Ab[i][d]; }
        P::acc_vjp(m, Y, tau, xs, ab, o.cfd != 0, o.beta, o.newton_maxit, Ybar, tb, st, HB ? hb : nullptr);
#pragma unroll
        for (int d = 0; d < NV; ++d) tb_acc[d] += tb[d];
      } else {
        stage_state<P>(y, A, 6, h, Y, dq, &qk, o.tableau);
      }
      if (i == 0) {
#pragma unroll
        for (int j = 0; j < NQ; ++j) qb[j] += Ybar[j];
#pragma unroll
        for (int d = 0; d < NV; ++d) vb[d] += Ybar[NQ + d];
      } else {
        double dqb[NV];
        P::qplus_vjp(y, dq, Ybar, qb, dqb, &qk);
        stage_distribute<P>(i, Ybar, dqb, h, vb, Ab, o.tableau);
      }
    }
#pragma unroll
    for (int i = 0; i < NQ; ++i) yb[i] = qb[i];
#pragma unroll
    for (int d = 0; d < NV; ++d) yb[NQ + d] = vb[d];
    asm volatile("" ::"v"(warm));
  }
  if (cur_k >= 0 && tl == 0) store_ubar<P>(m, tb_acc, ubw + (size_t)cur_k * a.nu, a.nu);
  team_store<NX, L>(a.x0bar + (size_t)w * NX, yb, tl);
  if (HB) store_params<L>(a, w, hb, tl);
  if (a.counters) {
    double c[kAdjCounters] = {(double)st.u_step, (double)st.u_vjp, (double)st.u_vcon, (double)st.u_vedge};
    team_sum_arr<L, kAdjCounters>(c);
    if (tl == 0)
      for (int i = 0; i < kAdjCounters; ++i) a.counters[(size_t)w * kAdjCounters + i] = (long long)c[i];
  }
}

template <class P, bool RECOMPUTE = false, bool HB = false>
__global__ void __launch_bounds__(64) adj_kernel(const typename P::Model* __restrict__ model, AdjArgs a) {
  constexpr int L = P::TEAM, NV = P::NV;
  const int gt = blockIdx.x * blockDim.x + threadIdx.x;
  const int team = gt / L, tl = gt & (L - 1);
  __shared__ double sA[64 / L][7][NV];
  __shared__ double sAb[64 / L][6][NV];
  double (*A)[NV] = sA[(threadIdx.x & 63) / L];
  double (*Ab)[NV] = sAb[(threadIdx.x & 63) / L];
  stage_pairs(*model);
  for (bool first = true;; first = false) {
    const int w = take_world<L>(a.g, a.W, team, first);
    if (w < 0) break;
    adj_world<P, RECOMPUTE, HB>(*model, a, w, tl, A, Ab);
  }
}

// ------------------------------------------------------------ optimize-then-discretize
// The continuous adjoint equations (App. C.2, eq. adjoint-equations): for a
// loss on the final state, lam(T) = dL/dx(T), dlam/dt = -(dF/dx)^T lam, and
// each control interval's gradient is the integral of (dF/du)^T lam over it;
// with the straight-through rule (App. C.4) dF/dx is that of the CFD field at
// the trajectory of F.  They are solved backwards in time with the forward's
// Dormand-Prince pair and PI controller but their own steps, in raw
// coordinates (dq/dt = v, a free joint's quaternion (1/2) q (x) (0, w)), along
// x(t) from the continuous extension of the forward's accepted steps; each
// stage solves the contact problem at x(t) and applies acc_vjp and the
// kinematic VJP.  The adjoint's steps land on the interval ends, start from the
// forward's last step size and are floored at 1e-12 max(1, |t|) (a floor step
// is accepted: dF/dx jumps where a contact switches on).  The returned
// quaternion gradient is projected onto the tangent space at q(0).

// weights of the stage slopes in the fourth-order continuous extension of the
// Dormand-Prince pair (Hairer, Norsett and Wanner): over the fraction th of a
// step the increment is h sum_i w_i k_i with
// w = th b + th (1 - th) (e_1 - b) + th^2 (1 - th) (2 b - e_1 - e_7) + th^2 (1 - th)^2 d
constexpr double kDenseD[7] = {-12715105075.0 / 11282082432.0, 0.0, 87487479700.0 / 32700410799.0,
                               -10690763975.0 / 1880347072.0, 701980252875.0 / 199316789632.0,
                               -1453857185.0 / 822651844.0, 69997945.0 / 29380423.0};
DMX_DEV void dense_weights(double th, double* w) {
  const double p1 = th * (1.0 - th), p2 = th * p1, p3 = p2 * (1.0 - th);
#pragma unroll
  for (int i = 0; i < 7; ++i) {
    const double b = i < 6 ? kTab.a[6][i] : 0.0;
    const double e1 = i == 0 ? 1.0 : 0.0, e7 = i == 6 ? 1.0 : 0.0;
    w[i] = th * b + p1 * (e1 - b) + p2 * (2.0 * b - e1 - e7) + p3 * kDenseD[i];
  }
}

// A: stage accelerations and V: stage velocities (LDS, [7][NV]) of the
// forward step the continuous extension currently reads; G, TB: the adjoint's
// stage slopes (raw state cotangent rates, generalized-force cotangents).
// HB: the model parameters' cotangent is accumulated (a.hbar set).
template <class P, bool HB = false>
DMX_DEV void otd_world(const typename P::Model& m, const AdjArgs& a, int w, int tl, double (*A)[P::NV],
                       double (*V)[P::NV], double (*G)[P::NQ + P::NV], double (*TB)[P::NV]) {
  constexpr int L = P::TEAM, NQ = P::NQ, NV = P::NV, NX = NQ + NV;
  const SolverOpts& o = a.o;
  const int N = a.n_acc[w];
  const int n_int = world_intervals(a.g, a.n_int, w);
  const size_t nut = (size_t)(a.g.u_off ? n_int : a.n_int) * a.nu;
  const size_t uoff = world_u(a.g, a.n_int, a.nu, w);
  const double* uw = a.u ? a.u + uoff : nullptr;
  double* ubw = a.ubar ? a.ubar + uoff : nullptr;
  const double* tape_w = a.tape + world_tape(a.g, a.cap, w) * a.rec;
  const double nan = __longlong_as_double(0x7ff8000000000000ll);
  if (a.status[w] != 0 || N <= 0) {
    for (int i = tl; i < NX; i += L) a.x0bar[(size_t)w * NX + i] = nan;
    for (size_t i = tl; i < nut; i += L) ubw[i] = nan;
    if (HB) for (int i = tl; i < a.npar; i += L) a.hbar[(size_t)w * a.npar + i] = nan;
    return;
  }
  // a dense control row longer than the world's horizon: the intervals it
  // never reaches get 0 (its own intervals are written as the sweep leaves them)
  for (size_t i = (size_t)n_int * a.nu + tl; i < nut; i += L) ubw[i] = 0.0;
  // the model parameters' adjoint (a_theta of the adjoint equations): stage
  // slopes PB and its quadrature, accumulated only when asked for
  constexpr int NPH = HB ? kParams : 1;
  double PB[7][NPH], hacc[NPH];
#pragma unroll
  for (int q = 0; q < NPH; ++q) hacc[q] = 0.0;
  double lam[NX];
#pragma unroll
  for (int i = 0; i < NX; ++i) lam[i] = a.xbar[(size_t)w * NX + i];
  Stat st{};
  // the forward step read by the continuous extension
  int cur = -1, nguess = N - 1;
  double yc[NX], tc = 0.0, hc = 1.0;
  double xw[NV];
  bool have_xw = false;
  auto rec_end = [&](int n) { return tape_w[(size_t)n * a.rec] + tape_w[(size_t)n * a.rec + 1]; };
  auto load_step = [&](int n) {
    const double* r = tape_w + (size_t)n * a.rec;
    tc = r[0];
    hc = r[1];
    const int kn = (int)r[2];
#pragma unroll
    for (int i = 0; i < NX; ++i) yc[i] = r[3 + i];
    double* Af = &A[0][0];
#pragma unroll
    for (int rr = 0; rr < (6 * NV + L - 1) / L; ++rr) {
      const int j = tl + rr * L;
      if (j < 6 * NV) Af[j] = r[3 + NX + j];
    }
    wave_fence();
#pragma unroll
    for (int d = 0; d < NV; ++d) V[0][d] = yc[NQ + d];
    double Y[NX], dq[NV];
#pragma unroll 1
    for (int i = 1; i < 7; ++i) {
      stage_state<P>(yc, A, i, hc, Y, dq);
#pragma unroll
      for (int d = 0; d < NV; ++d) V[i][d] = Y[NQ + d];
    }
    // slope at y_{n+1} under this step's control: the next record's first
    // stage when it continues the same interval, else solved here
    if (n + 1 < N && (int)tape_w[(size_t)(n + 1) * a.rec + 2] == kn) {
      const double* r1 = tape_w + (size_t)(n + 1) * a.rec + 3 + NX;
#pragma unroll
      for (int d = 0; d < NV; ++d) A[6][d] = r1[d];
    } else {
      double taun[NV], a7[NV];
      load_tau<P>(m, uw, kn, a.nu, taun);
      P::acc(m, Y, taun, false, o.beta, o.newton_maxit, A[5], a7, st);
#pragma unroll
      for (int d = 0; d < NV; ++d) A[6][d] = a7[d];
    }
    wave_fence();
  };
  // x(tau): the first step with tau < t_n + h_n (the last one otherwise)
  auto dense = [&](double tau, double* x) {
    int n = nguess;
    while (n > 0 && tau < rec_end(n - 1)) --n;
    while (n < N - 1 && !(tau < rec_end(n))) ++n;
    nguess = n;
    if (n != cur) { load_step(n); cur = n; }
    double wt[7], dq[NV];
    dense_weights(fmin(1.0, fmax(0.0, (tau - tc) / hc)), wt);
#pragma unroll
    for (int d = 0; d < NV; ++d) {
      double sq = 0.0, sv = 0.0;
#pragma unroll
      for (int i = 0; i < 7; ++i) { sq += wt[i] * V[i][d]; sv += wt[i] * A[i][d]; }
      dq[d] = hc * sq;
      x[NQ + d] = yc[NQ + d] + hc * sv;
    }
    P::qplus(yc, dq, x);
  };
  // start of the last accepted forward step that begins before tt: the
  // adjoint's steps end on the forward's step boundaries, never across them,
  // so the short steps the forward took through a contact phase are never
  // skipped by one long adjoint step
  int nlo = N - 1;
  auto step_start = [&](double tt) {
    int n = nlo;
    while (n > 0 && !(tape_w[(size_t)n * a.rec] < tt)) --n;
    while (n < N - 1 && tape_w[(size_t)(n + 1) * a.rec] < tt) ++n;
    nlo = n;
    return tape_w[(size_t)n * a.rec];
  };
  double hprop = tape_w[(size_t)(N - 1) * a.rec + 1], eprev = 1.0;
  long long attempts = 0;
  bool failed = false;
  for (int kk = n_int - 1; kk >= 0 && !failed; --kk) {
    double tau[NV], tb_acc[NV];
    load_tau<P>(m, uw, kk, a.nu, tau);
#pragma unroll
    for (int d = 0; d < NV; ++d) tb_acc[d] = 0.0;
    const double tlo = (double)kk * a.dt;
    double t = (double)(kk + 1) * a.dt;
    bool have_g1 = false;
    while (t > tlo) {
      const double lo = fmax(tlo, step_start(t));
      const bool landing = t - 1.01 * hprop <= lo;
      const double H = landing ? t - lo : hprop;
      if (attempts >= o.max_attempts) { failed = true; break; }
      ++attempts;
#pragma unroll 1
      for (int i = 0; i < 7; ++i) {
        if (i == 0 && have_g1) continue;
        double Lam[NX];
        if (i == 0) {
#pragma unroll
          for (int r = 0; r < NX; ++r) Lam[r] = lam[r];
        } else {
          const StageCoef k = stage_coef(i);
#pragma unroll
          for (int r = 0; r < NX; ++r) {
            double s = 0.0;
#pragma unroll
            for (int j = 0; j < 6; ++j) s += k.a[j] * (j < i ? G[j][r] : 0.0);
            Lam[r] = lam[r] + H * s;
          }
        }
        double x[NX], xs[NV], tb[NV], ybar[NX];
        dense(t - kTab.c[i] * H, x);
        P::acc(m, x, tau, false, o.beta, o.newton_maxit, have_xw ? xw : nullptr, xs, st);
#pragma unroll
        for (int d = 0; d < NV; ++d) xw[d] = xs[d];
        have_xw = true;
#pragma unroll
        for (int r = 0; r < NX; ++r) ybar[r] = 0.0;
        double hbi[NPH];
#pragma unroll
        for (int q = 0; q < NPH; ++q) hbi[q] = 0.0;
        P::acc_vjp(m, x, tau, xs, Lam + NQ, o.cfd != 0, o.beta, o.newton_maxit, ybar, tb, st,
                   HB ? hbi : nullptr);
#pragma unroll
        for (int q = 0; q < NPH; ++q) PB[i][q] = hbi[q];
        P::kin_vjp(x, Lam, ybar);
#pragma unroll
        for (int r = 0; r < NX; ++r) G[i][r] = ybar[r];
#pragma unroll
        for (int d = 0; d < NV; ++d) TB[i][d] = tb[d];
        wave_fence();
      }
      if (st.status & 12) { failed = true; break; }
      double lamn[NX], acc2 = 0.0;
#pragma unroll
      for (int r = 0; r < NX; ++r) {
        double s5 = 0.0, se = 0.0;
#pragma unroll
        for (int i = 0; i < 7; ++i) {
          const double g = G[i][r];
          s5 += (i < 6 ? kTab.a[6][i] : 0.0) * g;
          se += kTab.e[i] * g;
        }
        lamn[r] = lam[r] + H * s5;
        const double q = (H * se) / (o.atol + o.rtol * fmax(fabs(lam[r]), fabs(lamn[r])));
        acc2 += q * q;
      }
      bool fin = true;
#pragma unroll
      for (int r = 0; r < NX; ++r) fin = fin && isfinite(lamn[r]);
      if (!fin) { failed = true; break; }  // a non-finite cotangent ends the world (NaN gradients)
      const double err = sqrt(acc2 / NX);
      const double hmin = 1e-12 * fmax(1.0, fabs(t));
      const bool accept = err <= 1.0 || H <= hmin;
      const double et = isfinite(err) ? fmax(err, o.err_floor) : 1e300;
      double fac = o.safety * pow(et, -(o.kP + o.kI) / o.err_order) * pow(eprev, o.kP / o.err_order);
      fac = fmin(o.facmax, fmax(o.facmin, fac));
      double hnext;
      if (accept) {
#pragma unroll
        for (int d = 0; d < NV; ++d) {
          double s = 0.0;
#pragma unroll
          for (int j = 0; j < 6; ++j) s += kTab.a[6][j] * TB[j][d];
          tb_acc[d] += H * s;
        }
        if (HB) {
#pragma unroll
          for (int q = 0; q < NPH; ++q) {
            double s = 0.0;
#pragma unroll
            for (int j = 0; j < 6; ++j) s += kTab.a[6][j] * PB[j][q];
            hacc[q] += H * s;
            PB[0][q] = PB[6][q];
          }
        }
#pragma unroll
        for (int r = 0; r < NX; ++r) { lam[r] = lamn[r]; G[0][r] = G[6][r]; }
#pragma unroll
        for (int d = 0; d < NV; ++d) TB[0][d] = TB[6][d];
        wave_fence();
        have_g1 = true;
        t = landing ? lo : t - H;
        eprev = et;
        hnext = quantize_step(fac * H, o.h_levels);
        if (tl == 0) st.u_step++;
      } else {
        hnext = quantize_step(fmin(1.0, fac) * H, o.h_levels);
      }
      hprop = fmax(hnext, hmin);
    }
    if (!failed && ubw && tl == 0) store_ubar<P>(m, tb_acc, ubw + (size_t)kk * a.nu, a.nu);
  }
  if (failed) {
    for (int i = tl; i < NX; i += L) a.x0bar[(size_t)w * NX + i] = nan;
    for (size_t i = tl; i < nut; i += L) ubw[i] = nan;
    if (HB) for (int i = tl; i < a.npar; i += L) a.hbar[(size_t)w * a.npar + i] = nan;
  } else {
    P::tangent_project(tape_w + 3, lam);
    team_store<NX, L>(a.x0bar + (size_t)w * NX, lam, tl);
    if (HB) store_params<L>(a, w, hacc, tl);
  }
  if (a.counters) {
    double c[kAdjCounters] = {(double)st.u_step, (double)st.u_vjp, (double)st.u_vcon, (double)st.u_vedge};
    team_sum_arr<L, kAdjCounters>(c);
    if (tl == 0)
      for (int i = 0; i < kAdjCounters; ++i) a.counters[(size_t)w * kAdjCounters + i] = (long long)c[i];
  }
}

// One team per world; the stage slopes of teams of two or more lanes sit in
// LDS, those of one-lane teams (64 worlds per wavefront) in private memory.
template <class P, bool HB = false>
__global__ void __launch_bounds__(64) otd_kernel(const typename P::Model* __restrict__ model, AdjArgs a) {
  constexpr int L = P::TEAM, NV = P::NV, NX = P::NQ + P::NV;
  const int gt = blockIdx.x * blockDim.x + threadIdx.x;
  const int team = gt / L, tl = gt & (L - 1);
  __shared__ double sA[64 / L][7][NV];
  __shared__ double sV[64 / L][7][NV];
  double (*A)[NV] = sA[(threadIdx.x & 63) / L];
  double (*V)[NV] = sV[(threadIdx.x & 63) / L];
  stage_pairs(*model);
  if constexpr (L == 1) {
    double Gp[7][NX], Tp[7][NV];
    for (bool first = true;; first = false) {
      const int w = take_world<L>(a.g, a.W, team, first);
      if (w < 0) break;
      otd_world<P, HB>(*model, a, w, tl, A, V, Gp, Tp);
    }
  } else {
    __shared__ double sG[64 / L][7][NX];
    __shared__ double sT[64 / L][7][NV];
    double (*G)[NX] = sG[(threadIdx.x & 63) / L];
    double (*T)[NV] = sT[(threadIdx.x & 63) / L];
    for (bool first = true;; first = false) {
      const int w = take_world<L>(a.g, a.W, team, first);
      if (w < 0) break;
      otd_world<P, HB>(*model, a, w, tl, A, V, G, T);
    }
  }
}

}  // namespace dmx
