// Free-body worlds: one body on a free joint touching world planes through
// sphere and capsule geoms.  Forward acceleration (team-parallel over contact
// slots) and its vector-Jacobian product.
//
// Physics (paper Sec. 2 and 2.1):
//  - v = (world linear velocity of the body origin, body-frame angular
//    velocity); with the centre of mass at the origin M = diag(m I3, I_body)
//    is constant and the bias is c = (-m g, w x I w).
//  - contacts with signed distance r < 0 (r < w_c for the CFD field) produce
//    the 4 edge rows J_n +- mu J_t of a pyramidal cone; a_ref = -b J v - k r,
//    b = 2/(d_w t_c), k = d(r)/(d_w^2 t_c^2 phi^2), R = A (1-d)/d, D = 1/R.
//  - the acceleration is the minimizer of the convex primal problem
//    1/2 |x - a0|_M^2 + sum_e 1/2 D_e min(0, J_e x - a_ref_e)^2, found by an
//    exact Newton method (Sec. 2.1).
#pragma once
#include "dmx_common.hpp"

namespace dmx {

constexpr int kMaxPairs = 16;
constexpr int kMaxSlots = 32;

struct PairF {
  int gtype, ncon;
  double l[3];     // geom centre, body frame
  double ax[3];    // capsule: half-length * axis, body frame; box: half sizes
  double gR[9];    // box: geom rotation in the body frame (row-major)
  double rad;
  double p0[3], n[3], t1[3], t2[3];  // world plane point, contact normal and tangents
  double mu, bcoef, kscale, ahat;
  double solref[2];  // (t_c, damping ratio) that bcoef and kscale come from
  double si[5], cf[5];
  double ssc[4];  // spline scales 1/mid^(p-1), 1/(1-mid)^(p-1): penetration (0, 1) and CFD (2, 3)
  double iwid[2]; // 1/width of the penetration and CFD splines
};

// Contact-pair constants and the slot -> (pair, capsule end) table, staged in
// LDS once per block by stage_pairs(): lanes read their own slots' pairs, so
// from global memory these would be vector loads with a full memory latency
// each right-hand side.
DMX_DEV PairF* lds_pairs() {
  __shared__ PairF s[kMaxPairs];
  return s;
}
DMX_DEV int* lds_slots() {  // [0, kMaxSlots): pair of slot; [kMaxSlots, 2 kMaxSlots): capsule end
  __shared__ int s[2 * kMaxSlots];
  return s;
}
DMX_DEV const PairF& slot_pair(int c) { return lds_pairs()[lds_slots()[c]]; }
DMX_DEV int slot_sub(int c) { return lds_slots()[kMaxSlots + c]; }

// Block-wide copy of a model's pair table into LDS (every thread of the block
// calls it before any thread leaves).
template <class M>
DMX_DEV void stage_pairs(const M& mod) {
  const double* src = (const double*)mod.pair;
  double* dst = (double*)lds_pairs();
  constexpr int n = (int)(sizeof(PairF) * kMaxPairs / sizeof(double));
  for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
  int* sl = lds_slots();
  for (int i = threadIdx.x; i < kMaxSlots; i += blockDim.x) {
    sl[i] = mod.cpair[i];
    sl[kMaxSlots + i] = mod.csub[i];
  }
  __syncthreads();
}

struct FreeModel {
  int np, nc, nu;
  int cpair[kMaxSlots], csub[kMaxSlots];
  int ctrl[8];
  double mass, imass, I[9], Iinv[9], grav[3];
  PairF pair[kMaxPairs];
};

// Per-world status and work-unit counters.  Team-level events are counted
// by lane 0 of the team, per-contact events by the lane owning the contact;
// the counters are summed over the team when written out.
struct Stat {
  int newton_it;
  int status;
  long long u_att, u_rhs, u_con, u_nit, u_ncon, u_nedge, u_ls;  // forward
  long long u_step, u_vjp, u_vcon, u_vedge;                      // reverse
};
DMX_DEV bool team_leader(int L) { return (threadIdx.x & (L - 1)) == 0; }

// ------------------------------------------------------------ impedance
// x^e for the spline exponent e = power - 1 (small integer exponents by
// multiplication; the exponent is a model constant, so the branch is uniform).
DMX_DEV double spline_pow(double x, double e) {
  if (e == 1.0) return x;
  if (e == 2.0) return x * x;
  if (e == 0.0) return 1.0;
  if (e == 3.0) return x * x * x;
  return pow(x, e);
}

// MuJoCo-style polynomial spline y(x) on [0, 1] with midpoint and power, and
// dy/dx; s_lo = 1/mid^(pw-1) and s_hi = 1/(1-mid)^(pw-1) are precomputed.
DMX_DEV double imp_spline(double x, double mid, double pw, double s_lo, double s_hi, double* dydx) {
  if (x >= 1.0) { *dydx = 0.0; return 1.0; }
  if (x <= 0.0) { *dydx = 0.0; return 0.0; }
  if (x <= mid) {
    const double xp = spline_pow(x, pw - 1.0) * s_lo;
    *dydx = pw * xp;
    return xp * x;
  }
  const double z = 1.0 - x;
  const double zp = spline_pow(z, pw - 1.0) * s_hi;
  *dydx = pw * zp;
  return 1.0 - zp * z;
}

// Impedance d(r) and dd/dr.  Penetration (r < 0): solimp spline of -r/width
// from d0 to dwidth.  Contacts from distance (r >= 0, CFD field only): the
// continuation from d_0 at r = 0 to d_c at r = w_c.
DMX_DEV double impedance(const PairF& p, double r, double* ddr) {
  double dy;
  if (r < 0.0) {
    double x = -r * p.iwid[0];
    double y = imp_spline(x, p.si[3], p.si[4], p.ssc[0], p.ssc[1], &dy);
    *ddr = -dy * p.iwid[0] * (p.si[1] - p.si[0]);
    return p.si[0] + y * (p.si[1] - p.si[0]);
  }
  double x = r * p.iwid[1];
  double y = imp_spline(x, p.cf[3], p.cf[4], p.ssc[2], p.ssc[3], &dy);
  *ddr = dy * p.iwid[1] * (p.cf[0] - p.cf[1]);
  return p.cf[1] + y * (p.cf[0] - p.cf[1]);
}

// Derivatives of the penetration impedance d(r) (r < 0) with respect to the
// solimp parameters (d0, dwidth, width, midpoint, power); zero for r >= 0,
// where the contacts-from-distance spline (its own parameters) or no row
// applies.  With x = -r / width and the power spline y(x):
// d = d0 + y (dwidth - d0); dy/dmid and dy/dpower from y = x^p / mid^(p-1)
// below the midpoint and y = 1 - (1-x)^p / (1-mid)^(p-1) above it.
DMX_DEV void impedance_solimp_grad(const PairF& p, double r, double* g) {
#pragma unroll
  for (int i = 0; i < 5; ++i) g[i] = 0.0;
  if (r >= 0.0) return;
  const double x = -r * p.iwid[0], mid = p.si[3], pw = p.si[4], span = p.si[1] - p.si[0];
  double dy;
  const double y = imp_spline(x, mid, pw, p.ssc[0], p.ssc[1], &dy);
  g[0] = 1.0 - y;
  g[1] = y;
  if (x >= 1.0) return;
  g[2] = -span * dy * x * p.iwid[0];
  if (x <= mid) {
    g[3] = -span * (pw - 1.0) * y / mid;
    g[4] = span * y * log(x / mid);
  } else {
    g[3] = -span * (pw - 1.0) * (1.0 - y) / (1.0 - mid);
    g[4] = -span * (1.0 - y) * log((1.0 - x) / (1.0 - mid));
  }
}

DMX_DEV double softplus(double z, double beta, double* dsp) {
  double bz = beta * z;
  if (bz > 30.0) {
    double e = exp(-bz);
    *dsp = 1.0 / (1.0 + e);
    return z + log1p(e) / beta;
  }
  double e = exp(bz);
  *dsp = e / (1.0 + e);
  return log1p(e) / beta;
}

// ------------------------------------------------------------ contact rows
// Rows of a lane's contact slots: the normal row and NT tangent rows.  NT = 2:
// both tangent directions and the four pyramid edges J_n + mu J_t1,
// J_n - mu J_t1, J_n + mu J_t2, J_n - mu J_t2 on one lane.  NT = 1: a contact
// sits on two lanes of the team, lane l < L/2 and its mirror L-1-l; the first
// holds tangent direction t1 and its two edges, the second t2 and its two;
// every per-contact sum is linear in the edge terms, so the team sums add the
// halves.
template <int CPL, int NT>
struct FreeRows {
  bool on[CPL];
  bool first[CPL];  // the lane that counts the contact (one per contact)
  int slot[CPL];
  int half[CPL];    // NT = 1: tangent direction t1 (0) or t2 (1) of this lane
  double r[CPL], mu[CPL], D[CPL];
  double Jn[CPL][6], Jt[CPL][NT][6];
  double aref[CPL][2 * NT];
};

DMX_DEV double dot6(const double* a, const double* b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2] + a[3] * b[3] + a[4] * b[4] + a[5] * b[5];
}

// Vertex k of a box pair in the body frame: centre + geom rotation * (+-h),
// with the sign of coordinate x from bit 0 of k, y from bit 1, z from bit 2.
DMX_DEV V3 box_vertex(const PairF& pr, int k) {
  const V3 v = mk3((k & 1) ? pr.ax[0] : -pr.ax[0], (k & 2) ? pr.ax[1] : -pr.ax[1], (k & 4) ? pr.ax[2] : -pr.ax[2]);
  const double* g = pr.gR;
  return ld3(pr.l) + mk3(g[0] * v.x + g[1] * v.y + g[2] * v.z, g[3] * v.x + g[4] * v.y + g[5] * v.z,
                         g[6] * v.x + g[7] * v.y + g[8] * v.z);
}

DMX_DEV double smoothstep01(double t, double* dt) {
  if (t <= 0.0) { *dt = 0.0; return 0.0; }
  if (t >= 1.0) { *dt = 0.0; return 1.0; }
  *dt = 6.0 * t * (1.0 - t);
  return t * t * (3.0 - 2.0 * t);
}

// Smoothed plane-box detection (App. C.1): vertex supports s_k below the
// plane, a soft mask (C^1 smoothstep) keeping the vertices within a 1 mm skin
// of the deepest one, the four largest masked supports in stable descending
// order (ties to the lower vertex index), contact at the vertex moved to the
// midpoint, r = -mask * s.  Slot `rank` takes the rank-th vertex.  For the
// reverse sweep: dr/dg_k (g = height of the vertex above the plane) and
// dr/dg_deepest through the skin threshold, with the deepest vertex.
struct BoxSlot {
  int k, kmax;
  double r, drdg, drdgmax;
};
DMX_DEV BoxSlot box_plane_slot(const PairF& pr, V3 p, const M3& R, int rank) {
  const V3 n = ld3(pr.n), p0 = ld3(pr.p0);
  double sup[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) sup[k] = -dot(n, p + mul(R, box_vertex(pr, k)) - p0);
  int kmax = 0;
#pragma unroll
  for (int k = 1; k < 8; ++k) kmax = sup[k] > sup[kmax] ? k : kmax;
  const bool thr_on = sup[kmax] - 1e-3 > 0.0;
  const double thr = thr_on ? sup[kmax] - 1e-3 : 0.0;
  const double lo = thr - 1e-3, wdt = thr - lo;
  double sm[8], msk[8], dmsk[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    msk[k] = smoothstep01((sup[k] - lo) / wdt, &dmsk[k]);
    sm[k] = msk[k] * sup[k];
  }
  BoxSlot b{0, kmax, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    int rk = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) rk += (sm[j] > sm[k]) || (j < k && sm[j] == sm[k]);
    if (rk == rank) b.k = k;
  }
  // r = -m(u) s with u = (s - lo) / w, s = -g, lo = thr - 1e-3, thr = s_max - 1e-3
  double sk = 0.0, mk = 0.0, dk = 0.0;
#pragma unroll
  for (int k = 0; k < 8; ++k)
    if (k == b.k) { sk = sup[k]; mk = msk[k]; dk = dmsk[k]; }
  b.r = -sm[b.k];
  b.drdg = mk + sk * dk / wdt;             // d(-m s)/ds * ds/dg, ds/dg = -1
  b.drdgmax = thr_on ? -sk * dk / wdt : 0.0;  // via thr: du/dthr = -1/w, dthr/dg_max = -1
  return b;
}

// Contact point of slot c: the sphere (or capsule end sphere) centre, or the
// selected box vertex, in the world; signed distance to the plane and the
// midpoint between the surfaces.
DMX_DEV void slot_geom(const FreeModel& m, int c, V3 p, const M3& R, V3* lc, V3* ctr, double* r, V3* P) {
  const PairF& pr = slot_pair(c);
  const V3 n = ld3(pr.n);
  if (pr.gtype == 3) {
    const BoxSlot b = box_plane_slot(pr, p, R, slot_sub(c));
    *lc = box_vertex(pr, b.k);
    *ctr = p + mul(R, *lc);
    *r = b.r;
    *P = *ctr - (0.5 * b.r) * n;
    return;
  }
  V3 l = ld3(pr.l);
  if (pr.gtype == 2) l = (slot_sub(c) == 0) ? l + ld3(pr.ax) : l - ld3(pr.ax);
  V3 ce = p + mul(R, l);
  double rr = dot(n, ce - ld3(pr.p0)) - pr.rad;
  *lc = l;
  *ctr = ce;
  *r = rr;
  *P = ce - (pr.rad + 0.5 * rr) * n;
}

// Rows of this lane's contact slots at (q, v).  J_u = [u, R^T (d x u)] for a
// frame direction u, with d the contact point relative to the body origin.
template <int CPL, int L, int NT>
DMX_DEV void free_rows(const FreeModel& m, V3 p, const M3& R, const double* v, bool cfd, double beta,
                       FreeRows<CPL, NT>& rw) {
  const int tl = threadIdx.x & (L - 1);
#pragma unroll
  for (int k = 0; k < CPL; ++k) {
    // NT = 2: slot tl + k L; NT = 1 (one slot per lane pair): slot tl on
    // the first half of the team, L - 1 - tl on the second
    const int h = NT == 2 ? 0 : tl / (L / 2);
    const int c = NT == 2 ? tl + k * L : (h ? L - 1 - tl : tl);
    rw.slot[k] = c;
    rw.half[k] = h;
    rw.first[k] = h == 0;
    rw.on[k] = false;
    if (c >= m.nc) continue;
    const PairF& pr = slot_pair(c);
    V3 lc, ce, P;
    double r;
    slot_geom(m, c, p, R, &lc, &ce, &r, &P);
    rw.r[k] = r;
    bool on = cfd ? (r < pr.cf[2]) : (r < 0.0);
    rw.on[k] = on;
    if (!on) continue;
    V3 d = P - p;
    V3 n = ld3(pr.n);
    V3 wn = mulT(R, cross(d, n));
    double* Jn = rw.Jn[k];
    Jn[0] = n.x; Jn[1] = n.y; Jn[2] = n.z; Jn[3] = wn.x; Jn[4] = wn.y; Jn[5] = wn.z;
#pragma unroll
    for (int a = 0; a < NT; ++a) {
      const V3 t = (NT == 2 ? a == 1 : h == 1) ? ld3(pr.t2) : ld3(pr.t1);
      const V3 wt = mulT(R, cross(d, t));
      double* Ja = rw.Jt[k][a];
      Ja[0] = t.x; Ja[1] = t.y; Ja[2] = t.z; Ja[3] = wt.x; Ja[4] = wt.y; Ja[5] = wt.z;
    }
    double ddr;
    double dimp = impedance(pr, r, &ddr);
    double kk = dimp * pr.kscale;
    rw.mu[k] = pr.mu;
    rw.D[k] = dimp / (pr.ahat * (1.0 - dimp));
    double pterm;
    if (cfd) { double dsp; pterm = kk * softplus(-r, beta, &dsp); }
    else pterm = -kk * r;
    const double jnv = dot6(Jn, v);
#pragma unroll
    for (int a = 0; a < NT; ++a) {
      const double jtv = dot6(rw.Jt[k][a], v);
      rw.aref[k][2 * a] = -pr.bcoef * (jnv + pr.mu * jtv) + pterm;
      rw.aref[k][2 * a + 1] = -pr.bcoef * (jnv - pr.mu * jtv) + pterm;
    }
  }
}

// Team sum of a long array: staged through LDS for teams of 8 or more lanes
// (fewer instructions than log2(L) butterfly levels of N moves and adds),
// butterflies otherwise.
template <int L, int LIVE, int N>
DMX_DEV void team_sum_big(double* v) {
  if constexpr (L >= 8) team_sum_lds<L, LIVE, N>(v);
  else team_sum_arr<L, N>(v);
}

// y = M x for the constant free-body mass matrix
DMX_DEV void free_Mmul(const FreeModel& m, const double* x, double* y) {
  y[0] = m.mass * x[0]; y[1] = m.mass * x[1]; y[2] = m.mass * x[2];
  y[3] = m.I[0] * x[3] + m.I[1] * x[4] + m.I[2] * x[5];
  y[4] = m.I[3] * x[3] + m.I[4] * x[4] + m.I[5] * x[5];
  y[5] = m.I[6] * x[3] + m.I[7] * x[4] + m.I[8] * x[5];
}

// H = M + sum over this team's active edges of D J_e J_e^T, packed lower
// triangle (21 entries).  With J_e = J_n + s_e J_t(e), s = (mu, -mu, mu, -mu)
// on (J_t1, J_t1, J_t2, J_t2), a contact's four edges sum to
//   w_nn J_n J_n^T + w_n1 (J_n J_t1^T + J_t1 J_n^T) + w_n2 (J_n J_t2^T + J_t2 J_n^T)
//   + w_11 J_t1 J_t1^T + w_22 J_t2 J_t2^T
// with the weights below (an inactive edge has weight 0).
// This lane's share (its own slots) of the contact part, before the team sum.
template <int CPL, int NT>
DMX_DEV void free_hessian_lane(const FreeRows<CPL, NT>& rw, const uint32_t* act, double* hp) {
#pragma unroll
  for (int i = 0; i < 21; ++i) hp[i] = 0.0;
#pragma unroll
  for (int k = 0; k < CPL; ++k) {
    if (act[k] == 0u) continue;
    const double D = rw.D[k], mu = rw.mu[k];
    double o[2 * NT];
#pragma unroll
    for (int e = 0; e < 2 * NT; ++e) o[e] = ((act[k] >> e) & 1u) ? D : 0.0;
    double waa[NT], wna[NT];
#pragma unroll
    for (int a = 0; a < NT; ++a) { waa[a] = o[2 * a] + o[2 * a + 1]; wna[a] = mu * (o[2 * a] - o[2 * a + 1]); }
    const double wnn = NT == 2 ? waa[0] + waa[NT - 1] : waa[0];
    const double mm = mu * mu;
    const double* Jn = rw.Jn[k];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      double ui = wnn * Jn[i];
      double va[NT];
#pragma unroll
      for (int a = 0; a < NT; ++a) {
        ui += wna[a] * rw.Jt[k][a][i];
        va[a] = wna[a] * Jn[i] + mm * waa[a] * rw.Jt[k][a][i];
      }
#pragma unroll
      for (int j = 0; j <= i; ++j) {
        double hij = ui * Jn[j];
#pragma unroll
        for (int a = 0; a < NT; ++a) hij += va[a] * rw.Jt[k][a][j];
        hp[tri(i, j)] += hij;
      }
    }
  }
}
DMX_DEV void free_add_mass(const FreeModel& m, double* hp) {
  hp[tri(0, 0)] += m.mass; hp[tri(1, 1)] += m.mass; hp[tri(2, 2)] += m.mass;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) hp[tri(3 + i, 3 + j)] += m.I[i * 3 + j];
}
template <int CPL, int L, int LIVE, int NT>
DMX_DEV void free_hessian(const FreeModel& m, const FreeRows<CPL, NT>& rw, const uint32_t* act, double* hp) {
  free_hessian_lane<CPL, NT>(rw, act, hp);
  team_sum_big<L, LIVE, 21>(hp);
  free_add_mass(m, hp);
}

// Active edges at x: bit e of act[k] set iff J_e x - a_ref_e < 0.
template <int CPL, int NT>
DMX_DEV void free_active(const FreeRows<CPL, NT>& rw, const double* x, uint32_t* act, double (*s)[4]) {
#pragma unroll
  for (int k = 0; k < CPL; ++k) {
    act[k] = 0u;
    if (!rw.on[k]) continue;
    const double jn = dot6(rw.Jn[k], x);
    const double mu = rw.mu[k];
#pragma unroll
    for (int a = 0; a < NT; ++a) {
      const double ja = dot6(rw.Jt[k][a], x);
      const double jx[2] = {jn + mu * ja, jn - mu * ja};
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int e = 2 * a + b;
        s[k][e] = jx[b] - rw.aref[k][e];
        if (s[k][e] < 0.0) act[k] |= 1u << e;
      }
    }
  }
}

// Active-edge mask of the contact on this lane and on its mirror lane
// L - 1 - l (NT = 1 splits a contact over the two).
template <int NT, int L>
DMX_DEV uint32_t contact_bits(uint32_t act) {
  if constexpr (NT == 2) {
    return act;
  } else {
    static_assert(L == 8 || L == 16, "mirror exchange within a row of 16");
    return act | (uint32_t)__builtin_amdgcn_mov_dpp((int)act, L == 8 ? 0x141 : 0x140, 0xF, 0xF, true);
  }
}

template <int CPL, int L>
DMX_DEV bool same_active(const uint32_t* a, const uint32_t* b) {
  bool same = true;
#pragma unroll
  for (int k = 0; k < CPL; ++k) same = same && (a[k] == b[k]);
  return team_all<L>(same);
}

// Exact Newton solve of the primal problem, started at a0.  Each iteration
// takes the Newton direction of the current active set; if no row changes
// activity on the unit step it is the exact minimizer (the active set is
// then unchanged) and the solve ends; otherwise the exact minimizer along the
// direction is found by a bracketed semismooth Newton iteration on the
// piecewise-linear directional derivative.
template <int CPL, int L, int LIVE, int NT>
DMX_DEV void free_newton(const FreeModel& m, const FreeRows<CPL, NT>& rw, const double* a0, const double* xw, double* x,
                         int maxit, Stat& st) {
  constexpr int NE = 2 * NT;  // edges per lane slot
#pragma unroll
  for (int i = 0; i < 6; ++i) x[i] = a0[i];
  uint32_t act[CPL];
  double s[CPL][4];
  free_active<CPL, NT>(rw, x, act, s);
  bool any = false;
#pragma unroll
  for (int k = 0; k < CPL; ++k) any = any || (act[k] != 0u);
  if (!team_any<L>(any)) return;  // no row active at a0: a0 is the minimizer
  // warm start (a nearby solution, e.g. the previous stage's): the iteration
  // below converges to the same unique minimizer from any start
  if (xw) {
#pragma unroll
    for (int i = 0; i < 6; ++i) x[i] = xw[i];
    free_active<CPL, NT>(rw, x, act, s);
  }
  for (int it = 0; it < maxit; ++it) {
    st.newton_it++;
    if (team_leader(L)) st.u_nit++;
#pragma unroll
    for (int k = 0; k < CPL; ++k) {
      const uint32_t cb = contact_bits<NT, L>(act[k]);
      st.u_ncon += rw.first[k] && cb != 0u;
      st.u_nedge += __popc(act[k]);
    }
    // gradient and Hessian of the active set, summed over the team together
    double gh[27];
    double* gp = gh;
    double* H = gh + 6;
#pragma unroll
    for (int i = 0; i < 6; ++i) gp[i] = 0.0;
#pragma unroll
    for (int k = 0; k < CPL; ++k) {
      if (act[k] == 0u) continue;
      // sum_e w_e (J_n + s_e J_t) = (sum w_e) J_n + mu (w0 - w1) J_t1 + mu (w2 - w3) J_t2
      double we[NE];
#pragma unroll
      for (int e = 0; e < NE; ++e) we[e] = ((act[k] >> e) & 1u) ? rw.D[k] * s[k][e] : 0.0;
      const double cn = NT == 2 ? (we[0] + we[1]) + (we[NE - 2] + we[NE - 1]) : we[0] + we[1];
      double ca[NT];
#pragma unroll
      for (int a = 0; a < NT; ++a) ca[a] = rw.mu[k] * (we[2 * a] - we[2 * a + 1]);
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        double g = cn * rw.Jn[k][i];
#pragma unroll
        for (int a = 0; a < NT; ++a) g += ca[a] * rw.Jt[k][a][i];
        gp[i] += g;
      }
    }
    free_hessian_lane<CPL, NT>(rw, act, H);
    team_sum_big<L, LIVE, 27>(gh);
    free_add_mass(m, H);
    double dx[6], Mdx[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) dx[i] = x[i] - a0[i];
    free_Mmul(m, dx, Mdx);
    if (!chol_packed<6>(H)) { st.status |= 4; return; }
    double dl[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) dl[i] = -(Mdx[i] + gp[i]);
    chol_solve_packed<6>(H, dl);
    // a step at rounding level of the iterate: x + dl is the minimizer to
    // working precision (an activity flip there is a rounding artefact)
    double dmax = 0.0, xmax = 1.0;
#pragma unroll
    for (int i = 0; i < 6; ++i) { dmax = fmax(dmax, fabs(dl[i])); xmax = fmax(xmax, fmax(fabs(x[i]), fabs(a0[i]))); }
    if (dmax <= 1e-13 * xmax) {
#pragma unroll
      for (int i = 0; i < 6; ++i) x[i] += dl[i];
      return;
    }
    // directional data of every row
    double t[CPL][4];
    uint32_t act1[CPL];
#pragma unroll
    for (int k = 0; k < CPL; ++k) {
      act1[k] = 0u;
      if (!rw.on[k]) continue;
      const double jn = dot6(rw.Jn[k], dl);
      const double mu = rw.mu[k];
#pragma unroll
      for (int a = 0; a < NT; ++a) {
        const double ja = dot6(rw.Jt[k][a], dl);
        t[k][2 * a] = jn + mu * ja; t[k][2 * a + 1] = jn - mu * ja;
      }
#pragma unroll
      for (int e = 0; e < NE; ++e)
        if (s[k][e] + t[k][e] < 0.0) act1[k] |= 1u << e;
    }
    if (same_active<CPL, L>(act, act1)) {
#pragma unroll
      for (int i = 0; i < 6; ++i) x[i] += dl[i];
      return;
    }
    // exact line search: root of phi'(a) = a C2(a) + C1(a)
    double Mdl[6];
    free_Mmul(m, dl, Mdl);
    double dMd = dot6(dl, Mdl), xMd = dot6(dx, Mdl);
    double lo = 0.0, hi = 1e300, a = 1.0;
    for (int ls = 0; ls < 60; ++ls) {
#pragma unroll
      for (int k = 0; k < CPL; ++k) st.u_ls += rw.on[k] && rw.first[k];
      double c1 = 0.0, c2 = 0.0;
      uint32_t sa[CPL];
#pragma unroll
      for (int k = 0; k < CPL; ++k) {
        sa[k] = 0u;
        if (!rw.on[k]) continue;
#pragma unroll
        for (int e = 0; e < NE; ++e) {
          const bool on = s[k][e] + a * t[k][e] < 0.0;
          sa[k] |= on ? (1u << e) : 0u;
          const double dt = on ? rw.D[k] * t[k][e] : 0.0;
          c2 += dt * t[k][e];
          c1 += dt * s[k][e];
        }
      }
      double cc[2] = {c1, c2};
      team_sum_arr<L, 2>(cc);
      c1 = cc[0] + xMd;
      c2 = cc[1] + dMd;
      double dphi = a * c2 + c1;
      if (dphi > 0.0) hi = a; else lo = a;
      double an = (c2 > 0.0) ? -c1 / c2 : a;
      if (!isfinite(an)) an = a;
      uint32_t sn[CPL];
#pragma unroll
      for (int k = 0; k < CPL; ++k) {
        sn[k] = 0u;
        if (!rw.on[k]) continue;
#pragma unroll
        for (int e = 0; e < NE; ++e)
          if (s[k][e] + an * t[k][e] < 0.0) sn[k] |= 1u << e;
      }
      if (same_active<CPL, L>(sa, sn)) { a = an; break; }
      if (!(an > lo && an < hi)) an = (hi < 1e299) ? 0.5 * (lo + hi) : 2.0 * a;
      a = an;
      if (hi - lo <= 1e-15 * hi) break;  // root at a kink of the piecewise-linear derivative
      if (ls == 59) a = lo > 0.0 ? lo : a;
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) x[i] += a * dl[i];
    free_active<CPL, NT>(rw, x, act, s);
  }
  st.status |= 8;
}

// Forward acceleration of a free-body world at state y = (q[7], v[6]) with
// generalized force tau.
template <int NC, int L>
struct FreePhys {
  static constexpr int NQ = 7, NV = 6, TEAM = L;
  // a team of 8 or 16 lanes for half as many slots holds each contact on a
  // lane and its mirror lane (one tangent direction each); otherwise slot c
  // sits on lane c mod L
  static constexpr int NT = ((L == 8 || L == 16) && 2 * NC == L) ? 1 : 2;
  static constexpr int CPL = NT == 1 ? 1 : (NC + L - 1) / L;
  static constexpr int LIVE = NT == 1 ? L : live_lanes(NC, L);  // lanes that hold slots
  using Model = FreeModel;

  DMX_DEV static void frame(const double* q, V3* p, M3* R, Q4* qh, double* inv) {
    *p = mk3(q[0], q[1], q[2]);
    *qh = qnormalize(mkq(q[3], q[4], q[5], q[6]), inv);
    *R = quat2mat(*qh);
  }

  DMX_DEV static void a0_of(const Model& m, const double* v, const double* tau, double* a0) {
    V3 w = mk3(v[3], v[4], v[5]);
    V3 Iw = mk3(m.I[0] * w.x + m.I[1] * w.y + m.I[2] * w.z, m.I[3] * w.x + m.I[4] * w.y + m.I[5] * w.z,
                m.I[6] * w.x + m.I[7] * w.y + m.I[8] * w.z);
    V3 gy = cross(w, Iw);
    double fa[3] = {tau[3] - gy.x, tau[4] - gy.y, tau[5] - gy.z};
#pragma unroll
    for (int i = 0; i < 3; ++i) a0[i] = tau[i] * m.imass + m.grav[i];
#pragma unroll
    for (int i = 0; i < 3; ++i) a0[3 + i] = m.Iinv[3 * i] * fa[0] + m.Iinv[3 * i + 1] * fa[1] + m.Iinv[3 * i + 2] * fa[2];
  }

  DMX_DEV static void acc(const Model& m, const double* y, const double* tau, bool cfd, double beta, int maxit,
                          const double* xw, double* a, Stat& st) {
    V3 p; M3 R; Q4 qh; double inv;
    frame(y, &p, &R, &qh, &inv);
    const double* v = y + NQ;
    double a0[6];
    a0_of(m, v, tau, a0);
    FreeRows<CPL, NT> rw;
    free_rows<CPL, L, NT>(m, p, R, v, cfd, beta, rw);
    if (team_leader(L)) st.u_rhs++;
#pragma unroll
    for (int k = 0; k < CPL; ++k) st.u_con += rw.on[k] && rw.first[k];
    free_newton<CPL, L, LIVE, NT>(m, rw, a0, xw, a, maxit, st);
  }

  // Cotangent of the acceleration map.  x* solves H x* = (tau - c) + sum_A
  // D_e a_ref_e J_e^T at its active set A (the same set the forward solve
  // ended with), so with lam = H^-1 abar: tau_bar = lam, c_bar = -lam,
  // D_bar_e = (J_e lam)(a_ref_e - J_e x*), a_ref_bar_e = D_e (J_e lam),
  // J_bar_e = f_e lam - D_e (J_e lam) x*; then back through a_ref, d(r), the
  // contact geometry and the body frame to (q, v).  For the CFD field x* is
  // solved here (its rows differ from the forward's).
  // hbar (optional, [kParams]): += the cotangents of the model parameters:
  // the box geom's half sizes (the contact vertices are l + gR (s * h)), then
  // the friction coefficient, the solref time constant and damping ratio, each
  // as one value shared by every contact pair (a common shift of all pairs),
  // the body's mass, and the five solimp parameters (shared likewise)
  DMX_DEV static void acc_vjp(const Model& m, const double* y, const double* tau, const double* xs_in,
                              const double* abar, bool cfd, double beta, int maxit, double* ybar, double* taubar,
                              Stat& st, double* hbar = nullptr) {
    V3 p; M3 R; Q4 qh; double inv;
    frame(y, &p, &R, &qh, &inv);
    const double* v = y + NQ;
    FreeRows<CPL, NT> rw;
    free_rows<CPL, L, NT>(m, p, R, v, cfd, beta, rw);
    double xs[6];
    if (cfd) {
      double a0[6];
      a0_of(m, v, tau, a0);
      free_newton<CPL, L, LIVE, NT>(m, rw, a0, nullptr, xs, maxit, st);
    } else {
#pragma unroll
      for (int i = 0; i < 6; ++i) xs[i] = xs_in[i];
    }
    uint32_t act[CPL];
    double s[CPL][4];
    free_active<CPL, NT>(rw, xs, act, s);
    if (team_leader(L)) st.u_vjp++;
#pragma unroll
    for (int k = 0; k < CPL; ++k) { st.u_vcon += rw.on[k] && rw.first[k]; st.u_vedge += __popc(act[k]); }
    double H[21];
    free_hessian<CPL, L, LIVE, NT>(m, rw, act, H);
    chol_packed<6>(H);
    double lam[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) lam[i] = abar[i];
    chol_solve_packed<6>(H, lam);
    // per-lane partial cotangents: p, R, v
    double acc_[18];  // pb[3], Rb[9], vb[6]
#pragma unroll
    for (int i = 0; i < 18; ++i) acc_[i] = 0.0;
    double hb_[kParams];
#pragma unroll
    for (int i = 0; i < kParams; ++i) hb_[i] = 0.0;
    const int tl = threadIdx.x & (L - 1);
    (void)tl;
#pragma unroll
    for (int k = 0; k < CPL; ++k) {
      if (!rw.on[k] || act[k] == 0u) continue;
      const PairF& pr = slot_pair(rw.slot[k]);
      const double mu = rw.mu[k], D = rw.D[k];
      const double* Jn = rw.Jn[k];
      double rbar = 0.0;
      double ddr;
      double dimp = impedance(pr, rw.r[k], &ddr);
      double dD = ddr / (pr.ahat * (1.0 - dimp) * (1.0 - dimp));
      double kk = dimp * pr.kscale;
      double dpt;  // d pterm / dr
      double ptd;  // d pterm / d(impedance) / kscale
      if (cfd) {
        double dsp;
        double sp = softplus(-rw.r[k], beta, &dsp);
        dpt = pr.kscale * ddr * sp - kk * dsp;
        ptd = sp;
      } else {
        dpt = -(pr.kscale * ddr * rw.r[k] + kk);
        ptd = -rw.r[k];
      }
      // Per edge e (J_e = J_n + s_e J_t(e), force f_e = D (aref_e - J_e x)):
      // J_e_bar = f_e lam - arb_e (x + bcoef v) with arb_e = D J_e lam, and
      // v_bar -= bcoef arb_e J_e.  Summed over the lane's edges these become
      // combinations of the frame rows (inactive edges weigh 0).
      constexpr int NE = 2 * NT;
      const double ln = dot6(Jn, lam), xn = dot6(Jn, xs);
      double la[NT], xa[NT];
#pragma unroll
      for (int a = 0; a < NT; ++a) { la[a] = dot6(rw.Jt[k][a], lam); xa[a] = dot6(rw.Jt[k][a], xs); }
      double fe[NE], ae[NE];
      double dsum = 0.0;  // sum of the edges' D cotangents
#pragma unroll
      for (int e = 0; e < NE; ++e) {
        const bool on = (act[k] >> e) & 1u;
        const double sg = (e & 1) ? -mu : mu;
        const double sl = ln + sg * la[e >> 1], sx = xn + sg * xa[e >> 1];
        const double De = on ? D : 0.0;
        const double gap = rw.aref[k][e] - sx;
        fe[e] = De * gap;
        ae[e] = De * sl;
        const double Dbar = on ? sl * gap : 0.0;
        rbar += ae[e] * dpt + Dbar * dD;
        dsum += Dbar;
      }
      const double Fn = NT == 2 ? (fe[0] + fe[1]) + (fe[NE - 2] + fe[NE - 1]) : fe[0] + fe[1];
      const double An = NT == 2 ? (ae[0] + ae[1]) + (ae[NE - 2] + ae[NE - 1]) : ae[0] + ae[1];
      double Fa[NT], Aa[NT];
#pragma unroll
      for (int a = 0; a < NT; ++a) { Fa[a] = mu * (fe[2 * a] - fe[2 * a + 1]); Aa[a] = mu * (ae[2 * a] - ae[2 * a + 1]); }
      if (hbar) {
        // friction: J_e = J_n +- mu J_t (in the force and in a_ref's damping
        // term) and D = d / (Ahat (1 - d)) with Ahat = (1 + mu^2) w; solref:
        // a_ref = -bcoef J_e v + kscale (d(r) times the position term), with
        // bcoef = 2 / (dw t_c) and kscale = 1 / (dw^2 t_c^2 dr^2)
        const double vn = dot6(Jn, v);
        double mub = dsum * (-2.0 * mu * D / (1.0 + mu * mu)), bb = 0.0;
#pragma unroll
        for (int a = 0; a < NT; ++a) {
          const double vt = dot6(rw.Jt[k][a], v);
          const double fd = fe[2 * a] - fe[2 * a + 1], ad = ae[2 * a] - ae[2 * a + 1];
          mub += fd * la[a] - ad * (xa[a] + pr.bcoef * vt);
          bb -= (ae[2 * a] + ae[2 * a + 1]) * vn + mu * ad * vt;
        }
        const double kb = An * dimp * ptd;
        const double sb = pr.bcoef * bb + 2.0 * pr.kscale * kb;  // b and k go as 1/t_c, 1/t_c^2 (and dwidth)
        hb_[3] += mub;
        hb_[4] -= sb / pr.solref[0];
        hb_[5] -= 2.0 * pr.kscale * kb / pr.solref[1];
        // solimp: through d(r) (in D and the position term) and, for dwidth,
        // through b and k as well
        const double dbar = dsum / (pr.ahat * (1.0 - dimp) * (1.0 - dimp)) + An * pr.kscale * ptd;
        double gs[5];
        impedance_solimp_grad(pr, rw.r[k], gs);
#pragma unroll
        for (int i = 0; i < 5; ++i) hb_[7 + i] += dbar * gs[i];
        hb_[8] -= sb / pr.si[1];
      }
      double Jb[1 + NT][6];  // cotangents of J_n and the lane's tangent rows
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        const double z = xs[i] + pr.bcoef * v[i];
        Jb[0][i] = Fn * lam[i] - An * z;
        double vt = An * Jn[i];
#pragma unroll
        for (int a = 0; a < NT; ++a) {
          Jb[1 + a][i] = Fa[a] * lam[i] - Aa[a] * z;
          vt += Aa[a] * rw.Jt[k][a][i];
        }
        acc_[12 + i] -= pr.bcoef * vt;
      }
      // J_u = [u, R^T (d x u)]: angular part back to d and R
      V3 lc, ce, P;
      double r;
      slot_geom(m, rw.slot[k], p, R, &lc, &ce, &r, &P);
      V3 d = P - p;
      V3 db = mk3(0, 0, 0);
#pragma unroll
      for (int a = 0; a < 1 + NT; ++a) {
        const V3 u = a == 0 ? ld3(pr.n) : ((NT == 2 ? a == 2 : rw.half[k] == 1) ? ld3(pr.t2) : ld3(pr.t1));
        const double* jb = Jb[a];
        V3 wb = mk3(jb[3], jb[4], jb[5]);
        V3 z = cross(d, u);
        V3 zb = mul(R, wb);
        // R_bar += z wb^T
        M3 Rb;
#pragma unroll
        for (int i = 0; i < 9; ++i) Rb.a[i] = 0.0;
        outer_add(Rb, z, wb);
#pragma unroll
        for (int i = 0; i < 9; ++i) acc_[3 + i] += Rb.a[i];
        db += cross(u, zb);
      }
      // d = P - p; P = ce - (rad + r/2) n; r = n.(ce - p0) - rad (sphere,
      // capsule end) or r = r(g_k, g_deepest) with g = n.(ce - p0) (box
      // vertex); ce = p + R lc
      V3 n = ld3(pr.n);
      V3 Pb = db;
      V3 pb = mk3(-db.x, -db.y, -db.z);
      rbar += -0.5 * dot(n, Pb);
      double gbar = rbar;
      M3 Rb2;
#pragma unroll
      for (int i = 0; i < 9; ++i) Rb2.a[i] = 0.0;
      if (pr.gtype == 3) {
        const BoxSlot bs = box_plane_slot(pr, p, R, slot_sub(rw.slot[k]));
        gbar = rbar * bs.drdg;
        const V3 cm = (rbar * bs.drdgmax) * n;  // the deepest vertex, through the skin threshold
        pb += cm;
        outer_add(Rb2, cm, box_vertex(pr, bs.kmax));
        if (hbar) {  // vertex k: d/dh of gR (s * h) in the body frame, s the vertex's signs
          const V3 ceb0 = Pb + gbar * n;
          const double* g = pr.gR;
          const int kv[2] = {bs.k, bs.kmax};
          const V3 wb[2] = {mulT(R, ceb0), mulT(R, cm)};
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            const V3 lb = mk3(g[0] * wb[q].x + g[3] * wb[q].y + g[6] * wb[q].z,
                              g[1] * wb[q].x + g[4] * wb[q].y + g[7] * wb[q].z,
                              g[2] * wb[q].x + g[5] * wb[q].y + g[8] * wb[q].z);
            hb_[0] += (kv[q] & 1) ? lb.x : -lb.x;
            hb_[1] += (kv[q] & 2) ? lb.y : -lb.y;
            hb_[2] += (kv[q] & 4) ? lb.z : -lb.z;
          }
        }
      }
      V3 ceb = Pb + gbar * n;
      pb += ceb;
      outer_add(Rb2, ceb, lc);
      acc_[0] += pb.x; acc_[1] += pb.y; acc_[2] += pb.z;
#pragma unroll
      for (int i = 0; i < 9; ++i) acc_[3 + i] += Rb2.a[i];
    }
    team_sum_big<L, LIVE, 18>(acc_);
    if (hbar) {
      team_sum_big<L, LIVE, kParams>(hb_);
#pragma unroll
      for (int i = 0; i < kParams; ++i) hbar[i] += hb_[i];
      // mass: the inertia of a uniform solid, the bias (-m g, w x I w) and D
      // (through Ahat = (1 + mu^2) / m) all scale with m, so H x* = rhs keeps
      // x* = H^-1 tau + (a part free of m) and m_bar = -lam . tau / m
      hbar[6] -= dot6(lam, tau) * m.imass;
    }
    // bias c = (-m g, w x I w) with c_bar = -lam
    V3 w = mk3(v[3], v[4], v[5]);
    V3 Iw = mk3(m.I[0] * w.x + m.I[1] * w.y + m.I[2] * w.z, m.I[3] * w.x + m.I[4] * w.y + m.I[5] * w.z,
                m.I[6] * w.x + m.I[7] * w.y + m.I[8] * w.z);
    V3 cb = mk3(-lam[3], -lam[4], -lam[5]);
    V3 t1 = cross(Iw, cb);
    V3 t2 = cross(cb, w);
    V3 It2 = mk3(m.I[0] * t2.x + m.I[1] * t2.y + m.I[2] * t2.z, m.I[3] * t2.x + m.I[4] * t2.y + m.I[5] * t2.z,
                 m.I[6] * t2.x + m.I[7] * t2.y + m.I[8] * t2.z);
    M3 Rb;
#pragma unroll
    for (int i = 0; i < 9; ++i) Rb.a[i] = acc_[3 + i];
    Q4 qhb = quat2mat_vjp(qh, Rb);
    Q4 qb = qnormalize_vjp(qh, inv, qhb);
    ybar[0] = acc_[0]; ybar[1] = acc_[1]; ybar[2] = acc_[2];
    ybar[3] = qb.w; ybar[4] = qb.x; ybar[5] = qb.y; ybar[6] = qb.z;
#pragma unroll
    for (int i = 0; i < 6; ++i) ybar[NQ + i] = acc_[12 + i];
    ybar[NQ + 3] += t1.x + It2.x;
    ybar[NQ + 4] += t1.y + It2.y;
    ybar[NQ + 5] += t1.z + It2.z;
#pragma unroll
    for (int i = 0; i < 6; ++i) taubar[i] = lam[i];
  }

  // q (+) dq for the free joint: position += dq_lin; quat <- normalize(quat *
  // exp(dq_ang / 2)) (exact integration of the body-frame rotation).
  DMX_DEV static void qplus(const double* q, const double* dq, double* out) {
    out[0] = q[0] + dq[0]; out[1] = q[1] + dq[1]; out[2] = q[2] + dq[2];
    Q4 e = qexp_half(mk3(dq[3], dq[4], dq[5]), nullptr, nullptr, nullptr, nullptr);
    Q4 w = qmul(mkq(q[3], q[4], q[5], q[6]), e);
    Q4 r = qnormalize(w, nullptr);
    out[3] = r.w; out[4] = r.x; out[5] = r.y; out[6] = r.z;
  }
  // (+) that also keeps the half-angle exponential's coefficients and their
  // derivatives, for the VJP at the same increment
  struct QPlusKeep { double c, s, dc, ds; };
  DMX_DEV static void qplus_keep(const double* q, const double* dq, double* out, QPlusKeep* k) {
    out[0] = q[0] + dq[0]; out[1] = q[1] + dq[1]; out[2] = q[2] + dq[2];
    Q4 e = qexp_half(mk3(dq[3], dq[4], dq[5]), &k->c, &k->s, &k->dc, &k->ds);
    Q4 w = qmul(mkq(q[3], q[4], q[5], q[6]), e);
    Q4 r = qnormalize(w, nullptr);
    out[3] = r.w; out[4] = r.x; out[5] = r.y; out[6] = r.z;
  }
  // qbar += d out / d q ^T ob ; dqb = d out / d dq ^T ob
  DMX_DEV static void qplus_vjp(const double* q, const double* dq, const double* ob, double* qbar, double* dqb,
                                const QPlusKeep* kept = nullptr) {
    qbar[0] += ob[0]; qbar[1] += ob[1]; qbar[2] += ob[2];
    dqb[0] = ob[0]; dqb[1] = ob[1]; dqb[2] = ob[2];
    V3 th = mk3(dq[3], dq[4], dq[5]);
    double c, s, dc, ds;
    Q4 e;
    if (kept) {
      c = kept->c; s = kept->s; dc = kept->dc; ds = kept->ds;
      e = mkq(c, s * th.x, s * th.y, s * th.z);
    } else {
      e = qexp_half(th, &c, &s, &dc, &ds);
    }
    Q4 q4 = mkq(q[3], q[4], q[5], q[6]);
    Q4 w = qmul(q4, e);
    double inv;
    Q4 r = qnormalize(w, &inv);
    Q4 wb = qnormalize_vjp(r, inv, mkq(ob[3], ob[4], ob[5], ob[6]));
    Q4 qb = qmul(wb, qconj(e));
    Q4 eb = qmul(qconj(q4), wb);
    qbar[3] += qb.w; qbar[4] += qb.x; qbar[5] += qb.y; qbar[6] += qb.z;
    double tv = eb.x * th.x + eb.y * th.y + eb.z * th.z;
    double g = 2.0 * (dc * eb.w + ds * tv);
    dqb[3] = s * eb.x + g * th.x;
    dqb[4] = s * eb.y + g * th.y;
    dqb[5] = s * eb.z + g * th.z;
  }

  // Cotangent of the raw coordinate rates dq/dt = (v_lin, (1/2) q (x) (0, w))
  // at x = (q, v), for the adjoint ODE in raw coordinates: xbar[NQ + d] +=
  // (d(dq/dt)/dv)^T lq and xbar[0..NQ) += (d(dq/dt)/dq)^T lq.  Right
  // multiplication by (0, w) has the transpose right multiplication by
  // (0, -w); left multiplication by q has the transpose left multiplication by
  // conj(q).
  DMX_DEV static void kin_vjp(const double* x, const double* lq, double* xbar) {
#pragma unroll
    for (int i = 0; i < 3; ++i) xbar[NQ + i] += lq[i];
    const Q4 q = mkq(x[3], x[4], x[5], x[6]);
    const Q4 l = mkq(lq[3], lq[4], lq[5], lq[6]);
    const Q4 qb = qmul(l, mkq(0.0, -x[NQ + 3], -x[NQ + 4], -x[NQ + 5]));
    const Q4 wb = qmul(qconj(q), l);
    xbar[3] += 0.5 * qb.w; xbar[4] += 0.5 * qb.x; xbar[5] += 0.5 * qb.y; xbar[6] += 0.5 * qb.z;
    xbar[NQ + 3] += 0.5 * wb.x; xbar[NQ + 4] += 0.5 * wb.y; xbar[NQ + 5] += 0.5 * wb.z;
  }
  // the quaternion part of a raw-coordinate gradient projected onto the
  // tangent space of the unit sphere at q0 (the radial part is not a
  // direction of the state space)
  DMX_DEV static void tangent_project(const double* q0, double* g) {
    const double nn = q0[3] * q0[3] + q0[4] * q0[4] + q0[5] * q0[5] + q0[6] * q0[6];
    const double dp = g[3] * q0[3] + g[4] * q0[4] + g[5] * q0[5] + g[6] * q0[6];
#pragma unroll
    for (int i = 3; i < 7; ++i) g[i] -= dp / nn * q0[i];
  }

  // coordinates of q integrated as plain sums (positions); the rest are quaternion components
  DMX_DEV static bool q_is_linear(int i) { return i < 3; }
  DMX_DEV static int q_dof(int i) { return i; }
};

}  // namespace dmx
