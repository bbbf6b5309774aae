// Articulated worlds: a tree of bodies on hinge and slide joints (nq = nv =
// number of joints) with sphere/capsule geoms touching world planes.
//
// Forward (Sec. 2, eq. EOM; Sec. 2.1): forward kinematics along the tree,
// joint-space inertia M = sum_b (m Jp^T Jp + Jr^T I_w Jr) and bias
// c = sum_b (Jp^T m (a0_b - g) + Jr^T (I_w al0_b + w_b x I_w w_b)) from the
// body Jacobians and the velocity-product accelerations, pyramidal contact rows
// and the exact Newton solve of the primal problem.
//
// VJP: x* solves H x* = (tau - c) + sum_A D a_ref J^T; with lam = H^-1 abar the
// cotangent of the state is -d/dY [ lam^T ID(q, v, x*) - sum_A (J_e lam) f_e ],
// ID(q, v, qdd) = M qdd + c the inverse dynamics.  The ID term is
// differentiated by a reverse sweep through the joint recursion (body motion
// under velocities v, accelerations x* and velocities lam), the contact term
// through the point Jacobians and contact geometry, both into a reverse sweep
// of the forward kinematics.
#pragma once
#include "dmx_free.hpp"

namespace dmx {

constexpr int kTreeBodies = 8;
constexpr int kTreeJoints = 8;

struct TreeModel {
  int nb, nj, np, nc, nu;
  int bparent[kTreeBodies], bj0[kTreeBodies], bjn[kTreeBodies];
  unsigned banc[kTreeBodies];  // bit d set if joint d moves body b (joints of b and of its ancestors)
  double bpos[kTreeBodies][3], bR[kTreeBodies][9];
  double bmass[kTreeBodies], bI[kTreeBodies][9];
  int jtype[kTreeJoints];
  double jaxis[kTreeJoints][3], jpos[kTreeJoints][3];
  int cpair[kMaxSlots], csub[kMaxSlots];
  int pbody[kMaxPairs];
  int ctrl[8];
  double grav[3];
  PairF pair[kMaxPairs];
};

// --------------------------------------------------------------- small helpers
DMX_DEV M3 mmul(const M3& a, const M3& b) {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) r.a[i * 3 + j] = a.a[i * 3] * b.a[j] + a.a[i * 3 + 1] * b.a[3 + j] + a.a[i * 3 + 2] * b.a[6 + j];
  return r;
}
DMX_DEV M3 mmulT(const M3& a, const M3& b) {  // a b^T
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) r.a[i * 3 + j] = a.a[i * 3] * b.a[j * 3] + a.a[i * 3 + 1] * b.a[j * 3 + 1] + a.a[i * 3 + 2] * b.a[j * 3 + 2];
  return r;
}
DMX_DEV M3 ldm(const double* p) { M3 r; for (int i = 0; i < 9; ++i) r.a[i] = p[i]; return r; }
DMX_DEV void stm(double* p, const M3& m) { for (int i = 0; i < 9; ++i) p[i] = m.a[i]; }
DMX_DEV void st3(double* p, V3 v) { p[0] = v.x; p[1] = v.y; p[2] = v.z; }
DMX_DEV V3 neg(V3 a) { return mk3(-a.x, -a.y, -a.z); }
// rotation by angle th about a unit axis k (body frame)
DMX_DEV M3 axis_rot(V3 k, double th, double* c_out, double* s_out) {
  double c = cos(th), s = sin(th), t = 1.0 - c;
  M3 m;
  m.a[0] = t * k.x * k.x + c;       m.a[1] = t * k.x * k.y - s * k.z; m.a[2] = t * k.x * k.z + s * k.y;
  m.a[3] = t * k.x * k.y + s * k.z; m.a[4] = t * k.y * k.y + c;       m.a[5] = t * k.y * k.z - s * k.x;
  m.a[6] = t * k.x * k.z - s * k.y; m.a[7] = t * k.y * k.z + s * k.x; m.a[8] = t * k.z * k.z + c;
  if (c_out) { *c_out = c; *s_out = s; }
  return m;
}
// d/dth of axis_rot
DMX_DEV M3 axis_rot_d(V3 k, double c, double s) {
  M3 m;
  m.a[0] = s * k.x * k.x - s;       m.a[1] = s * k.x * k.y - c * k.z; m.a[2] = s * k.x * k.z + c * k.y;
  m.a[3] = s * k.x * k.y + c * k.z; m.a[4] = s * k.y * k.y - s;       m.a[5] = s * k.y * k.z - c * k.x;
  m.a[6] = s * k.x * k.z - c * k.y; m.a[7] = s * k.y * k.z + c * k.x; m.a[8] = s * k.z * k.z - s;
  return m;
}

// per-world workspace in LDS (one copy per team; every lane writes the same
// values), sized by the model's body count NB and joint count NV
template <int NV, int NB>
struct TreeWs {
  double p[NB][3], R[NB][9];
  double w[NB][3], vel[NB][3], al[NB][3], ac[NB][3];
  double kap[NB][3], ell[NB][3];
  double ax[NV][3], an[NV][3];
  // reverse-sweep storage: frame and motion before each joint, frame after
  double jp_in[NV][3], jR_in[NV][9], jp_out[NV][3], jm_in[NV][18];
  // cotangent accumulators
  double bpb[NB][3], bRb[NB][9], bmb[NB][18];
  double jab[NV][3], jobar[NV][3];
};

// Forward kinematics with body motion.  qd: joint velocities; qdd: joint
// accelerations (null = 0); lam: a second velocity field (null = skip).
// Stores body frames/motion, joint axes/anchors, and (if store_rev) the
// per-joint frame and motion before each joint.
template <int NV, int NB>
DMX_DEV void tree_kin(const TreeModel& m, const double* q, const double* qd, const double* qdd, const double* lam,
                      TreeWs<NV, NB>& ws, bool store_rev) {
  for (int b = 0; b < m.nb; ++b) {
    const int pa = m.bparent[b];
    V3 pp = mk3(0, 0, 0), wp = pp, vp = pp, ap = pp, cp = pp, kp = pp, lp = pp;
    M3 Rp;
    for (int i = 0; i < 9; ++i) Rp.a[i] = (i % 4 == 0) ? 1.0 : 0.0;
    if (pa >= 0) {
      pp = ld3(ws.p[pa]); Rp = ldm(ws.R[pa]); wp = ld3(ws.w[pa]); vp = ld3(ws.vel[pa]);
      ap = ld3(ws.al[pa]); cp = ld3(ws.ac[pa]); kp = ld3(ws.kap[pa]); lp = ld3(ws.ell[pa]);
    }
    V3 p = pp + mul(Rp, ld3(m.bpos[b]));
    M3 R = mmul(Rp, ldm(m.bR[b]));
    V3 r = p - pp;
    V3 w = wp, v = vp + cross(wp, r), al = ap, ac = cp + cross(ap, r) + cross(wp, cross(wp, r));
    V3 kap = kp, ell = lp + cross(kp, r);
    for (int j = m.bj0[b]; j < m.bj0[b] + m.bjn[b]; ++j) {
      const V3 jax = ld3(m.jaxis[j]), jps = ld3(m.jpos[j]);
      const double qj = q[j], qdj = qd[j], qddj = qdd ? qdd[j] : 0.0, lj = lam ? lam[j] : 0.0;
      if (store_rev) {
        st3(ws.jp_in[j], p); stm(ws.jR_in[j], R);
        double* mm = ws.jm_in[j];
        st3(mm, w); st3(mm + 3, v); st3(mm + 6, al); st3(mm + 9, ac); st3(mm + 12, kap); st3(mm + 15, ell);
      }
      const V3 a = mul(R, jax);
      const V3 o = p + mul(R, jps);
      st3(ws.ax[j], a); st3(ws.an[j], o);
      if (m.jtype[j] == 1) {  // hinge about its anchor
        const V3 r1 = o - p;
        const V3 vo = v + cross(w, r1), ao = ac + cross(al, r1) + cross(w, cross(w, r1)), lo = ell + cross(kap, r1);
        const V3 wa = qdj * a;
        const V3 w2 = w + wa, al2 = al + cross(w, wa) + qddj * a, k2 = kap + lj * a;
        R = mmul(R, axis_rot(jax, qj, nullptr, nullptr));
        const V3 p2 = o - mul(R, jps);
        const V3 r2 = p2 - o;
        v = vo + cross(w2, r2);
        ac = ao + cross(al2, r2) + cross(w2, cross(w2, r2));
        ell = lo + cross(k2, r2);
        w = w2; al = al2; kap = k2; p = p2;
      } else {  // slide
        const V3 rr = qj * a;
        const V3 wa = qdj * a;
        ac = ac + cross(al, rr) + cross(w, cross(w, rr)) + 2.0 * cross(w, wa) + qddj * a;
        v = v + cross(w, rr) + wa;
        ell = ell + cross(kap, rr) + lj * a;
        p = p + rr;
      }
      if (store_rev) st3(ws.jp_out[j], p);
    }
    st3(ws.p[b], p); stm(ws.R[b], R); st3(ws.w[b], w); st3(ws.vel[b], v);
    st3(ws.al[b], al); st3(ws.ac[b], ac); st3(ws.kap[b], kap); st3(ws.ell[b], ell);
  }
}

// Jacobian columns of a point P attached to body b: Jp[3][NV], Jr[3][NV] (Jr may be null)
template <int NV, int NB>
DMX_DEV void tree_point_jac(const TreeModel& m, const TreeWs<NV, NB>& ws, int b, V3 P, double (*Jp)[NV], double (*Jr)[NV]) {
  const unsigned anc = m.banc[b];
#pragma unroll
  for (int d = 0; d < NV; ++d) {
    V3 cp = mk3(0, 0, 0), cr = mk3(0, 0, 0);
    if ((anc >> d) & 1u) {
      const V3 a = ld3(ws.ax[d]);
      if (m.jtype[d] == 1) { cp = cross(a, P - ld3(ws.an[d])); cr = a; }
      else cp = a;
    }
    Jp[0][d] = cp.x; Jp[1][d] = cp.y; Jp[2][d] = cp.z;
    if (Jr) { Jr[0][d] = cr.x; Jr[1][d] = cr.y; Jr[2][d] = cr.z; }
  }
}

// M (dense, row-major) and bias c from the body Jacobians.
template <int NV, int NB>
DMX_DEV void tree_mass_bias(const TreeModel& m, const TreeWs<NV, NB>& ws, double* M, double* c) {
  // M: packed lower triangle, M[tri(i, j)] for i >= j
#pragma unroll
  for (int i = 0; i < NV * (NV + 1) / 2; ++i) M[i] = 0.0;
#pragma unroll
  for (int i = 0; i < NV; ++i) c[i] = 0.0;
  for (int b = 0; b < m.nb; ++b) {
    double Jp[3][NV], Jr[3][NV];
    tree_point_jac<NV, NB>(m, ws, b, ld3(ws.p[b]), Jp, Jr);
    const M3 R = ldm(ws.R[b]);
    const M3 Iw = mmulT(mmul(R, ldm(m.bI[b])), R);
    const double mb = m.bmass[b];
    const V3 w = ld3(ws.w[b]);
    const V3 f = mb * (ld3(ws.ac[b]) - ld3(m.grav));
    const V3 tq = mul(Iw, ld3(ws.al[b])) + cross(w, mul(Iw, w));
    double IJ[3][NV];
#pragma unroll
    for (int d = 0; d < NV; ++d) {
      const V3 col = mul(Iw, mk3(Jr[0][d], Jr[1][d], Jr[2][d]));
      IJ[0][d] = col.x; IJ[1][d] = col.y; IJ[2][d] = col.z;
      c[d] += Jp[0][d] * f.x + Jp[1][d] * f.y + Jp[2][d] * f.z + Jr[0][d] * tq.x + Jr[1][d] * tq.y + Jr[2][d] * tq.z;
    }
#pragma unroll
    for (int i = 0; i < NV; ++i)
#pragma unroll
      for (int j = 0; j <= i; ++j) {
        const double s = mb * (Jp[0][i] * Jp[0][j] + Jp[1][i] * Jp[1][j] + Jp[2][i] * Jp[2][j]) +
                         Jr[0][i] * IJ[0][j] + Jr[1][i] * IJ[1][j] + Jr[2][i] * IJ[2][j];
        M[tri(i, j)] += s;
      }
  }
}

// y = M x for a packed symmetric M
template <int NV>
DMX_DEV void symv_packed(const double* M, const double* x, double* y) {
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < NV; ++j) s += M[i >= j ? tri(i, j) : tri(j, i)] * x[j];
    y[i] = s;
  }
}

// Rows of a lane's contact slots (the free-body rows' layout): NTG = 2, both
// tangent directions and four pyramid edges per slot; NTG = 1, a contact on
// two lanes l and L-1-l, each with one tangent direction and its two edges.
template <int NV, int CPL, int NTG>
struct TreeRows {
  bool on[CPL];
  bool first[CPL];  // the lane that counts the contact
  int slot[CPL], body[CPL], half[CPL];
  double r[CPL], mu[CPL], D[CPL];
  double Jn[CPL][NV], Jt[CPL][NTG][NV];
  double aref[CPL][2 * NTG];
};

template <int NV>
DMX_DEV double dotn(const double* a, const double* b) {
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < NV; ++i) s += a[i] * b[i];
  return s;
}

DMX_DEV void tree_slot_geom(const TreeModel& m, int c, V3 pb, const M3& Rb, V3* lc, double* r, V3* P) {
  const PairF& pr = slot_pair(c);
  V3 l = ld3(pr.l);
  if (pr.gtype == 2) l = (slot_sub(c) == 0) ? l + ld3(pr.ax) : l - ld3(pr.ax);
  const V3 ce = pb + mul(Rb, l);
  const V3 n = ld3(pr.n);
  const double rr = dot(n, ce - ld3(pr.p0)) - pr.rad;
  *lc = l;
  *r = rr;
  *P = ce - (pr.rad + 0.5 * rr) * n;
}

template <int NV, int NB, int CPL, int L, int NTG>
DMX_DEV void tree_rows(const TreeModel& m, const TreeWs<NV, NB>& ws, const double* v, bool cfd, double beta,
                       TreeRows<NV, CPL, NTG>& rw) {
  const int tl = threadIdx.x & (L - 1);
#pragma unroll
  for (int k = 0; k < CPL; ++k) {
    // NTG = 2: slot tl + k L; NTG = 1: slot tl on the first half of the
    // team, L - 1 - tl on the second (a lane and its mirror share a slot)
    const int h = NTG == 2 ? 0 : tl / (L / 2);
    const int c = NTG == 2 ? tl + k * L : (h ? L - 1 - tl : tl);
    rw.slot[k] = c;
    rw.half[k] = h;
    rw.first[k] = h == 0;
    rw.on[k] = false;
    if (c >= m.nc) continue;
    const PairF& pr = slot_pair(c);
    const int b = m.pbody[lds_slots()[c]];
    rw.body[k] = b;
    V3 lc, P;
    double r;
    tree_slot_geom(m, c, ld3(ws.p[b]), ldm(ws.R[b]), &lc, &r, &P);
    rw.r[k] = r;
    const bool on = cfd ? (r < pr.cf[2]) : (r < 0.0);
    rw.on[k] = on;
    if (!on) continue;
    double Jp[3][NV];
    tree_point_jac<NV, NB>(m, ws, b, P, Jp, nullptr);
    const V3 n = ld3(pr.n);
#pragma unroll
    for (int d = 0; d < NV; ++d) rw.Jn[k][d] = n.x * Jp[0][d] + n.y * Jp[1][d] + n.z * Jp[2][d];
#pragma unroll
    for (int a = 0; a < NTG; ++a) {
      const V3 t = (NTG == 2 ? a == 1 : h == 1) ? ld3(pr.t2) : ld3(pr.t1);
#pragma unroll
      for (int d = 0; d < NV; ++d) rw.Jt[k][a][d] = t.x * Jp[0][d] + t.y * Jp[1][d] + t.z * Jp[2][d];
    }
    double ddr;
    const double dimp = impedance(pr, r, &ddr);
    const double kk = dimp * pr.kscale;
    rw.mu[k] = pr.mu;
    rw.D[k] = dimp / (pr.ahat * (1.0 - dimp));
    double pterm;
    if (cfd) { double dsp; pterm = kk * softplus(-r, beta, &dsp); }
    else pterm = -kk * r;
    const double jnv = dotn<NV>(rw.Jn[k], v);
#pragma unroll
    for (int a = 0; a < NTG; ++a) {
      const double jtv = dotn<NV>(rw.Jt[k][a], v);
      rw.aref[k][2 * a] = -pr.bcoef * (jnv + pr.mu * jtv) + pterm;
      rw.aref[k][2 * a + 1] = -pr.bcoef * (jnv - pr.mu * jtv) + pterm;
    }
  }
}

template <int NV, int CPL, int NTG>
DMX_DEV void tree_active(const TreeRows<NV, CPL, NTG>& rw, const double* x, uint32_t* act, double (*s)[4]) {
#pragma unroll
  for (int k = 0; k < CPL; ++k) {
    act[k] = 0u;
    if (!rw.on[k]) continue;
    const double jn = dotn<NV>(rw.Jn[k], x);
    const double mu = rw.mu[k];
#pragma unroll
    for (int a = 0; a < NTG; ++a) {
      const double ja = dotn<NV>(rw.Jt[k][a], x);
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
// L - 1 - l (NTG = 1 splits a contact over the two).
template <int NTG, int L>
DMX_DEV uint32_t tree_contact_bits(uint32_t act) {
  if constexpr (NTG == 2) {
    return act;
  } else {
    static_assert(L == 8 || L == 16, "mirror exchange within a row of 16");
    return act | (uint32_t)__builtin_amdgcn_mov_dpp((int)act, L == 8 ? 0x141 : 0x140, 0xF, 0xF, true);
  }
}

// H = M + sum over active edges of D J_e J_e^T (packed, team-summed;
// inactive edges enter with weight 0)
// This lane's share (its own slots) of the contact part, before the team sum.
template <int NV, int CPL, int NTG>
DMX_DEV void tree_hessian_lane(const TreeRows<NV, CPL, NTG>& rw, const uint32_t* act, double* H) {
  constexpr int NT = NV * (NV + 1) / 2;
#pragma unroll
  for (int i = 0; i < NT; ++i) H[i] = 0.0;
#pragma unroll
  for (int k = 0; k < CPL; ++k) {
    if (act[k] == 0u) continue;
    // the lane's edges J_n + s_e J_t(e) as combinations of its frame rows
    // (the free-body Hessian uses the same expansion)
    const double D = rw.D[k], mu = rw.mu[k];
    double o[2 * NTG];
#pragma unroll
    for (int e = 0; e < 2 * NTG; ++e) o[e] = ((act[k] >> e) & 1u) ? D : 0.0;
    double waa[NTG], wna[NTG];
#pragma unroll
    for (int a = 0; a < NTG; ++a) { waa[a] = o[2 * a] + o[2 * a + 1]; wna[a] = mu * (o[2 * a] - o[2 * a + 1]); }
    const double wnn = NTG == 2 ? waa[0] + waa[NTG - 1] : waa[0];
    const double mm = mu * mu;
    const double* Jn = rw.Jn[k];
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      double ui = wnn * Jn[i];
      double va[NTG];
#pragma unroll
      for (int a = 0; a < NTG; ++a) {
        ui += wna[a] * rw.Jt[k][a][i];
        va[a] = wna[a] * Jn[i] + mm * waa[a] * rw.Jt[k][a][i];
      }
#pragma unroll
      for (int j = 0; j <= i; ++j) {
        double hij = ui * Jn[j];
#pragma unroll
        for (int a = 0; a < NTG; ++a) hij += va[a] * rw.Jt[k][a][j];
        H[tri(i, j)] += hij;
      }
    }
  }
}
template <int NV, int CPL, int L, int NTG>
DMX_DEV void tree_hessian(const double* M, const TreeRows<NV, CPL, NTG>& rw, const uint32_t* act, double* H) {
  constexpr int NT = NV * (NV + 1) / 2;
  tree_hessian_lane<NV, CPL, NTG>(rw, act, H);
  team_sum_arr<L, NT>(H);
#pragma unroll
  for (int i = 0; i < NT; ++i) H[i] += M[i];
}

template <int NV, int CPL, int L>
DMX_DEV bool tree_same(const uint32_t* a, const uint32_t* b) {
  bool same = true;
#pragma unroll
  for (int k = 0; k < CPL; ++k) same = same && (a[k] == b[k]);
  return team_all<L>(same);
}

// exact Newton on the primal problem with dense M (see free_newton)
template <int NV, int CPL, int L, int NTG>
DMX_DEV void tree_newton(const double* M, const TreeRows<NV, CPL, NTG>& rw, const double* a0, const double* xw,
                         double* x, int maxit, Stat& st) {
  constexpr int NE = 2 * NTG;  // edges per lane slot
#pragma unroll
  for (int i = 0; i < NV; ++i) x[i] = a0[i];
  uint32_t act[CPL];
  double s[CPL][4];
  tree_active<NV, CPL, NTG>(rw, x, act, s);
  bool any = false;
#pragma unroll
  for (int k = 0; k < CPL; ++k) any = any || (act[k] != 0u);
  if (!team_any<L>(any)) return;  // no row active at a0: a0 is the minimizer
  if (xw) {  // warm start; the iteration converges to the same minimizer
#pragma unroll
    for (int i = 0; i < NV; ++i) x[i] = xw[i];
    tree_active<NV, CPL, NTG>(rw, x, act, s);
  }
  for (int it = 0; it < maxit; ++it) {
    st.newton_it++;
    if (team_leader(L)) st.u_nit++;
#pragma unroll
    for (int k = 0; k < CPL; ++k) {
      st.u_ncon += rw.first[k] && tree_contact_bits<NTG, L>(act[k]) != 0u;
      st.u_nedge += __popc(act[k]);
    }
    // gradient and Hessian of the active set, summed over the team together
    constexpr int NT = NV * (NV + 1) / 2;
    double gh[NV + NT];
    double* gp = gh;
    double* H = gh + NV;
#pragma unroll
    for (int i = 0; i < NV; ++i) gp[i] = 0.0;
#pragma unroll
    for (int k = 0; k < CPL; ++k) {
      if (act[k] == 0u) continue;
      // sum_e w_e (J_n + s_e J_t) = (sum w_e) J_n + mu (w0 - w1) J_t1 + mu (w2 - w3) J_t2
      double we[NE];
#pragma unroll
      for (int e = 0; e < NE; ++e) we[e] = ((act[k] >> e) & 1u) ? rw.D[k] * s[k][e] : 0.0;
      const double cn = NTG == 2 ? (we[0] + we[1]) + (we[NE - 2] + we[NE - 1]) : we[0] + we[1];
      double ca[NTG];
#pragma unroll
      for (int a = 0; a < NTG; ++a) ca[a] = rw.mu[k] * (we[2 * a] - we[2 * a + 1]);
#pragma unroll
      for (int i = 0; i < NV; ++i) {
        double g = cn * rw.Jn[k][i];
#pragma unroll
        for (int a = 0; a < NTG; ++a) g += ca[a] * rw.Jt[k][a][i];
        gp[i] += g;
      }
    }
    tree_hessian_lane<NV, CPL, NTG>(rw, act, H);
    team_sum_arr<L, NV + NT>(gh);
#pragma unroll
    for (int i = 0; i < NT; ++i) H[i] += M[i];
    double dx[NV], dl[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) dx[i] = x[i] - a0[i];
    symv_packed<NV>(M, dx, dl);
#pragma unroll
    for (int i = 0; i < NV; ++i) dl[i] = -(dl[i] + gp[i]);
    if (!chol_packed<NV>(H)) { st.status |= 4; return; }
    chol_solve_packed<NV>(H, dl);
    double dmax = 0.0, xmax = 1.0;
#pragma unroll
    for (int i = 0; i < NV; ++i) { dmax = fmax(dmax, fabs(dl[i])); xmax = fmax(xmax, fmax(fabs(x[i]), fabs(a0[i]))); }
    if (dmax <= 1e-13 * xmax) {
#pragma unroll
      for (int i = 0; i < NV; ++i) x[i] += dl[i];
      return;
    }
    double t[CPL][4];
    uint32_t act1[CPL];
#pragma unroll
    for (int k = 0; k < CPL; ++k) {
      act1[k] = 0u;
      if (!rw.on[k]) continue;
      const double jn = dotn<NV>(rw.Jn[k], dl);
      const double mu = rw.mu[k];
#pragma unroll
      for (int a = 0; a < NTG; ++a) {
        const double ja = dotn<NV>(rw.Jt[k][a], dl);
        t[k][2 * a] = jn + mu * ja; t[k][2 * a + 1] = jn - mu * ja;
      }
#pragma unroll
      for (int e = 0; e < NE; ++e)
        if (s[k][e] + t[k][e] < 0.0) act1[k] |= 1u << e;
    }
    if (tree_same<NV, CPL, L>(act, act1)) {
#pragma unroll
      for (int i = 0; i < NV; ++i) x[i] += dl[i];
      return;
    }
    double Mdl[NV];
    symv_packed<NV>(M, dl, Mdl);
    const double dMd = dotn<NV>(dl, Mdl), xMd = dotn<NV>(dx, Mdl);
    double lo = 0.0, hi = 1e300, a = 1.0;
    for (int ls = 0; ls < 60; ++ls) {
#pragma unroll
      for (int k = 0; k < CPL; ++k) st.u_ls += rw.on[k] && rw.first[k];
      double c1 = 0.0, c2 = 0.0;
      uint32_t sa[CPL], sn[CPL];
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
      if (a * c2 + c1 > 0.0) hi = a; else lo = a;
      double an = (c2 > 0.0) ? -c1 / c2 : a;
      if (!isfinite(an)) an = a;
#pragma unroll
      for (int k = 0; k < CPL; ++k) {
        sn[k] = 0u;
        if (!rw.on[k]) continue;
#pragma unroll
        for (int e = 0; e < NE; ++e)
          if (s[k][e] + an * t[k][e] < 0.0) sn[k] |= 1u << e;
      }
      if (tree_same<NV, CPL, L>(sa, sn)) { a = an; break; }
      if (!(an > lo && an < hi)) an = (hi < 1e299) ? 0.5 * (lo + hi) : 2.0 * a;
      a = an;
      if (hi - lo <= 1e-15 * hi) break;
      if (ls == 59) a = lo > 0.0 ? lo : a;
    }
#pragma unroll
    for (int i = 0; i < NV; ++i) x[i] += a * dl[i];
    tree_active<NV, CPL, NTG>(rw, x, act, s);
  }
  st.status |= 8;
}

// cross-product reverse: c = u x w with cotangent cb -> ub += w x cb, wb += cb x u
DMX_DEV void cross_rev(V3 u, V3 w, V3 cb, V3& ub, V3& wb) { ub += cross(w, cb); wb += cross(cb, u); }

template <int kNV, int NB, int NC, int L>
struct TreePhys {
  static constexpr int NV = kNV, NQ = kNV, TEAM = L;
  // a team of 8 or 16 lanes for half as many slots holds each contact on a
  // lane and its mirror lane (one tangent direction each)
  static constexpr int NTG = ((L == 8 || L == 16) && 2 * NC == L) ? 1 : 2;
  static constexpr int CPL = NTG == 1 ? 1 : (NC + L - 1) / L;
  using Model = TreeModel;

  DMX_DEV static TreeWs<NV, NB>& ws() {
    __shared__ TreeWs<NV, NB> s_ws[64 / L];
    return s_ws[(threadIdx.x & 63) / L];
  }

  DMX_DEV static void acc(const Model& m, const double* y, const double* tau, bool cfd, double beta, int maxit,
                          const double* xw, double* a, Stat& st) {
    TreeWs<NV, NB>& w = ws();
    const double* v = y + NQ;
    tree_kin<NV, NB>(m, y, v, nullptr, nullptr, w, false);
    double M[NV * (NV + 1) / 2], c[NV];
    tree_mass_bias<NV, NB>(m, w, M, c);
    double a0[NV], L_[NV * (NV + 1) / 2];
#pragma unroll
    for (int i = 0; i < NV * (NV + 1) / 2; ++i) L_[i] = M[i];
    if (!chol_packed<NV>(L_)) st.status |= 4;
#pragma unroll
    for (int i = 0; i < NV; ++i) a0[i] = tau[i] - c[i];
    chol_solve_packed<NV>(L_, a0);
    TreeRows<NV, CPL, NTG> rw;
    tree_rows<NV, NB, CPL, L, NTG>(m, w, v, cfd, beta, rw);
    if (team_leader(L)) st.u_rhs++;
#pragma unroll
    for (int k = 0; k < CPL; ++k) st.u_con += rw.on[k] && rw.first[k];
    tree_newton<NV, CPL, L, NTG>(M, rw, a0, xw, a, maxit, st);
  }

  DMX_DEV static void acc_vjp(const Model& m, const double* y, const double* tau, const double* xs_in,
                              const double* abar, bool cfd, double beta, int maxit, double* ybar, double* taubar,
                              Stat& st, double* hbar = nullptr) {
    // hbar (optional, [kParams]): += the contact parameters' cotangents
    // (friction, solref, solimp as one value shared by every pair, as for
    // single free bodies); no box geom (half sizes stay 0), and the mass entry
    // is NaN: a tree has one mass per body
    TreeWs<NV, NB>& w = ws();
    const double* q = y;
    const double* v = y + NQ;
    // frames and velocities; M, rows, active set at x*, lam
    tree_kin<NV, NB>(m, q, v, nullptr, nullptr, w, false);
    double M[NV * (NV + 1) / 2], c[NV];
    tree_mass_bias<NV, NB>(m, w, M, c);
    TreeRows<NV, CPL, NTG> rw;
    tree_rows<NV, NB, CPL, L, NTG>(m, w, v, cfd, beta, rw);
    double xs[NV];
    if (cfd) {
      double Lm[NV * (NV + 1) / 2], a0[NV];
#pragma unroll
      for (int i = 0; i < NV * (NV + 1) / 2; ++i) Lm[i] = M[i];
      chol_packed<NV>(Lm);
#pragma unroll
      for (int i = 0; i < NV; ++i) a0[i] = tau[i] - c[i];
      chol_solve_packed<NV>(Lm, a0);
      tree_newton<NV, CPL, L, NTG>(M, rw, a0, nullptr, xs, maxit, st);
    } else {
#pragma unroll
      for (int i = 0; i < NV; ++i) xs[i] = xs_in[i];
    }
    uint32_t act[CPL];
    double s[CPL][4];
    tree_active<NV, CPL, NTG>(rw, xs, act, s);
    if (team_leader(L)) st.u_vjp++;
#pragma unroll
    for (int k = 0; k < CPL; ++k) { st.u_vcon += rw.on[k] && rw.first[k]; st.u_vedge += __popc(act[k]); }
    double H[NV * (NV + 1) / 2];
    tree_hessian<NV, CPL, L, NTG>(M, rw, act, H);
    chol_packed<NV>(H);
    double lam[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) lam[i] = abar[i];
    chol_solve_packed<NV>(H, lam);
    // motion under (v, x*) and the lam velocity field, with reverse storage
    tree_kin<NV, NB>(m, q, v, xs, lam, w, true);
    // zero the cotangent accumulators
    for (int b = 0; b < m.nb; ++b) {
      for (int i = 0; i < 3; ++i) w.bpb[b][i] = 0.0;
      for (int i = 0; i < 9; ++i) w.bRb[b][i] = 0.0;
      for (int i = 0; i < 18; ++i) w.bmb[b][i] = 0.0;
    }
    for (int j = 0; j < m.nj; ++j)
      for (int i = 0; i < 3; ++i) { w.jab[j][i] = 0.0; w.jobar[j][i] = 0.0; }
    // ---- contact term: Psi_c = -sum_A (J_e lam) f_e, cotangents of rows
    double vb[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) vb[i] = 0.0;
    // per-lane partial cotangents of body frames and joint axes/anchors (team-summed below)
    double cpb[NB][3], cRb[NB][9], cab[NV][3], cob[NV][3];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
#pragma unroll
      for (int i = 0; i < 3; ++i) cpb[b][i] = 0.0;
#pragma unroll
      for (int i = 0; i < 9; ++i) cRb[b][i] = 0.0;
    }
#pragma unroll
    for (int j = 0; j < NV; ++j)
#pragma unroll
      for (int i = 0; i < 3; ++i) { cab[j][i] = 0.0; cob[j][i] = 0.0; }
    double hb_[kParams];
#pragma unroll
    for (int i = 0; i < kParams; ++i) hb_[i] = 0.0;
#pragma unroll
    for (int k = 0; k < CPL; ++k) {
      if (!rw.on[k] || act[k] == 0u) continue;
      const PairF& pr = slot_pair(rw.slot[k]);
      const double mu = rw.mu[k], D = rw.D[k];
      double rbar = 0.0, ddr;
      const double dimp = impedance(pr, rw.r[k], &ddr);
      const double dD = ddr / (pr.ahat * (1.0 - dimp) * (1.0 - dimp));
      const double kk = dimp * pr.kscale;
      double dpt, ptd;  // d pterm / dr, d pterm / d(impedance) / kscale
      if (cfd) {
        double dsp;
        const double sp = softplus(-rw.r[k], beta, &dsp);
        dpt = pr.kscale * ddr * sp - kk * dsp;
        ptd = sp;
      } else {
        dpt = -(pr.kscale * ddr * rw.r[k] + kk);
        ptd = -rw.r[k];
      }
      // per-edge reverse summed over the lane's edges as combinations of its
      // frame rows (as in the free-body reverse; inactive edges weigh 0)
      constexpr int NE = 2 * NTG;
      const double* Jn = rw.Jn[k];
      const double ln = dotn<NV>(Jn, lam), xn = dotn<NV>(Jn, xs);
      double la[NTG], xa[NTG];
#pragma unroll
      for (int a = 0; a < NTG; ++a) { la[a] = dotn<NV>(rw.Jt[k][a], lam); xa[a] = dotn<NV>(rw.Jt[k][a], xs); }
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
      const double Fn = NTG == 2 ? (fe[0] + fe[1]) + (fe[NE - 2] + fe[NE - 1]) : fe[0] + fe[1];
      const double An = NTG == 2 ? (ae[0] + ae[1]) + (ae[NE - 2] + ae[NE - 1]) : ae[0] + ae[1];
      if (hbar) {
        // the contact parameters, as in the free-body reverse: friction in the
        // edges J_n +- mu J_t and in Ahat = (1 + mu^2) w, solref in a_ref's b
        // and k, solimp in d(r) (and dwidth in b and k)
        const double vn = dotn<NV>(Jn, v);
        double mub = dsum * (-2.0 * mu * D / (1.0 + mu * mu)), bb = 0.0;
#pragma unroll
        for (int a = 0; a < NTG; ++a) {
          const double vt = dotn<NV>(rw.Jt[k][a], v);
          const double fd = fe[2 * a] - fe[2 * a + 1], ad = ae[2 * a] - ae[2 * a + 1];
          mub += fd * la[a] - ad * (xa[a] + pr.bcoef * vt);
          bb -= (ae[2 * a] + ae[2 * a + 1]) * vn + mu * ad * vt;
        }
        const double kb = An * dimp * ptd;
        const double sb = pr.bcoef * bb + 2.0 * pr.kscale * kb;
        hb_[3] += mub;
        hb_[4] -= sb / pr.solref[0];
        hb_[5] -= 2.0 * pr.kscale * kb / pr.solref[1];
        const double dbar = dsum / (pr.ahat * (1.0 - dimp) * (1.0 - dimp)) + An * pr.kscale * ptd;
        double gs[5];
        impedance_solimp_grad(pr, rw.r[k], gs);
#pragma unroll
        for (int i = 0; i < 5; ++i) hb_[7 + i] += dbar * gs[i];
        hb_[8] -= sb / pr.si[1];
      }
      double Fa[NTG], Aa[NTG];
#pragma unroll
      for (int a = 0; a < NTG; ++a) { Fa[a] = mu * (fe[2 * a] - fe[2 * a + 1]); Aa[a] = mu * (ae[2 * a] - ae[2 * a + 1]); }
      double Jb[1 + NTG][NV];  // cotangents of J_n and the lane's tangent rows
#pragma unroll
      for (int i = 0; i < NV; ++i) {
        const double z = xs[i] + pr.bcoef * v[i];
        Jb[0][i] = Fn * lam[i] - An * z;
        double vt = An * Jn[i];
#pragma unroll
        for (int a = 0; a < NTG; ++a) {
          Jb[1 + a][i] = Fa[a] * lam[i] - Aa[a] * z;
          vt += Aa[a] * rw.Jt[k][a][i];
        }
        vb[i] -= pr.bcoef * vt;
      }
      // J_u[d] = u . (a_d x (P - o_d)) (hinge) or u . a_d (slide)
      const int b = rw.body[k];
      V3 lc, P;
      double r;
      tree_slot_geom(m, rw.slot[k], ld3(w.p[b]), ldm(w.R[b]), &lc, &r, &P);
      V3 Pb = mk3(0, 0, 0);
      V3 us[1 + NTG];
      us[0] = ld3(pr.n);
#pragma unroll
      for (int a = 0; a < NTG; ++a) us[1 + a] = (NTG == 2 ? a == 1 : rw.half[k] == 1) ? ld3(pr.t2) : ld3(pr.t1);
      const unsigned anc = m.banc[b];
#pragma unroll
      for (int d = 0; d < NV; ++d) {
        if (!((anc >> d) & 1u)) continue;
        const V3 a = ld3(w.ax[d]);
        V3 ab = mk3(0, 0, 0), ob = mk3(0, 0, 0);
        if (m.jtype[d] == 1) {
          const V3 rel = P - ld3(w.an[d]);
#pragma unroll
          for (int u = 0; u < 1 + NTG; ++u) {
            const double g = Jb[u][d];
            ab += g * cross(rel, us[u]);
            const V3 ua = cross(us[u], a);
            Pb += g * ua;
            ob -= g * ua;
          }
        } else {
#pragma unroll
          for (int u = 0; u < 1 + NTG; ++u) ab += Jb[u][d] * us[u];
        }
        cab[d][0] += ab.x; cab[d][1] += ab.y; cab[d][2] += ab.z;
        cob[d][0] += ob.x; cob[d][1] += ob.y; cob[d][2] += ob.z;
      }
      // P = ce - (rad + r/2) n; r = n.(ce - p0) - rad; ce = p_b + R_b lc
      const V3 n = ld3(pr.n);
      rbar += -0.5 * dot(n, Pb);
      const V3 ceb = Pb + rbar * n;
      M3 Rb2;
#pragma unroll
      for (int i = 0; i < 9; ++i) Rb2.a[i] = 0.0;
      outer_add(Rb2, ceb, lc);
#pragma unroll
      for (int bb = 0; bb < NB; ++bb)
        if (bb == b) {
          cpb[bb][0] += ceb.x; cpb[bb][1] += ceb.y; cpb[bb][2] += ceb.z;
#pragma unroll
          for (int i = 0; i < 9; ++i) cRb[bb][i] += Rb2.a[i];
        }
    }
    if (hbar) {
      team_sum_arr<L, kParams>(hb_);
#pragma unroll
      for (int i = 0; i < kParams; ++i) hbar[i] += hb_[i];
      hbar[6] = __longlong_as_double(0x7ff8000000000000ll);
    }
    // team sums; the contact term enters Psi with a minus sign, Ybar = -grad Psi
    team_sum_arr<L, NV>(vb);
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      double tmp[12];
#pragma unroll
      for (int i = 0; i < 3; ++i) tmp[i] = cpb[b][i];
#pragma unroll
      for (int i = 0; i < 9; ++i) tmp[3 + i] = cRb[b][i];
      team_sum_arr<L, 12>(tmp);
#pragma unroll
      for (int i = 0; i < 3; ++i) w.bpb[b][i] = -tmp[i];
#pragma unroll
      for (int i = 0; i < 9; ++i) w.bRb[b][i] = -tmp[3 + i];
    }
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      double tmp[6];
#pragma unroll
      for (int i = 0; i < 3; ++i) { tmp[i] = cab[j][i]; tmp[3 + i] = cob[j][i]; }
      team_sum_arr<L, 6>(tmp);
#pragma unroll
      for (int i = 0; i < 3; ++i) { w.jab[j][i] = -tmp[i]; w.jobar[j][i] = -tmp[3 + i]; }
    }
    // ---- inverse-dynamics term: seeds per body of lam^T ID
    for (int b = 0; b < m.nb; ++b) {
      const M3 R = ldm(w.R[b]);
      const M3 Ib = ldm(m.bI[b]);
      const M3 Iw = mmulT(mmul(R, Ib), R);
      const V3 om = ld3(w.w[b]), al = ld3(w.al[b]), ac = ld3(w.ac[b]), kap = ld3(w.kap[b]), ell = ld3(w.ell[b]);
      const double mb = m.bmass[b];
      const V3 Iom = mul(Iw, om);
      const V3 kxo = cross(kap, om);
      // d/d(motion): w, vel, al, ac, kap, ell
      const V3 wb = cross(Iom, kap) + mul(Iw, kxo);
      const V3 alb = mul(Iw, kap);
      const V3 acb = mb * ell;
      const V3 kapb = mul(Iw, al) + cross(om, Iom);
      const V3 ellb = mb * (ac - ld3(m.grav));
      double* mb_ = w.bmb[b];
      mb_[0] += wb.x; mb_[1] += wb.y; mb_[2] += wb.z;
      mb_[6] += alb.x; mb_[7] += alb.y; mb_[8] += alb.z;
      mb_[9] += acb.x; mb_[10] += acb.y; mb_[11] += acb.z;
      mb_[12] += kapb.x; mb_[13] += kapb.y; mb_[14] += kapb.z;
      mb_[15] += ellb.x; mb_[16] += ellb.y; mb_[17] += ellb.z;
      // I_w = R Ib R^T: Ibar_w = kap al^T + (kap x w) w^T; Rbar += (Ibar + Ibar^T) R Ib
      M3 Ibar;
#pragma unroll
      for (int i = 0; i < 9; ++i) Ibar.a[i] = 0.0;
      outer_add(Ibar, kap, al);
      outer_add(Ibar, kxo, om);
      M3 S;
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) S.a[i * 3 + j] = Ibar.a[i * 3 + j] + Ibar.a[j * 3 + i];
      const M3 G = mmul(mmul(S, R), Ib);
#pragma unroll
      for (int i = 0; i < 9; ++i) w.bRb[b][i] += G.a[i];
    }
    // ---- reverse sweep over bodies and joints (ID seeds enter with +, Ybar = -grad)
    double qb[NV], vdb[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) { qb[i] = 0.0; vdb[i] = 0.0; }
    for (int b = m.nb - 1; b >= 0; --b) {
      V3 pbar = ld3(w.bpb[b]);
      M3 Rbar = ldm(w.bRb[b]);
      const double* mb_ = w.bmb[b];
      V3 wbar = ld3(mb_), vbar = ld3(mb_ + 3), albar = ld3(mb_ + 6), acbar = ld3(mb_ + 9), kbar = ld3(mb_ + 12),
         lbar = ld3(mb_ + 15);
      for (int j = m.bj0[b] + m.bjn[b] - 1; j >= m.bj0[b]; --j) {
        const double* mm = w.jm_in[j];
        const V3 w0 = ld3(mm), al0 = ld3(mm + 6), k0 = ld3(mm + 12);
        const V3 p_in = ld3(w.jp_in[j]), p_out = ld3(w.jp_out[j]);
        const M3 R_in = ldm(w.jR_in[j]);
        const V3 a = ld3(w.ax[j]), o = ld3(w.an[j]);
        const V3 jax = ld3(m.jaxis[j]), jps = ld3(m.jpos[j]);
        const double qdj = v[j], qddj = xs[j], lj = lam[j];
        V3 ab = ld3(w.jab[j]), obar = ld3(w.jobar[j]);
        if (m.jtype[j] == 1) {
          const V3 wa = qdj * a;
          const V3 w2 = w0 + wa, al2 = al0 + cross(w0, wa) + qddj * a, k2 = k0 + lj * a;
          const V3 r1 = o - p_in, r2 = p_out - o;
          // ell' = lo + k2 x r2
          V3 lob = lbar, k2b = kbar, r2b = mk3(0, 0, 0), r1b = mk3(0, 0, 0);
          cross_rev(k2, r2, lbar, k2b, r2b);
          // ac' = ao + al2 x r2 + w2 x (w2 x r2)
          V3 aob = acbar, al2b = albar, w2b = wbar;
          cross_rev(al2, r2, acbar, al2b, r2b);
          {
            const V3 z = cross(w2, r2);
            V3 zb = mk3(0, 0, 0);
            cross_rev(w2, z, acbar, w2b, zb);
            cross_rev(w2, r2, zb, w2b, r2b);
          }
          // vel' = vo + w2 x r2
          V3 vob = vbar;
          cross_rev(w2, r2, vbar, w2b, r2b);
          // r2 = p_out - o ; p_out = o - R_out jps
          V3 poutb = pbar + r2b;
          obar -= r2b;
          obar += poutb;
          M3 Routb = Rbar;
          {
            M3 t;
#pragma unroll
            for (int i = 0; i < 9; ++i) t.a[i] = 0.0;
            outer_add(t, neg(poutb), jps);
#pragma unroll
            for (int i = 0; i < 9; ++i) Routb.a[i] += t.a[i];
          }
          // k2 = k0 + lam a
          V3 k0b = k2b;
          ab += lj * k2b;
          // al2 = al0 + w0 x wa + qdd a
          V3 al0b = al2b, w0b = mk3(0, 0, 0), wab = mk3(0, 0, 0);
          cross_rev(w0, wa, al2b, w0b, wab);
          ab += qddj * al2b;
          // w2 = w0 + wa
          w0b += w2b;
          wab += w2b;
          // wa = qd a
          ab += qdj * wab;
          vdb[j] += dot(wab, a);
          // lo = ell0 + k0 x r1
          V3 l0b = lob;
          cross_rev(k0, r1, lob, k0b, r1b);
          // ao = ac0 + al0 x r1 + w0 x (w0 x r1)
          V3 ac0b = aob;
          cross_rev(al0, r1, aob, al0b, r1b);
          {
            const V3 z = cross(w0, r1);
            V3 zb = mk3(0, 0, 0);
            cross_rev(w0, z, aob, w0b, zb);
            cross_rev(w0, r1, zb, w0b, r1b);
          }
          // vo = vel0 + w0 x r1
          V3 v0b = vob;
          cross_rev(w0, r1, vob, w0b, r1b);
          // r1 = o - p_in
          obar += r1b;
          V3 pinb = neg(r1b);
          // R_out = R_in Rot(th): Rbar_in = Rbar_out Rot^T; th_bar = <Rbar_out, R_in dRot>
          double c, sn;
          const M3 Rot = axis_rot(jax, q[j], &c, &sn);
          const M3 dRot = axis_rot_d(jax, c, sn);
          M3 Rinb = mmulT(Routb, Rot);
          const M3 RdR = mmul(R_in, dRot);
          double thb = 0.0;
#pragma unroll
          for (int i = 0; i < 9; ++i) thb += Routb.a[i] * RdR.a[i];
          qb[j] += thb;
          // o = p_in + R_in jps ; a = R_in jax
          pinb += obar;
          outer_add(Rinb, obar, jps);
          outer_add(Rinb, ab, jax);
          pbar = pinb;
          Rbar = Rinb;
          wbar = w0b; vbar = v0b; albar = al0b; acbar = ac0b; kbar = k0b; lbar = l0b;
        } else {
          const double sj = q[j];
          const V3 rr = sj * a, wa = qdj * a;
          // ell' = ell + k x rr + lam a
          V3 rrb = mk3(0, 0, 0), k0b = kbar, w0b = wbar, al0b = albar;
          cross_rev(k0, rr, lbar, k0b, rrb);
          ab += lj * lbar;
          // ac' = ac + al x rr + w x (w x rr) + 2 w x wa + qdd a
          cross_rev(al0, rr, acbar, al0b, rrb);
          {
            const V3 z = cross(w0, rr);
            V3 zb = mk3(0, 0, 0);
            cross_rev(w0, z, acbar, w0b, zb);
            cross_rev(w0, rr, zb, w0b, rrb);
          }
          V3 wab = mk3(0, 0, 0);
          cross_rev(w0, wa, 2.0 * acbar, w0b, wab);
          ab += qddj * acbar;
          // vel' = vel + w x rr + wa
          cross_rev(w0, rr, vbar, w0b, rrb);
          wab += vbar;
          ab += qdj * wab;
          vdb[j] += dot(wab, a);
          // p' = p + rr ; rr = s a
          V3 pinb = pbar + obar;  // o = p_in + R_in jps (anchor, unused in the dynamics but tracked)
          ab += sj * (rrb + pbar);
          qb[j] += dot(rrb + pbar, a);
          M3 Rinb = Rbar;
          outer_add(Rinb, obar, jps);
          outer_add(Rinb, ab, jax);
          pbar = pinb;
          Rbar = Rinb;
          wbar = w0b; albar = al0b; kbar = k0b;
          // vel, ac, ell pass through
        }
      }
      // body entry: p = p_par + R_par bpos ; R = R_par bR ; motion transfer over r = p - p_par
      const int pa = m.bparent[b];
      if (pa >= 0) {
        const V3 pp = ld3(w.p[pa]);
        const M3 Rp = ldm(w.R[pa]);
        const V3 wp = ld3(w.w[pa]), ap = ld3(w.al[pa]), kp = ld3(w.kap[pa]);
        const V3 p0 = pp + mul(Rp, ld3(m.bpos[b]));
        const V3 r = p0 - pp;
        V3 rb = mk3(0, 0, 0), wpb = wbar, apb = albar, kpb = kbar;
        // ell = ell_p + kp x r
        cross_rev(kp, r, lbar, kpb, rb);
        // ac = ac_p + ap x r + wp x (wp x r)
        cross_rev(ap, r, acbar, apb, rb);
        {
          const V3 z = cross(wp, r);
          V3 zb = mk3(0, 0, 0);
          cross_rev(wp, z, acbar, wpb, zb);
          cross_rev(wp, r, zb, wpb, rb);
        }
        // vel = v_p + wp x r
        cross_rev(wp, r, vbar, wpb, rb);
        // r = p0 - pp ; p0 = pp + Rp bpos
        const V3 p0b = pbar + rb;
        V3 ppb = p0b - rb;
        M3 Rpb = mmulT(Rbar, ldm(m.bR[b]));
        outer_add(Rpb, p0b, ld3(m.bpos[b]));
        double* dst = w.bmb[pa];
        const V3 add6[6] = {wpb, vbar, apb, acbar, kpb, lbar};
#pragma unroll
        for (int u = 0; u < 6; ++u) { dst[3 * u] += add6[u].x; dst[3 * u + 1] += add6[u].y; dst[3 * u + 2] += add6[u].z; }
        w.bpb[pa][0] += ppb.x; w.bpb[pa][1] += ppb.y; w.bpb[pa][2] += ppb.z;
#pragma unroll
        for (int i = 0; i < 9; ++i) w.bRb[pa][i] += Rpb.a[i];
      }
    }
    // Ybar = -grad(Psi); the contact part was pre-negated into the accumulators,
    // the ID part is negated here; v also gets the a_ref cotangent (pre-negated)
#pragma unroll
    for (int i = 0; i < NV; ++i) { ybar[i] = -qb[i]; ybar[NQ + i] = -vdb[i] + vb[i]; }
#pragma unroll
    for (int i = 0; i < NV; ++i) taubar[i] = lam[i];
  }

  DMX_DEV static void qplus(const double* q, const double* dq, double* out) {
#pragma unroll
    for (int i = 0; i < NQ; ++i) out[i] = q[i] + dq[i];
  }
  struct QPlusKeep {};
  DMX_DEV static void qplus_keep(const double* q, const double* dq, double* out, QPlusKeep*) { qplus(q, dq, out); }
  DMX_DEV static void qplus_vjp(const double* q, const double* dq, const double* ob, double* qbar, double* dqb,
                                const QPlusKeep* = nullptr) {
#pragma unroll
    for (int i = 0; i < NQ; ++i) { qbar[i] += ob[i]; dqb[i] = ob[i]; }
  }
  // cotangent of the raw rates dq/dt = v (hinge and slide coordinates)
  DMX_DEV static void kin_vjp(const double*, const double* lq, double* xbar) {
#pragma unroll
    for (int d = 0; d < NV; ++d) xbar[NQ + d] += lq[d];
  }
  DMX_DEV static void tangent_project(const double*, double*) {}
  DMX_DEV static bool q_is_linear(int) { return true; }
  DMX_DEV static int q_dof(int i) { return i; }
};

}  // namespace dmx
