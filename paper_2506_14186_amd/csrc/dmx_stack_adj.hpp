// Reverse sweep of cube-stack rollouts (discretize-then-optimize, App. C.2):
// step sizes fixed, each accepted step reversed through its stage
// combinations, the (+) map and the acceleration map.
//
// VJP of the acceleration x* = qacc(Y) at the converged active set A
// (implicit differentiation of the optimality system, as for single bodies):
// lambda = H^-1 a_bar, then Y_bar = -(dG/dY)^T lambda with
// G = M x* - tau + c(Y) - sum_A J_e^T f_e, f_e = D_e (aref_e - J_e x*).  M is
// constant in these coordinates, so the terms are the bias c = (-m g,
// w x I w), and Phi = sum_A (J_e lambda) f_e, whose dependence on the body
// poses runs through the contact geometry (points, normals, frames, depths,
// impedances).  The pose derivatives of Phi are taken by dual-number passes,
// one per pose direction of each body of a pair (translations and body-frame
// rotations), through the same contact routine that produced the contact
// set: its discrete choices (separating axis, faces, clipping, the top four
// vertices) are fixed by the values, which every pass computes identically.
#pragma once
#include "dmx_stack_rk.hpp"

namespace dmx {

// Contacts of a pair at given (dual) poses.  One non-inlined instance serves
// the value pass and every derivative pass, so the value arithmetic (and with
// it every discrete choice) is the same in all of them.
__device__ __noinline__ int pair_geom_dual(const StackModel& m, int pair, const TV<Dual1>* cA, const TM<Dual1>* RA,
                                           const TV<Dual1>* cB, const TM<Dual1>* RB, double margin,
                                           const BoxChoice* ch, Dual1* r, TV<Dual1>* p, TV<Dual1>* n) {
  if (pair == 1) {
    const int cnt = box_plane_t<Dual1>(m.h, m.p0, m.pn, *cB, *RB, margin, r, p);
    for (int j = 0; j < cnt; ++j) n[j] = liftv<Dual1>(m.pn);
    return cnt;
  }
  return box_box_contacts<Dual1>(m.h, m.h, *cA, *RA, *cB, *RB, margin, *ch, r, p, n);
}

DMX_DEV void load_pose_dual(const StackLds& S, int b, TV<Dual1>* c, TM<Dual1>* R) {
  *c = tv<Dual1>(mkd(S.P[b][0]), mkd(S.P[b][1]), mkd(S.P[b][2]));
#pragma unroll
  for (int i = 0; i < 9; ++i) R->a[i] = mkd(S.R[b][i]);
}
// seed direction j of a body pose: j < 3 translation e_j, else the body-frame
// rotation R <- R exp([e_(j-3)]x), dR = R [e]x
DMX_DEV void seed_pose(const StackLds& S, int b, int j, TV<Dual1>* c, TM<Dual1>* R) {
  if (j < 3) {
    if (j == 0) c->x.d = 1.0; else if (j == 1) c->y.d = 1.0; else c->z.d = 1.0;
    return;
  }
  const int a = j - 3;
  const double* Rv = S.R[b];
#pragma unroll
  for (int col = 0; col < 3; ++col) {
    // column col of R [e_a]x is R (e_a x e_col)
    double e[3] = {0.0, 0.0, 0.0};
    const int c1 = (a + 1) % 3, c2 = (a + 2) % 3;
    if (col == c1) e[c2] = 1.0;        // e_a x e_(a+1) = e_(a+2)
    else if (col == c2) e[c1] = -1.0;  // e_a x e_(a+2) = -e_(a+1)
#pragma unroll
    for (int row = 0; row < 3; ++row)
      R->a[3 * row + col].d = Rv[3 * row] * e[0] + Rv[3 * row + 1] * e[1] + Rv[3 * row + 2] * e[2];
  }
}

// velocity at a contact of body b for a generalized vector (linear part,
// body-frame angular part) given the body's (dual) rotation and lever arm
DMX_DEV TV<Dual1> gen_vel(const double* w, const TM<Dual1>& R, const TV<Dual1>& rb) {
  const TV<Dual1> om = tmul(R, tv<Dual1>(mkd(w[3]), mkd(w[4]), mkd(w[5])));
  return tv<Dual1>(mkd(w[0]), mkd(w[1]), mkd(w[2])) + tcross(om, rb);
}

DMX_DEV Dual1 imp_dual(const StackModel& m, Dual1 r) {
  double ddr;
  const double d = stack_imp(m, r.v, &ddr);
  return mkd(d, ddr * r.d);
}
DMX_DEV Dual1 softplus_dual(Dual1 z, double beta) {
  double dsp;
  const double s = stack_softplus(z.v, beta, &dsp);
  return mkd(s, dsp * z.d);
}

// Phi of a pair's contacts (edges active per `act`, 4 bits per contact) for
// the generalized vectors lam, xs, v of the two bodies (S.vec[kVecD/X/V]).
DMX_DEV Dual1 pair_phi(const StackModel& m, const StackLds& S, int b1, int b2, double ahat, bool cfd, double beta,
                       int cnt, unsigned act, const Dual1* r, const TV<Dual1>* p, const TV<Dual1>* n,
                       const TV<Dual1>& c1, const TM<Dual1>& R1, const TV<Dual1>& c2, const TM<Dual1>& R2) {
  Dual1 phi = mkd(0.0);
  for (int j = 0; j < cnt; ++j) {
    const unsigned a = (act >> (4 * j)) & 15u;
    if (!a) continue;
    TV<Dual1> t1, t2;
    make_frame_t<Dual1>(n[j], &t1, &t2);
    const TV<Dual1> r2 = p[j] - c2;
    TV<Dual1> ul = gen_vel(S.vec[kVecD][b2], R2, r2), ux = gen_vel(S.vec[kVecX][b2], R2, r2),
              uv = gen_vel(S.vec[kVecV][b2], R2, r2);
    if (b1 >= 0) {
      const TV<Dual1> r1 = p[j] - c1;
      ul = ul - gen_vel(S.vec[kVecD][b1], R1, r1);
      ux = ux - gen_vel(S.vec[kVecX][b1], R1, r1);
      uv = uv - gen_vel(S.vec[kVecV][b1], R1, r1);
    }
    const Dual1 d = imp_dual(m, r[j]);
    const Dual1 D = d / (ahat * (1.0 - d));
    const Dual1 kk = d * m.kscale;
    const Dual1 pterm = cfd ? kk * softplus_dual(mkd(0.0) - r[j], beta) : mkd(0.0) - kk * r[j];
    const Dual1 ln = tdot(n[j], ul), l1 = tdot(t1, ul), l2 = tdot(t2, ul);
    const Dual1 xn = tdot(n[j], ux), x1 = tdot(t1, ux), x2 = tdot(t2, ux);
    const Dual1 vn = tdot(n[j], uv), v1 = tdot(t1, uv), v2 = tdot(t2, uv);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      if (!((a >> e) & 1u)) continue;
      const double sg = (e & 1) ? -m.mu : m.mu;
      const Dual1 le = ln + sg * (e < 2 ? l1 : l2);
      const Dual1 xe = xn + sg * (e < 2 ? x1 : x2);
      const Dual1 ve = vn + sg * (e < 2 ? v1 : v2);
      const Dual1 aref = pterm - m.bcoef * ve;
      phi += le * (D * (aref - xe));
    }
  }
  return phi;
}

// VJP of the acceleration map at this lane's stage state (yq, yv) with the
// stage acceleration xs (unless cfd: then the contacts-from-distance field's
// own acceleration, solved here) and the cotangent ab: cotangents of the
// state (qb: 3 or 4, vb: 3) and of this lane's generalized forces (tb).
DMX_DEV void stack_acc_vjp(const StackModel& m, StackLds& S, const StackRole& ro, const double* yq,
                           const double* yv, const double* tau, const double* xs_in, const double* ab, bool cfd,
                           double beta, int maxit, double* qb, double* vb, double* tb, StackStat& st) {
  // frames and velocity twists
  if (ro.dof) {
    if (ro.half == 0) {
      S.P[ro.b][0] = yq[0]; S.P[ro.b][1] = yq[1]; S.P[ro.b][2] = yq[2];
      double* t = S.vec[kVecV][ro.b];
      t[0] = yv[0]; t[1] = yv[1]; t[2] = yv[2];
    } else {
      const Q4 qh = qnormalize(mkq(yq[0], yq[1], yq[2], yq[3]), nullptr);
      const M3 R = quat2mat(qh);
#pragma unroll
      for (int i = 0; i < 9; ++i) S.R[ro.b][i] = R.a[i];
      const V3 w = mul(R, mk3(yv[0], yv[1], yv[2]));
      double* t = S.vec[kVecV][ro.b] + 3;
      t[0] = w.x; t[1] = w.y; t[2] = w.z;
    }
  }
  wave_fence();
  // value pass of the pair's contacts (the dual routine with zero seeds)
  const double margin = cfd ? m.cf[2] : 0.0;
  BoxChoice ch{-1, 0};
  bool near = false;
  TV<Dual1> cA, cB;
  TM<Dual1> RA, RB;
  int cnt = 0;
  Dual1 r[kBoxBoxMax];
  TV<Dual1> p[kBoxBoxMax], n[kBoxBoxMax];
  if (ro.pair) {
    load_pose_dual(S, ro.pb2, &cB, &RB);
    if (ro.pair == 1) {
      near = dot(ld3(m.pn), ld3(S.P[ro.pb2]) - ld3(m.p0)) < m.rbound + margin;
    } else {
      load_pose_dual(S, ro.pb1, &cA, &RA);
      const V3 dc = ld3(S.P[ro.pb2]) - ld3(S.P[ro.pb1]);
      near = sqrt(dot(dc, dc)) < 2.0 * m.rbound + margin;
      if (near) {
        TM<double> Ra, Rb;
#pragma unroll
        for (int i = 0; i < 9; ++i) { Ra.a[i] = S.R[ro.pb1][i]; Rb.a[i] = S.R[ro.pb2][i]; }
        near = box_box_choose(m.h, m.h, tv<double>(S.P[ro.pb1][0], S.P[ro.pb1][1], S.P[ro.pb1][2]), Ra,
                              tv<double>(S.P[ro.pb2][0], S.P[ro.pb2][1], S.P[ro.pb2][2]), Rb, margin, &ch);
      }
    }
    if (near) cnt = pair_geom_dual(m, ro.pair, &cA, &RA, &cB, &RB, margin, &ch, r, p, n);
  }
  if (nonneighbour_contact(m, S, margin)) st.status |= kStGraph;
  int total;
  const int off = wave_excl_scan(cnt, &total);
  const int keep = max(0, min(cnt, kStackContacts - off));
  for (int j = 0; j < keep; ++j) {
    const int c = off + j;
    S.cp[0][c] = p[j].x.v; S.cp[1][c] = p[j].y.v; S.cp[2][c] = p[j].z.v;
    S.cn[0][c] = n[j].x.v; S.cn[1][c] = n[j].y.v; S.cn[2][c] = n[j].z.v;
    S.cr[c] = r[j].v;
  }
  wave_fence();
  PairSlots ps;
  ps.off = off;
  ps.cnt = keep;
  ps.act = 0u;
  ps.ahat = ro.pair == 2 ? m.ahat_box : m.ahat_plane;
  double a0[3], xs[3];
  stack_a0(m, ro, yv, tau, a0);
  if (cfd) {
    stack_newton(m, S, ro, ps, true, beta, maxit, a0, nullptr, xs, st);
  } else {
#pragma unroll
    for (int j = 0; j < 3; ++j) xs[j] = xs_in[j];
  }
  // active set at x* and the Hessian there
  publish_twist(S, ro, kVecX, xs);
  ps.act = pair_activity(m, S, ro, ps, kVecX, cfd, beta);
  if (ro.lane == 0) st.u_vjp++;
  if (ro.pair) { st.u_vedge += __popc(ps.act); for (int j = 0; j < ps.cnt; ++j) st.u_vcon += ((ps.act >> (4 * j)) & 15u) != 0u; }
  assemble(m, S, ro, ps, cfd, beta, xs, a0);
  if (ro.dof) {
#pragma unroll
    for (int j = 0; j < 3; ++j) S.gv[ro.b][3 * ro.half + j] = ab[j];
  }
  wave_fence();
  if (!block_chol(S, m.k)) st.status |= 4;
  block_solve(S, m.k);
  double lam[3] = {0.0, 0.0, 0.0};
  if (ro.dof) {
#pragma unroll
    for (int j = 0; j < 3; ++j) lam[j] = S.gv[ro.b][3 * ro.half + j];
  }
  wave_fence();
  // generalized vectors of the bodies: lambda, x*, v
  if (ro.dof) {
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      S.vec[kVecD][ro.b][3 * ro.half + j] = lam[j];
      S.vec[kVecX][ro.b][3 * ro.half + j] = xs[j];
      S.vec[kVecV][ro.b][3 * ro.half + j] = yv[j];
    }
  }
  wave_fence();
  // pair lanes: pose cotangents of their bodies (dual passes) and velocity
  // cotangents (Phi is linear in v through aref = -b J v + ...)
  double pose1[6] = {0, 0, 0, 0, 0, 0}, pose2[6] = {0, 0, 0, 0, 0, 0};
  double vel1[6] = {0, 0, 0, 0, 0, 0}, vel2[6] = {0, 0, 0, 0, 0, 0};
  if (ro.pair && ps.cnt > 0 && ps.act != 0u) {
    const int nb = ro.pair == 2 ? 2 : 1;
#pragma unroll 1
    for (int pass = 0; pass < 6 * nb; ++pass) {
      const int body = pass < 6 ? ro.pb2 : ro.pb1;
      const int dir = pass % 6;
      TV<Dual1> sA = cA, sB = cB;
      TM<Dual1> tA = RA, tB = RB;
      if (body == ro.pb2) seed_pose(S, body, dir, &sB, &tB);
      else seed_pose(S, body, dir, &sA, &tA);
      Dual1 rr[kBoxBoxMax];
      TV<Dual1> pp[kBoxBoxMax], nn[kBoxBoxMax];
      const int c2 = pair_geom_dual(m, ro.pair, &sA, &tA, &sB, &tB, margin, &ch, rr, pp, nn);
      const int use = min(c2, ps.cnt);
      const Dual1 phi = pair_phi(m, S, ro.pb1, ro.pb2, ps.ahat, cfd, beta, use, ps.act, rr, pp, nn, sA, tA, sB, tB);
      if (body == ro.pb2) pose2[dir] = phi.d; else pose1[dir] = phi.d;
    }
    // d Phi / d v = sum_A (J_e lambda) D (-b) J_e^T
    for (int j = 0; j < ps.cnt; ++j) {
      const unsigned a = (ps.act >> (4 * j)) & 15u;
      if (!a) continue;
      CRow w;
      const V3 pc = mk3(S.cp[0][ps.off + j], S.cp[1][ps.off + j], S.cp[2][ps.off + j]);
      w.n = mk3(S.cn[0][ps.off + j], S.cn[1][ps.off + j], S.cn[2][ps.off + j]);
      TV<double> t1, t2;
      make_frame_t<double>(tv<double>(w.n.x, w.n.y, w.n.z), &t1, &t2);
      w.t1 = mk3(t1.x, t1.y, t1.z);
      w.t2 = mk3(t2.x, t2.y, t2.z);
      w.r2 = pc - ld3(S.P[ro.pb2]);
      w.r1 = ro.pb1 >= 0 ? pc - ld3(S.P[ro.pb1]) : mk3(0, 0, 0);
      double ddr;
      const double d = stack_imp(m, S.cr[ps.off + j], &ddr);
      const double D = d / (ps.ahat * (1.0 - d));
      // J_d lambda from the body twists of lambda
      auto twist = [&](int b, V3 rb) {
        const double* g = S.vec[kVecD][b];
        const V3 om = mul(*(const M3*)S.R[b], mk3(g[3], g[4], g[5]));
        return mk3(g[0], g[1], g[2]) + cross(om, rb);
      };
      V3 ul = twist(ro.pb2, w.r2);
      if (ro.pb1 >= 0) ul -= twist(ro.pb1, w.r1);
      V3 fv = mk3(0, 0, 0);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        if (!((a >> e) & 1u)) continue;
        const V3 de = edge_vec(w, m.mu, e);
        fv += (-m.bcoef * D * dot(de, ul)) * de;
      }
      const V3 m2 = mulT(*(const M3*)S.R[ro.pb2], cross(w.r2, fv));
      vel2[0] += fv.x; vel2[1] += fv.y; vel2[2] += fv.z; vel2[3] += m2.x; vel2[4] += m2.y; vel2[5] += m2.z;
      if (ro.pb1 >= 0) {
        const V3 m1 = mulT(*(const M3*)S.R[ro.pb1], cross(w.r1, fv));
        vel1[0] -= fv.x; vel1[1] -= fv.y; vel1[2] -= fv.z; vel1[3] -= m1.x; vel1[4] -= m1.y; vel1[5] -= m1.z;
      }
    }
  }
  // gather per body in a fixed order: plane pair, lower-body share of the box
  // pair above... (S.gv: pose cotangent, S.Ho[b][0..5]: velocity cotangent)
  if (ro.pair == 1) {
#pragma unroll
    for (int i = 0; i < 6; ++i) { S.gv[ro.pb2][i] = pose2[i]; S.Ho[ro.pb2][i] = vel2[i]; }
  }
  wave_fence();
  if (ro.pair == 2) {
#pragma unroll
    for (int i = 0; i < 6; ++i) { S.gv[ro.pb1][i] += pose1[i]; S.Ho[ro.pb1][i] += vel1[i]; }
  }
  wave_fence();
  if (ro.pair == 2) {
#pragma unroll
    for (int i = 0; i < 6; ++i) { S.gv[ro.pb2][i] += pose2[i]; S.Ho[ro.pb2][i] += vel2[i]; }
  }
  wave_fence();
#pragma unroll
  for (int j = 0; j < 4; ++j) qb[j] = 0.0;
#pragma unroll
  for (int j = 0; j < 3; ++j) { vb[j] = 0.0; tb[j] = 0.0; }
  if (ro.dof) {
    const double* pg = S.gv[ro.b];
    const double* vg = S.Ho[ro.b];
    if (ro.half == 0) {
#pragma unroll
      for (int j = 0; j < 3; ++j) { qb[j] = pg[j]; vb[j] = vg[j]; }
    } else {
      double inv;
      const Q4 qh = qnormalize(mkq(yq[0], yq[1], yq[2], yq[3]), &inv);
      const Q4 qhb = qscale(2.0, qmul(qh, mkq(0.0, pg[3], pg[4], pg[5])));
      const Q4 q4 = qnormalize_vjp(qh, inv, qhb);
      qb[0] = q4.w; qb[1] = q4.x; qb[2] = q4.y; qb[3] = q4.z;
      // bias w x I w: v_bar -= I w x lam + I (lam x w)
      const V3 w = mk3(yv[0], yv[1], yv[2]);
      const V3 Iw = mk3(m.I[0] * w.x, m.I[1] * w.y, m.I[2] * w.z);
      const V3 lm = mk3(lam[0], lam[1], lam[2]);
      const V3 t1 = cross(Iw, lm), t2 = cross(lm, w);
      vb[0] = vg[3] - t1.x - m.I[0] * t2.x;
      vb[1] = vg[4] - t1.y - m.I[1] * t2.y;
      vb[2] = vg[5] - t1.z - m.I[2] * t2.z;
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) tb[j] = lam[j];
  }
  wave_fence();
}

// (+) VJP on this lane: position lanes pass the cotangent through; quaternion
// lanes back through normalize(quat exp(dq / 2)).
DMX_DEV void stack_qplus_vjp(const StackRole& ro, const double* yq, const double* dq, const double* ob, double* qbar,
                             double* dqb) {
  if (ro.half == 0) {
#pragma unroll
    for (int j = 0; j < 3; ++j) { qbar[j] += ob[j]; dqb[j] = ob[j]; }
    return;
  }
  const V3 th = mk3(dq[0], dq[1], dq[2]);
  double c, s, dc, ds;
  const Q4 e = qexp_half(th, &c, &s, &dc, &ds);
  const Q4 q4 = mkq(yq[0], yq[1], yq[2], yq[3]);
  const Q4 w = qmul(q4, e);
  double inv;
  const Q4 r = qnormalize(w, &inv);
  const Q4 wb = qnormalize_vjp(r, inv, mkq(ob[0], ob[1], ob[2], ob[3]));
  const Q4 qq = qmul(wb, qconj(e));
  const Q4 eb = qmul(qconj(q4), wb);
  qbar[0] += qq.w; qbar[1] += qq.x; qbar[2] += qq.y; qbar[3] += qq.z;
  const double tv = eb.x * th.x + eb.y * th.y + eb.z * th.z;
  const double g = 2.0 * (dc * eb.w + ds * tv);
  dqb[0] = s * eb.x + g * th.x;
  dqb[1] = s * eb.y + g * th.y;
  dqb[2] = s * eb.z + g * th.z;
}

template <bool RECOMPUTE>
DMX_DEV void stack_adj_world(const StackModel& m, StackLds& S, const StackArgs& a, int w) {
  const StackRole ro = stack_role(m);
  const SolverOpts& o = a.o;
  const int nsteps = a.n_acc[w];
  const int n_int = a.n_int_w ? a.n_int_w[w] : a.n_int;
  const int NX = 13 * m.k;
  const int rec = stack_rec(m.k, a.stages);
  const double* uw = (a.u && m.nu) ? a.u + st_uoff(a, w) : nullptr;
  double* ubw = (a.ubar && m.nu) ? a.ubar + st_uoff(a, w) : nullptr;
  const size_t nut = (size_t)n_int * m.nu;
  const double* tape_w = a.tape + st_toff(a, w);
  double* x0b = a.x0bar + st_xoff(a, w);
  if (a.status[w] & ~kStOverflow) {
    const double nan = __longlong_as_double(0x7ff8000000000000ll);
    for (int i = ro.lane; i < NX; i += 64) x0b[i] = nan;
    if (ubw) for (size_t i = ro.lane; i < nut; i += 64) ubw[i] = nan;
    return;
  }
  if (ubw) for (size_t i = ro.lane; i < nut; i += 64) ubw[i] = 0.0;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __syncthreads();
  double ybq[4], ybv[3];
  load_state(m, ro, a.xbar + st_xoff(a, w), ybq, ybv);
  double tau[3] = {0, 0, 0}, tbacc[3] = {0, 0, 0};
  int cur_k = -1;
  StackStat st{};
  auto flush_ubar = [&](int kk) {
    if (!ubw || !ro.dof) return;
    for (int i = 0; i < m.nu; ++i) {
      const int d = m.ctrl[i] - 6 * ro.b - 3 * ro.half;
      if (d >= 0 && d < 3) {
        double g = 0.0;
#pragma unroll
        for (int j = 0; j < 3; ++j) if (j == d) g = tbacc[j];
        ubw[(size_t)kk * m.nu + i] += g;
      }
    }
  };
  for (int s = nsteps - 1; s >= 0; --s) {
    const double* r = tape_w + (size_t)s * rec;
    const double h = r[1];
    const int kk = (int)r[2];
    if (ro.lane == 0) st.u_step++;
    if (kk != cur_k) {
      if (cur_k >= 0) flush_ubar(cur_k);
      cur_k = kk;
      stack_tau(m, ro, uw, kk, tau);
#pragma unroll
      for (int j = 0; j < 3; ++j) tbacc[j] = 0.0;
    }
    double yq[4], yv[3];
    load_state(m, ro, r + 3, yq, yv);
    double A[7][3], Ab[7][3];
#pragma unroll
    for (int i = 0; i < 7; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) { A[i][j] = 0.0; Ab[i][j] = 0.0; }
    if constexpr (RECOMPUTE) {
#pragma unroll 1
      for (int i = 0; i < 6; ++i) {
        double Yq[4], Yv[3], dq[3], ai[3], xw[3];
        if (i == 0) {
#pragma unroll
          for (int j = 0; j < 4; ++j) Yq[j] = yq[j];
#pragma unroll
          for (int j = 0; j < 3; ++j) Yv[j] = yv[j];
        } else {
          stack_stage(ro, yq, yv, A, i, h, Yq, Yv, dq);
        }
        const int prev = i > 0 ? i - 1 : 0;
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          double v = A[0][j];
#pragma unroll
          for (int l = 1; l < 6; ++l) v = (l == prev) ? A[l][j] : v;
          xw[j] = v;
        }
        stack_acc(m, S, ro, Yq, Yv, tau, false, o.beta, o.newton_maxit, i > 0 ? xw : nullptr, ai, st);
#pragma unroll
        for (int l = 0; l < 6; ++l)
#pragma unroll
          for (int j = 0; j < 3; ++j) A[l][j] = (l == i) ? ai[j] : A[l][j];
      }
    } else if (ro.dof) {
#pragma unroll
      for (int l = 0; l < 6; ++l)
#pragma unroll
        for (int j = 0; j < 3; ++j) A[l][j] = r[3 + NX + 6 * m.k * l + a_index(ro, j)];
    }
    double qb[4] = {0, 0, 0, 0}, vb[3] = {0, 0, 0};
    double Yb_q[4], Yb_v[3];
#pragma unroll
    for (int j = 0; j < 4; ++j) Yb_q[j] = ybq[j];
#pragma unroll
    for (int j = 0; j < 3; ++j) Yb_v[j] = ybv[j];
#pragma unroll 1
    for (int i = 6; i >= 0; --i) {
      double Yq[4], Yv[3], dq[3] = {0, 0, 0};
      if (i > 0) {
        stack_stage(ro, yq, yv, A, i, h, Yq, Yv, dq);
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) Yq[j] = yq[j];
#pragma unroll
        for (int j = 0; j < 3; ++j) Yv[j] = yv[j];
      }
      if (i < 6) {
        double xs[3], abi[3], tb[3];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          double v = 0.0, g = 0.0;
#pragma unroll
          for (int l = 0; l < 6; ++l) { v = (l == i) ? A[l][j] : v; g = (l == i) ? Ab[l][j] : g; }
          xs[j] = v;
          abi[j] = g;
        }
        stack_acc_vjp(m, S, ro, Yq, Yv, tau, xs, abi, o.cfd != 0, o.beta, o.newton_maxit, Yb_q, Yb_v, tb, st);
#pragma unroll
        for (int j = 0; j < 3; ++j) tbacc[j] += tb[j];
      }
      if (i == 0) {
#pragma unroll
        for (int j = 0; j < 4; ++j) qb[j] += Yb_q[j];
#pragma unroll
        for (int j = 0; j < 3; ++j) vb[j] += Yb_v[j];
      } else {
        double dqb[3];
        stack_qplus_vjp(ro, yq, dq, Yb_q, qb, dqb);
        const StageCoef k = stage_coef(i);
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          vb[j] += Yb_v[j] + h * k.c * dqb[j];
#pragma unroll
          for (int l = 0; l < 6; ++l) Ab[l][j] += h * k.a[l] * Yb_v[j] + h * h * k.a2[l] * dqb[j];
        }
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) ybq[j] = qb[j];
#pragma unroll
    for (int j = 0; j < 3; ++j) ybv[j] = vb[j];
  }
  if (cur_k >= 0) flush_ubar(cur_k);
  store_state(m, ro, x0b, ybq, ybv);
  if (a.adj_counters) {
    double c[kAdjCounters] = {(double)st.u_step, (double)st.u_vjp, (double)st.u_vcon, (double)st.u_vedge};
    wave_sum<kAdjCounters>(c);
    if (ro.lane == 0)
      for (int i = 0; i < kAdjCounters; ++i) a.adj_counters[(size_t)w * kAdjCounters + i] = (long long)c[i];
  }
}

template <bool RECOMPUTE>
__global__ void __launch_bounds__(64) stack_adj_kernel(StackArgs a) {
  __shared__ StackLds S;
  for (bool first = true;; first = false) {
    const int w = stack_take(a, nullptr, first);
    if (w < 0) break;
    stack_adj_world<RECOMPUTE>(st_model(a, w), S, a, w);
  }
}

}  // namespace dmx
