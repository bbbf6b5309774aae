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
// impedances) and on the velocities through aref = -b J_e v + ...  Each pair
// lane reverses Phi over its own contacts: the partials of Phi in the edge
// projections, depth and impedance, then the frame, the lever arms and the
// world twists, then the contact's construction (its code) back to the two
// body poses (centre c_b, rotation R_b).  A body-frame rotation
// R <- R exp([theta]x) moves Phi by theta . (G21 - G12, G02 - G20, G10 - G01)
// with G = R^T R_bar.
#pragma once
#include "dmx_stack_rk.hpp"

namespace dmx {

// cotangents of one pair lane's bodies: pose (c_bar, R_bar) and generalized
// velocity (linear, body-frame angular)
struct PairBar {
  V3 c1, c2;
  double R1[9], R2[9];
  double v1[6], v2[6];
};

// Reverse of Phi over contact c of this pair lane (active edges `act`) into
// pb; S.vec[kVecD / kVecX / kVecV] hold the generalized lambda, x*, v.
// hp (optional, [kParams]): += the contact parameters' cotangents (friction,
// solref, solimp, one value for every pair of the world).
DMX_DEV void contact_phi_vjp(const StackModel& m, const StackLds& S, const StackRole& ro, const PairSlots& ps,
                             int j, unsigned act, bool cfd, double beta, PairBar& pb, double* hp = nullptr) {
  const int b1 = ro.pb1, b2 = ro.pb2, c = ps.off + j;
  const bool two = b1 >= 0;
  const double ahat = ps.ahat;
  const V3 p = mk3(S.cp[0][c], S.cp[1][c], S.cp[2][c]);
  const V3 n = ps.n;
  const double r = S.cr[c];
  V3 t1, t2;
  make_frame(n, &t1, &t2);
  const V3 c2 = ld3(S.P[b2]);
  const V3 c1 = two ? ld3(S.P[b1]) : mk3(0.0, 0.0, 0.0);
  const V3 r2 = p - c2, r1 = p - c1;
  const M3& R2 = *(const M3*)S.R[b2];
  const M3& R1 = *(const M3*)S.R[two ? b1 : b2];
  // relative contact velocity of lambda, x*, v (index kVec*)
  V3 om2[3], om1[3], u[3];
#pragma unroll
  for (int g = 0; g < 3; ++g) {
    const double* w2 = S.vec[g][b2];
    om2[g] = mul(R2, mk3(w2[3], w2[4], w2[5]));
    u[g] = mk3(w2[0], w2[1], w2[2]) + cross(om2[g], r2);
    om1[g] = mk3(0.0, 0.0, 0.0);
    if (two) {
      const double* w1 = S.vec[g][b1];
      om1[g] = mul(R1, mk3(w1[3], w1[4], w1[5]));
      u[g] -= mk3(w1[0], w1[1], w1[2]) + cross(om1[g], r1);
    }
  }
  double ddr;
  const double d = stack_imp(m, r, &ddr);
  const double D = d / (ahat * (1.0 - d));
  const double dDdd = 1.0 / (ahat * (1.0 - d) * (1.0 - d));
  double pterm, dpdr, ptd;  // ptd: d pterm / d(impedance) / kscale
  if (cfd) {
    double dsp;
    const double sp = stack_softplus(-r, beta, &dsp);
    pterm = d * m.kscale * sp;
    dpdr = m.kscale * (ddr * sp - d * dsp);
    ptd = sp;
  } else {
    pterm = -d * m.kscale * r;
    dpdr = -m.kscale * (ddr * r + d);
    ptd = -r;
  }
  double mub = 0.0, bb = 0.0;  // friction and damping-coefficient cotangents
  V3 ub[3] = {mk3(0.0, 0.0, 0.0), mk3(0.0, 0.0, 0.0), mk3(0.0, 0.0, 0.0)};
  V3 nb = mk3(0.0, 0.0, 0.0), t1b = mk3(0.0, 0.0, 0.0), t2b = mk3(0.0, 0.0, 0.0);
  double Pbar = 0.0, Dbar = 0.0;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    if (!((act >> e) & 1u)) continue;
    const double sg = (e & 1) ? -m.mu : m.mu;
    const V3 de = n + sg * (e < 2 ? t1 : t2);
    const double L = dot(de, u[kVecD]), X = dot(de, u[kVecX]), Vv = dot(de, u[kVecV]);
    const double res = pterm - m.bcoef * Vv - X;  // aref_e - J_e x*
    const double Lb = D * res, Xb = -D * L, Vb = -m.bcoef * D * L;
    Pbar += D * L;
    Dbar += L * res;
    ub[kVecD] += Lb * de;
    ub[kVecX] += Xb * de;
    ub[kVecV] += Vb * de;
    const V3 deb = Lb * u[kVecD] + Xb * u[kVecX] + Vb * u[kVecV];
    nb += deb;
    if (e < 2) t1b += sg * deb; else t2b += sg * deb;
    if (hp) {
      const double tdeb = dot(e < 2 ? t1 : t2, deb);
      mub += (e & 1) ? -tdeb : tdeb;  // the edge direction n +- mu t
      bb -= D * L * Vv;
    }
  }
  if (hp) {
    // friction also through D (A-hat = (1 + mu^2) w); solref through a_ref's
    // b = 2 / (dwidth t_c) and k = 1 / (dwidth^2 t_c^2 dr^2); solimp through
    // d(r) in D and the position term, dwidth also through b and k
    const double dw = m.si[1];
    const double tc = 2.0 / (dw * m.bcoef);
    const double dr = 1.0 / (dw * tc * sqrt(m.kscale));
    const double kb = Pbar * d * ptd;
    const double sb = m.bcoef * bb + 2.0 * m.kscale * kb;
    hp[3] += mub + Dbar * (-2.0 * m.mu * D / (1.0 + m.mu * m.mu));
    hp[4] -= sb / tc;
    hp[5] -= 2.0 * m.kscale * kb / dr;
    const double dbar = Dbar * dDdd + Pbar * m.kscale * ptd;
    double gs[5];
    stack_imp_solimp_grad(m, r, gs);
#pragma unroll
    for (int i = 0; i < 5; ++i) hp[7 + i] += dbar * gs[i];
    hp[8] -= sb / dw;
  }
  const double rb = Pbar * dpdr + Dbar * dDdd * ddr;
  nb += make_frame_vjp(n, t1b, t2b);
  // u_g = v_g2 + om_g2 x r2 - (v_g1 + om_g1 x r1), om_gb = R_b w_gb
  V3 r2b = mk3(0.0, 0.0, 0.0), r1b = mk3(0.0, 0.0, 0.0);
#pragma unroll
  for (int g = 0; g < 3; ++g) {
    r2b += cross(ub[g], om2[g]);
    const V3 o2 = cross(r2, ub[g]);
    const double* w2 = S.vec[g][b2];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const double oi = i == 0 ? o2.x : (i == 1 ? o2.y : o2.z);
#pragma unroll
      for (int j = 0; j < 3; ++j) pb.R2[3 * i + j] += oi * w2[3 + j];
    }
    if (two) {
      r1b -= cross(ub[g], om1[g]);
      const V3 o1 = cross(r1, ub[g]);
      const double* w1 = S.vec[g][b1];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        const double oi = i == 0 ? o1.x : (i == 1 ? o1.y : o1.z);
#pragma unroll
        for (int j = 0; j < 3; ++j) pb.R1[3 * i + j] -= oi * w1[3 + j];
      }
    }
  }
  // velocity cotangents: the generalized v enters through u_V only
  {
    const V3 f = ub[kVecV];
    const V3 m2 = mulT(R2, cross(r2, f));
    pb.v2[0] += f.x; pb.v2[1] += f.y; pb.v2[2] += f.z; pb.v2[3] += m2.x; pb.v2[4] += m2.y; pb.v2[5] += m2.z;
    if (two) {
      const V3 m1 = mulT(R1, cross(r1, f));
      pb.v1[0] -= f.x; pb.v1[1] -= f.y; pb.v1[2] -= f.z; pb.v1[3] -= m1.x; pb.v1[4] -= m1.y; pb.v1[5] -= m1.z;
    }
  }
  // r_b = p - c_b
  const V3 pbar = r2b + r1b;
  pb.c2 -= r2b;
  if (two) pb.c1 -= r1b;
  if (two) box_box_vjp(m.h, m.h, c1, R1, c2, R2, S.code[c], rb, pbar, nb, &pb.c1, pb.R1, &pb.c2, pb.R2);
  else box_plane_vjp(m.h, m.p0, m.pn, c2, R2, S.code[c], rb, pbar, &pb.c2, pb.R2);
}

// pose cotangent (translation, body-frame rotation) from c_bar and R_bar
DMX_DEV void pose_bar(const double* R, V3 cb, const double* Rb, double* out) {
  double G[9];
  m3_RtA(R, Rb, G);
  out[0] = cb.x; out[1] = cb.y; out[2] = cb.z;
  out[3] = G[7] - G[5];
  out[4] = G[2] - G[6];
  out[5] = G[3] - G[1];
}

// VJP of the acceleration map at this lane's stage state (yq, yv) with the
// stage acceleration xs (unless cfd: then the contacts-from-distance field's
// own acceleration, solved here) and the cotangent ab: cotangents of the
// state (qb: 3 or 4, vb: 3) and of this lane's generalized forces (tb).
// hp (optional, [kParams]): += this lane's share of the model parameters'
// cotangents (contact parameters on pair lanes; the cubes' common mass on dof
// lanes: inertia, bias and D all scale with it, so m_bar = -lam . tau / m).
DMX_DEV void stack_acc_vjp(const StackModel& m, StackLds& S, const StackRole& ro, const double* yq,
                           const double* yv, const double* tau, const double* xs_in, const double* ab, bool cfd,
                           double beta, int maxit, double* qb, double* vb, double* tb, StackStat& st,
                           double* hp = nullptr) {
  PairSlots ps = stack_setup(m, S, ro, yq, yv, cfd, st, true);
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
  assemble(m, S, ro, ps, cfd, beta, xs, a0);
  if (ro.lane == 0) st.u_vjp++;
  if (ro.pair) { st.u_vedge += __popc(ps.act); for (int j = 0; j < ps.cnt; ++j) st.u_vcon += ((ps.act >> (4 * j)) & 15u) != 0u; }
  if (ro.dof) {
#pragma unroll
    for (int j = 0; j < 3; ++j) S.gv[ro.b][3 * ro.half + j] = ab[j];
  }
  wave_fence();
  if (!block_factor_solve(S, m.k)) st.status |= 4;
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
  // pair lanes: Phi reversed over their contacts
  PairBar pb;
  pb.c1 = mk3(0.0, 0.0, 0.0);
  pb.c2 = mk3(0.0, 0.0, 0.0);
#pragma unroll
  for (int i = 0; i < 9; ++i) { pb.R1[i] = 0.0; pb.R2[i] = 0.0; }
#pragma unroll
  for (int i = 0; i < 6; ++i) { pb.v1[i] = 0.0; pb.v2[i] = 0.0; }
  if (ro.pair) {
    for (int j = 0; j < ps.cnt; ++j) {
      const unsigned a = (ps.act >> (4 * j)) & 15u;
      if (a) contact_phi_vjp(m, S, ro, ps, j, a, cfd, beta, pb, hp);
    }
  }
  double pose1[6] = {0, 0, 0, 0, 0, 0}, pose2[6] = {0, 0, 0, 0, 0, 0};
  if (ro.pair) pose_bar(S.R[ro.pb2], pb.c2, pb.R2, pose2);
  if (ro.pair == 2) pose_bar(S.R[ro.pb1], pb.c1, pb.R1, pose1);
  // gather per body in a fixed order: plane pair, then the body's share of
  // the box pair above it, then of the box pair below it (S.gv: pose
  // cotangent, S.Hd[b][0..5]: velocity cotangent)
  if (ro.pair == 1) {
#pragma unroll
    for (int i = 0; i < 6; ++i) { S.gv[ro.pb2][i] = pose2[i]; S.Hd[ro.pb2][i] = pb.v2[i]; }
  }
  wave_fence();
  if (ro.pair == 2) {
#pragma unroll
    for (int i = 0; i < 6; ++i) { S.gv[ro.pb1][i] += pose1[i]; S.Hd[ro.pb1][i] += pb.v1[i]; }
  }
  wave_fence();
  if (ro.pair == 2) {
#pragma unroll
    for (int i = 0; i < 6; ++i) { S.gv[ro.pb2][i] += pose2[i]; S.Hd[ro.pb2][i] += pb.v2[i]; }
  }
  wave_fence();
#pragma unroll
  for (int j = 0; j < 4; ++j) qb[j] = 0.0;
#pragma unroll
  for (int j = 0; j < 3; ++j) { vb[j] = 0.0; tb[j] = 0.0; }
  if (ro.dof) {
    const double* pg = S.gv[ro.b];
    const double* vg = S.Hd[ro.b];
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
    if (hp) hp[6] -= (lam[0] * tau[0] + lam[1] * tau[1] + lam[2] * tau[2]) * m.imass;
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

// PAR: the model parameters' cotangents are accumulated and stored to a.pbar
// (a template flag: the plain reverse sweep carries none of their registers).
template <bool RECOMPUTE, bool PAR = false>
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
    if (PAR && ro.lane < kParams) a.pbar[(size_t)w * kParams + ro.lane] = nan;
    return;
  }
  // this lane's share of the model parameters' cotangents, summed over all
  // stages and steps (one wavefront sum at the end)
  double hacc[PAR ? kParams : 1];
#pragma unroll
  for (int i = 0; i < (PAR ? kParams : 1); ++i) hacc[i] = 0.0;
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
        stack_acc_vjp(m, S, ro, Yq, Yv, tau, xs, abi, o.cfd != 0, o.beta, o.newton_maxit, Yb_q, Yb_v, tb, st,
                      PAR ? hacc : nullptr);
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
  if constexpr (PAR) {
    wave_sum<kParams>(hacc);
    // the cubes' half sizes are not differentiated in stack worlds
    hacc[0] = hacc[1] = hacc[2] = __longlong_as_double(0x7ff8000000000000ll);
#pragma unroll
    for (int i = 0; i < kParams; ++i)
      if (ro.lane == i) a.pbar[(size_t)w * kParams + i] = hacc[i];
  }
  if (a.adj_counters) {
    double c[kAdjCounters] = {(double)st.u_step, (double)st.u_vjp, (double)st.u_vcon, (double)st.u_vedge};
    wave_sum<kAdjCounters>(c);
    if (ro.lane == 0)
      for (int i = 0; i < kAdjCounters; ++i) a.adj_counters[(size_t)w * kAdjCounters + i] = (long long)c[i];
  }
}

template <bool RECOMPUTE, bool PAR = false>
__global__ void __launch_bounds__(64) stack_adj_kernel(StackArgs a) {
  __shared__ StackLds S;
  for (bool first = true;; first = false) {
    const int w = stack_take(a, nullptr, first);
    if (w < 0) break;
    stack_adj_world<RECOMPUTE, PAR>(st_model(a, w), S, a, w);
  }
}

// Forward rollout and reverse sweep of each world in one persistent launch,
// for a final-state cotangent given before the rollout: a wavefront that has
// finished a world's forward rollout runs that world's reverse sweep on the
// tape it has just written, so the launch lasts as long as the slowest world's
// forward plus reverse rather than the slowest forward plus the slowest
// reverse (worlds differ by orders of magnitude in work, App. D).
template <bool RECOMPUTE>
__global__ void __launch_bounds__(64) stack_grad_kernel(StackArgs a) {
  __shared__ StackLds S;
  for (bool first = true;; first = false) {
    const int w = stack_take(a, nullptr, first);
    if (w < 0) break;
    const StackModel& m = st_model(a, w);
    stack_fwd_world(m, S, a, w);
    // the tape records, step count and status just stored by the lanes are
    // read back by other lanes of the wavefront
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    stack_adj_world<RECOMPUTE>(m, S, a, w);
  }
}

}  // namespace dmx
