// Oracle simulator (TEST INFRASTRUCTURE ONLY; see orc_api.h).
//
// Plain scalar FP64 code, written for readability against the paper rather
// than speed.  Each routine cites the passage it follows.  Where the paper is
// silent the oracle takes one stated reading (named "reading:" below); the
// HIP library implements the same readings independently.
#include "orc_api.h"
#include "orc_math.hpp"

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <thread>
#include <vector>

namespace orc {

constexpr double kPi = 3.14159265358979323846;
constexpr int kDir = 16;  // tangent directions per forward-mode pass
using DualT = Dual<kDir>;

inline void set_val(double& x, double v) { x = v; }
template <int N> inline void set_val(Dual<N>& x, double v) { x.v = v; }
inline void set_val(Flop& x, double v) { x.v = v; }
// scalar of the value-only parts (Newton iterations, error estimate): double,
// or the counting scalar when the rollout is counted
template <class S> struct ValueOf { using type = double; };
template <> struct ValueOf<Flop> { using type = Flop; };
// a value-only result back in the rollout's scalar
template <class S> struct FromValue { static S get(double x) { return S(x); } };
template <> struct FromValue<Flop> { static Flop get(const Flop& x) { return x; } };
template <class S> inline bool is_dual() { return false; }
template <> inline bool is_dual<DualT>() { return true; }

enum { J_FREE = 0, J_HINGE = 1, J_SLIDE = 2 };
enum { G_PLANE = 0, G_SPHERE = 1, G_CAPSULE = 2, G_BOX = 3 };

// ------------------------------------------------------------------ model
struct Model {
  int nb = 0, nj = 0, ng = 0, np = 0, nu = 0, nq = 0, nv = 0, ncmax = 0;
  std::vector<int> bparent, bjnt0, bjntn;
  std::vector<V3<double>> bpos;
  std::vector<Q4<double>> bquat;
  std::vector<double> bmass, binvw;
  std::vector<M3<double>> biner;
  std::vector<int> jbody, jtype, jqadr, jdadr;
  std::vector<V3<double>> jaxis, jpos;
  std::vector<int> gbody, gtype;
  std::vector<V3<double>> gsize, gpos;
  std::vector<Q4<double>> gquat;
  std::vector<int> pg1, pg2, pncon, pcadr;
  std::vector<double> pmu, psolref, psolimp, pcfd;
  std::vector<int> ctrl;
  V3<double> grav;
  std::vector<std::vector<int>> bdofs;  // dofs that move body b (its joints and its ancestors'), ascending
};

// Solid primitive of uniform density: mass and the principal inertia about its
// centre.  reading: density 1000 kg/m^3 where no mass is given; the body's
// centre of mass is its origin (no joint armature, damping or limits).
static void primitive_inertia(int type, const double* sz, double mass_in, double* mass, double* I) {
  double vol = 0.0;
  if (type == G_SPHERE) vol = 4.0 / 3.0 * kPi * sz[0] * sz[0] * sz[0];
  if (type == G_BOX) vol = 8.0 * sz[0] * sz[1] * sz[2];
  if (type == G_CAPSULE) vol = kPi * sz[0] * sz[0] * 2.0 * sz[1] + 4.0 / 3.0 * kPi * sz[0] * sz[0] * sz[0];
  double m = mass_in > 0.0 ? mass_in : 1000.0 * vol;
  *mass = m;
  if (type == G_SPHERE) {
    I[0] = I[1] = I[2] = 0.4 * m * sz[0] * sz[0];
  } else if (type == G_BOX) {
    I[0] = m / 3.0 * (sz[1] * sz[1] + sz[2] * sz[2]);
    I[1] = m / 3.0 * (sz[0] * sz[0] + sz[2] * sz[2]);
    I[2] = m / 3.0 * (sz[0] * sz[0] + sz[1] * sz[1]);
  } else {  // capsule along z: cylinder of length H plus two hemispherical caps
    double r = sz[0], H = 2.0 * sz[1];
    double vc = kPi * r * r * H, vs = 4.0 / 3.0 * kPi * r * r * r;
    double mc = m * vc / (vc + vs), ms = m * vs / (vc + vs);
    I[2] = mc * r * r / 2.0 + ms * 0.4 * r * r;
    I[0] = I[1] = mc * (r * r / 4.0 + H * H / 12.0) + ms * (0.4 * r * r + H * H / 4.0 + 3.0 * H * r / 8.0);
  }
}

template <class S>
struct Kin {
  std::vector<V3<S>> xpos, jax, janc, w, vel, alp, acc, gpos;
  std::vector<M3<S>> xmat, gmat;
};

// ------------------------------------------------------------------ kinematics
// Forward kinematics along the tree (Sec. 2: "recursive multi-body
// algorithms"), MuJoCo joint conventions: a free joint's q is the world
// position and the unit quaternion (w,x,y,z) of the body, its velocity the
// world linear velocity of the body origin and the angular velocity in the
// body frame; hinges rotate about their anchor, slides translate along their
// axis; joints of one body apply in order.  With v given, body angular
// velocities, origin velocities, and the accelerations they would have at
// zero joint acceleration are propagated (rigid-body velocity and
// acceleration transfer).
template <class S>
static void kinematics(const Model& m, const S* q, const S* v, Kin<S>& k) {
  k.xpos.assign(m.nb, vzero<S>()); k.xmat.assign(m.nb, eye3<S>());
  k.jax.assign(m.nj, vzero<S>()); k.janc.assign(m.nj, vzero<S>());
  k.w.assign(m.nb, vzero<S>()); k.vel.assign(m.nb, vzero<S>());
  k.alp.assign(m.nb, vzero<S>()); k.acc.assign(m.nb, vzero<S>());
  for (int b = 0; b < m.nb; ++b) {
    int pa = m.bparent[b];
    V3<S> pp = vzero<S>(), wp = vzero<S>(), vp = vzero<S>(), ap = vzero<S>(), cp = vzero<S>();
    M3<S> Rp = eye3<S>();
    if (pa >= 0) { pp = k.xpos[pa]; Rp = k.xmat[pa]; wp = k.w[pa]; vp = k.vel[pa]; ap = k.alp[pa]; cp = k.acc[pa]; }
    V3<S> p = add(pp, matvec(Rp, lift<S>(m.bpos[b])));
    Q4<S> bq; bq.w = S(m.bquat[b].w); bq.x = S(m.bquat[b].x); bq.y = S(m.bquat[b].y); bq.z = S(m.bquat[b].z);
    M3<S> R = matmul(Rp, qmat(bq));
    V3<S> r = sub(p, pp);
    V3<S> w = wp, vv = add(vp, cross(wp, r)), al = ap;
    V3<S> ac = add(cp, add(cross(ap, r), cross(wp, cross(wp, r))));
    for (int j = m.bjnt0[b]; j < m.bjnt0[b] + m.bjntn[b]; ++j) {
      int qa = m.jqadr[j], da = m.jdadr[j];
      if (m.jtype[j] == J_FREE) {
        p = v3<S>(q[qa], q[qa + 1], q[qa + 2]);
        Q4<S> qq; qq.w = q[qa + 3]; qq.x = q[qa + 4]; qq.y = q[qa + 5]; qq.z = q[qa + 6];
        R = qmat(qnormalize(qq));  // reading: FK normalizes the quaternion
        k.jax[j] = col(R, 2); k.janc[j] = p;
        if (v) {
          vv = v3<S>(v[da], v[da + 1], v[da + 2]);
          w = matvec(R, v3<S>(v[da + 3], v[da + 4], v[da + 5]));
          al = vzero<S>(); ac = vzero<S>();
        }
      } else if (m.jtype[j] == J_HINGE) {
        V3<S> o = add(p, matvec(R, lift<S>(m.jpos[j])));
        V3<S> a = matvec(R, lift<S>(m.jaxis[j]));
        k.jax[j] = a; k.janc[j] = o;
        V3<S> va = vzero<S>(), aa = vzero<S>(), wn = vzero<S>(), aln = vzero<S>();
        if (v) {
          V3<S> rr = sub(o, p);
          va = add(vv, cross(w, rr));
          aa = add(ac, add(cross(al, rr), cross(w, cross(w, rr))));
          V3<S> wj = scale(a, v[da]);
          wn = add(w, wj);
          aln = add(al, cross(w, wj));
        }
        R = matmul(R, axis_rot<S>(m.jaxis[j], q[qa]));
        p = sub(o, matvec(R, lift<S>(m.jpos[j])));
        if (v) {
          V3<S> rp = sub(p, o);
          vv = add(va, cross(wn, rp));
          ac = add(aa, add(cross(aln, rp), cross(wn, cross(wn, rp))));
          w = wn; al = aln;
        }
      } else {  // slide
        V3<S> a = matvec(R, lift<S>(m.jaxis[j]));
        k.jax[j] = a; k.janc[j] = add(p, matvec(R, lift<S>(m.jpos[j])));
        V3<S> rr = scale(a, q[qa]);
        if (v) {
          V3<S> as = scale(a, v[da]);
          ac = add(ac, add(add(cross(al, rr), cross(w, cross(w, rr))), scale(cross(w, as), 2.0)));
          vv = add(vv, add(cross(w, rr), as));
        }
        p = add(p, rr);
      }
    }
    k.xpos[b] = p; k.xmat[b] = R; k.w[b] = w; k.vel[b] = vv; k.alp[b] = al; k.acc[b] = ac;
  }
  k.gpos.assign(m.ng, vzero<S>()); k.gmat.assign(m.ng, eye3<S>());
  for (int g = 0; g < m.ng; ++g) {
    Q4<S> gq; gq.w = S(m.gquat[g].w); gq.x = S(m.gquat[g].x); gq.y = S(m.gquat[g].y); gq.z = S(m.gquat[g].z);
    int b = m.gbody[g];
    if (b < 0) { k.gpos[g] = lift<S>(m.gpos[g]); k.gmat[g] = qmat(gq); }
    else { k.gpos[g] = add(k.xpos[b], matvec(k.xmat[b], lift<S>(m.gpos[g]))); k.gmat[g] = matmul(k.xmat[b], qmat(gq)); }
  }
}

// Jacobian of the world velocity of a point attached to body b (3 x nv,
// row-major) and of the body's world angular velocity (may be null).
template <class S>
static void point_jac(const Model& m, const Kin<S>& k, int b, const V3<S>& P, S* Jp, S* Jr) {
  for (int i = 0; i < 3 * m.nv; ++i) { Jp[i] = S(0.0); if (Jr) Jr[i] = S(0.0); }
  for (; b >= 0; b = m.bparent[b]) {
    for (int j = m.bjnt0[b]; j < m.bjnt0[b] + m.bjntn[b]; ++j) {
      int d = m.jdadr[j];
      if (m.jtype[j] == J_FREE) {
        V3<S> rel = sub(P, k.xpos[b]);
        for (int i = 0; i < 3; ++i) {
          Jp[i * m.nv + d + i] = S(1.0);
          V3<S> e = col(k.xmat[b], i);
          V3<S> cv = cross(e, rel);
          for (int r = 0; r < 3; ++r) {
            Jp[r * m.nv + d + 3 + i] = cv.x[r];
            if (Jr) Jr[r * m.nv + d + 3 + i] = e.x[r];
          }
        }
      } else if (m.jtype[j] == J_HINGE) {
        V3<S> cv = cross(k.jax[j], sub(P, k.janc[j]));
        for (int r = 0; r < 3; ++r) { Jp[r * m.nv + d] = cv.x[r]; if (Jr) Jr[r * m.nv + d] = k.jax[j].x[r]; }
      } else {
        for (int r = 0; r < 3; ++r) Jp[r * m.nv + d] = k.jax[j].x[r];
      }
    }
  }
}

// Joint-space inertia M(q) and bias c(q, v) of the equation of motion (Sec. 2,
// eq. EOM).  M is written out from its definition, the kinetic energy
// T = 1/2 v^T M v summed over bodies; c is the Newton-Euler bias (velocity
// products and gravity) projected by the same body Jacobians.
template <class S>
static void mass_bias(const Model& m, const Kin<S>& k, S* M, S* c) {
  int nv = m.nv;
  for (int i = 0; i < nv * nv; ++i) M[i] = S(0.0);
  for (int i = 0; i < nv; ++i) c[i] = S(0.0);
  std::vector<S> Jp(3 * nv), Jr(3 * nv);
  for (int b = 0; b < m.nb; ++b) {
    point_jac(m, k, b, k.xpos[b], Jp.data(), Jr.data());
    M3<S> Iw = matmul(matmul(k.xmat[b], liftm<S>(m.biner[b])), transpose(k.xmat[b]));
    double mb = m.bmass[b];
    // M += m Jp^T Jp + Jr^T Iw Jr (the body's Jacobians vanish outside the
    // dofs that move it)
    for (int i : m.bdofs[b])
      for (int j : m.bdofs[b]) {
        S s = S(0.0);
        for (int r = 0; r < 3; ++r) s += Jp[r * nv + i] * Jp[r * nv + j] * mb;
        for (int r = 0; r < 3; ++r)
          for (int t = 0; t < 3; ++t) s += Jr[r * nv + i] * Iw.a[r][t] * Jr[t * nv + j];
        M[i * nv + j] += s;
      }
    V3<S> f = scale(sub(k.acc[b], lift<S>(m.grav)), mb);
    V3<S> tq = add(matvec(Iw, k.alp[b]), cross(k.w[b], matvec(Iw, k.w[b])));
    for (int i : m.bdofs[b])
      for (int r = 0; r < 3; ++r) c[i] += Jp[r * nv + i] * f.x[r] + Jr[r * nv + i] * tq.x[r];
  }
}

// ------------------------------------------------------------------ collision
template <class S>
struct Contact {
  S r;
  V3<S> pos, n, t1, t2;
  int pair;
};

// reading: tangent t1 = normalized (a - (a.n) n) with a = e_x unless |n_x| >= 0.5
// (then e_y), t2 = n x t1.
template <class S>
static void make_frame(const V3<S>& n, V3<S>& t1, V3<S>& t2) {
  V3<S> a = std::fabs(val(n.x[0])) < 0.5 ? v3<S>(S(1.0), S(0.0), S(0.0)) : v3<S>(S(0.0), S(1.0), S(0.0));
  V3<S> t = sub(a, scale(n, dot(a, n)));
  t1 = scale(t, 1.0 / sqrt_(dot(t, t)));
  t2 = cross(n, t1);
}

// sphere of centre c, radius rs vs a plane: signed distance r (< 0 in
// penetration, Sec. 2.1) and the midpoint between the surfaces.
template <class S>
static Contact<S> sphere_plane(const V3<S>& p0, const V3<S>& n, const V3<S>& c, double rs, int pair) {
  Contact<S> ct;
  ct.r = dot(n, sub(c, p0)) - rs;
  ct.pos = sub(c, scale(n, ct.r * 0.5 + rs));
  ct.n = n;
  make_frame(n, ct.t1, ct.t2);
  ct.pair = pair;
  return ct;
}

template <class S> static S smoothstep01(S t) {
  if (val(t) <= 0.0) return S(0.0);
  if (val(t) >= 1.0) return S(1.0);
  return t * t * (3.0 - 2.0 * t);
}

// Plane-box contacts by the smoothed four-deepest-vertex rule of App. C.1,
// where the paper replaces the hard case split of plane-box detection by a
// soft selection.  Stated in the world frame: vertex k sits at
// x_k = c + R s_k (s_k the half-size corner with coordinate signs from the
// bits of k: x bit 0, y bit 1, z bit 2) and penetrates the plane by
// e_k = -n.(x_k - p0).  Vertices within a 1 mm skin of the deepest one keep
// their depth: with the threshold tau = max(0, e_max - 1e-3), the weight w_k
// rises smoothly from 0 at depth tau - 1e-3 to 1 at tau (reading: the C^1
// smoothstep t^2 (3 - 2t) for the unnamed sigmoid), and the contacts are the
// four largest weighted depths z_k = w_k e_k (reading: equal values go to the
// lower vertex index), each with signed distance r = -z_k and its point
// halfway between the vertex and the plane, x_k + (z_k / 2) n.  A vertex
// whose weighted depth is 0 gives an inactive contact (r = 0).
template <class S>
static void box_plane(const V3<S>& p0, const V3<S>& nw, const V3<S>& c, const M3<S>& R, const V3<double>& hs,
                      int pair, std::vector<Contact<S>>& out) {
  V3<S> x[8];
  S depth[8];
  for (int k = 0; k < 8; ++k) {
    V3<double> s = v3<double>((k & 1) ? hs.x[0] : -hs.x[0], (k & 2) ? hs.x[1] : -hs.x[1],
                              (k & 4) ? hs.x[2] : -hs.x[2]);
    x[k] = add(c, matvec(R, lift<S>(s)));
    depth[k] = S(0.0) - dot(nw, sub(x[k], p0));
  }
  double emax = val(depth[0]);
  int kmax = 0;
  for (int k = 1; k < 8; ++k)
    if (val(depth[k]) > emax) { emax = val(depth[k]); kmax = k; }
  const double skin = 1e-3;
  S tau = emax > skin ? depth[kmax] - skin : S(0.0);
  S z[8];
  for (int k = 0; k < 8; ++k) {
    S w = smoothstep01((depth[k] - (tau - skin)) / skin);
    z[k] = w * depth[k];
  }
  // rank by weighted depth, deepest first; equal values keep vertex order
  std::vector<int> order = {0, 1, 2, 3, 4, 5, 6, 7};
  std::sort(order.begin(), order.end(), [&](int a, int b) {
    return val(z[a]) > val(z[b]) || (val(z[a]) == val(z[b]) && a < b);
  });
  for (int i = 0; i < 4; ++i) {
    const int k = order[i];
    Contact<S> ct;
    ct.r = S(0.0) - z[k];
    ct.pos = add(x[k], scale(nw, z[k] * 0.5));
    ct.n = nw;
    make_frame(nw, ct.t1, ct.t2);
    ct.pair = pair;
    out.push_back(ct);
  }
}

template <class S> static S sabs(const S& x) { return val(x) < 0.0 ? S(0.0) - x : x; }

// Box-box contacts.  reading (the paper names primitive-vs-primitive
// detection in Sec. 2.1 but prints no box-box routine): the separating-axis
// test over the 15 candidate axes (the three face normals of each box and the
// nine cross products of an edge direction of each, skipping crosses shorter
// than 1e-6).  The overlap of the boxes' projections on a unit axis L is
// o(L) = sum_i a_i |L.u_i| + sum_j b_j |L.w_j| - |L.(c_B - c_A)|, with u_i, w_j
// the box axes and a_i, b_j the half sizes; the contact axis is the one of
// least overlap, a face axis unless the least edge overlap is smaller than the
// least face overlap by more than 5% of its magnitude plus 1e-6 (ties: the
// lower axis index).  Face axis: the box that owns it is the reference, the
// other the incident box; the reference normal points from the reference box
// toward the incident one; the incident face is the incident box's face most
// opposed to it; its four corners, clipped against the four side planes of
// the reference face (Sutherland-Hodgman), give up to 8 points, and each point
// p with signed distance r = n.(p - f) to the reference face plane (through f)
// below the margin is a contact at the midpoint p - (r/2) n.  Edge axis: one
// contact between the two supporting edges (the edges of each box that
// point along the axis' factors and lie furthest toward the other box), r the
// signed distance between their lines along the axis, at the midpoint of the
// lines' closest points.  The normal is reported from box A (geom 1) toward
// box B; all decisions (axis, faces, clipping) are taken on values, so a
// derivative holds them fixed.
template <class S>
static void box_box(const V3<S>& cA, const M3<S>& RA, const V3<double>& ha, const V3<S>& cB, const M3<S>& RB,
                    const V3<double>& hb, double margin, int pair, std::vector<Contact<S>>& out) {
  V3<S> uA[3], uB[3];
  for (int i = 0; i < 3; ++i) { uA[i] = col(RA, i); uB[i] = col(RB, i); }
  const V3<S> d = sub(cB, cA);
  auto overlap = [&](const V3<S>& L) {
    S pa = S(0.0), pb = S(0.0);
    for (int i = 0; i < 3; ++i) { pa += sabs(dot(L, uA[i])) * ha.x[i]; pb += sabs(dot(L, uB[i])) * hb.x[i]; }
    return pa + pb - sabs(dot(L, d));
  };
  int face = 0, edge = -1;
  double of = HUGE_VAL, oe = HUGE_VAL;
  for (int i = 0; i < 6; ++i) {
    const double o = val(overlap(i < 3 ? uA[i] : uB[i - 3]));
    if (o < of) { of = o; face = i; }
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      const V3<S> c = cross(uA[i], uB[j]);
      const S cn = sqrt_(dot(c, c));
      if (val(cn) < 1e-6) continue;
      const double o = val(overlap(scale(c, S(1.0) / cn)));
      if (o < oe) { oe = o; edge = 3 * i + j; }
    }
  const bool use_edge = edge >= 0 && oe < of - (0.05 * std::fabs(of) + 1e-6);
  if (std::min(of, oe) <= -margin) return;  // separated by at least the margin along some axis
  if (!use_edge) {
    const bool refA = face < 3;
    const int ax = face % 3;
    const V3<S>* uR = refA ? uA : uB;
    const V3<S>* uI = refA ? uB : uA;
    const V3<double>& hR = refA ? ha : hb;
    const V3<double>& hI = refA ? hb : ha;
    const V3<S> cR = refA ? cA : cB, cI = refA ? cB : cA;
    V3<S> nR = uR[ax];
    if (val(dot(nR, sub(cI, cR))) < 0.0) nR = scale(nR, -1.0);
    int fj = 0;
    double best = -1.0;
    for (int j = 0; j < 3; ++j) {
      const double a = std::fabs(val(dot(nR, uI[j])));
      if (a > best) { best = a; fj = j; }
    }
    // outward normal of the incident face points against nR
    const double sg = val(dot(nR, uI[fj])) > 0.0 ? -1.0 : 1.0;
    const V3<S> fc = add(cI, scale(uI[fj], sg * hI.x[fj]));
    const int j1 = (fj + 1) % 3, j2 = (fj + 2) % 3;
    std::vector<V3<S>> poly;
    const double s1[4] = {1.0, -1.0, -1.0, 1.0}, s2[4] = {1.0, 1.0, -1.0, -1.0};
    for (int c = 0; c < 4; ++c)
      poly.push_back(add(fc, add(scale(uI[j1], s1[c] * hI.x[j1]), scale(uI[j2], s2[c] * hI.x[j2]))));
    for (int kk = 1; kk <= 2; ++kk) {
      const int k2 = (ax + kk) % 3;
      for (int sgn = 1; sgn >= -1; sgn -= 2) {
        // keep the side where sgn u_k.(p - c_R) <= h_k
        auto f = [&](const V3<S>& P) { return dot(uR[k2], sub(P, cR)) * (double)sgn - hR.x[k2]; };
        std::vector<V3<S>> nxt;
        const size_t np = poly.size();
        for (size_t i = 0; i < np; ++i) {
          const V3<S>& P = poly[i];
          const V3<S>& Q = poly[(i + 1) % np];
          const S fP = f(P), fQ = f(Q);
          const bool inP = val(fP) <= 0.0, inQ = val(fQ) <= 0.0;
          if (inP) nxt.push_back(P);
          if (inP != inQ) nxt.push_back(add(P, scale(sub(Q, P), fP / (fP - fQ))));
        }
        poly.swap(nxt);
      }
    }
    const V3<S> pf = add(cR, scale(nR, hR.x[ax]));
    for (const V3<S>& P : poly) {
      const S r = dot(nR, sub(P, pf));
      if (val(r) >= margin) continue;
      Contact<S> ct;
      ct.r = r;
      ct.pos = sub(P, scale(nR, r * 0.5));
      ct.n = refA ? nR : scale(nR, -1.0);
      make_frame(ct.n, ct.t1, ct.t2);
      ct.pair = pair;
      out.push_back(ct);
    }
    return;
  }
  const int i = edge / 3, j = edge % 3;
  V3<S> n = cross(uA[i], uB[j]);
  n = scale(n, S(1.0) / sqrt_(dot(n, n)));
  if (val(dot(n, d)) < 0.0) n = scale(n, -1.0);
  V3<S> pA = cA, pB = cB;
  for (int k2 = 0; k2 < 3; ++k2) {
    if (k2 != i) pA = add(pA, scale(uA[k2], (val(dot(n, uA[k2])) >= 0.0 ? 1.0 : -1.0) * ha.x[k2]));
    if (k2 != j) pB = add(pB, scale(uB[k2], (val(dot(n, uB[k2])) >= 0.0 ? -1.0 : 1.0) * hb.x[k2]));
  }
  // closest points of the lines pA + s uA_i and pB + t uB_j
  const V3<S> w = sub(pA, pB);
  const S b = dot(uA[i], uB[j]), dd = dot(uA[i], w), e = dot(uB[j], w);
  const S den = S(1.0) - b * b;
  const S sA = (b * e - dd) / den, tB = (e - b * dd) / den;
  const V3<S> PA = add(pA, scale(uA[i], sA)), PB = add(pB, scale(uB[j], tB));
  const S r = dot(n, sub(PB, PA));
  if (val(r) >= margin) return;
  Contact<S> ct;
  ct.r = r;
  ct.pos = scale(add(PA, PB), 0.5);
  ct.n = n;
  make_frame(n, ct.t1, ct.t2);
  ct.pair = pair;
  out.push_back(ct);
}

// Candidate contacts of every listed pair (Sec. 2.1, "Collision detection"),
// in pair order; plane pairs with a fixed number of slots per pair type.
// reading: a capsule against a plane emits both cap-centre spheres (+axis end
// first), with no case split (the smoothing of App. C.1 is then
// unnecessary).  Box-box pairs are first culled by their bounding spheres
// (radius |half sizes|; kept if the centres are closer than the radii plus
// the margin) and emit only contacts with r below the margin (the CFD width
// w_c of the pair when cfd, else 0).
template <class S>
static void collide(const Model& m, const Kin<S>& k, std::vector<Contact<S>>& out, bool cfd = false) {
  out.clear();
  for (int p = 0; p < m.np; ++p) {
    int g1 = m.pg1[p], g2 = m.pg2[p];
    if (m.gtype[g1] == G_BOX && m.gtype[g2] == G_BOX) {
      const double margin = cfd ? m.pcfd[5 * p + 2] : 0.0;
      const V3<double>& ha = m.gsize[g1];
      const V3<double>& hb = m.gsize[g2];
      const double ra = std::sqrt(ha.x[0] * ha.x[0] + ha.x[1] * ha.x[1] + ha.x[2] * ha.x[2]);
      const double rb = std::sqrt(hb.x[0] * hb.x[0] + hb.x[1] * hb.x[1] + hb.x[2] * hb.x[2]);
      const V3<S> dc = sub(k.gpos[g2], k.gpos[g1]);
      if (std::sqrt(val(dot(dc, dc))) >= ra + rb + margin) continue;
      box_box(k.gpos[g1], k.gmat[g1], ha, k.gpos[g2], k.gmat[g2], hb, margin, p, out);
      continue;
    }
    V3<S> n = col(k.gmat[g1], 2), p0 = k.gpos[g1];
    if (m.gtype[g2] == G_SPHERE) {
      out.push_back(sphere_plane(p0, n, k.gpos[g2], m.gsize[g2].x[0], p));
    } else if (m.gtype[g2] == G_CAPSULE) {
      V3<S> ax = scale(col(k.gmat[g2], 2), m.gsize[g2].x[1]);
      out.push_back(sphere_plane(p0, n, add(k.gpos[g2], ax), m.gsize[g2].x[0], p));
      out.push_back(sphere_plane(p0, n, sub(k.gpos[g2], ax), m.gsize[g2].x[0], p));
    } else if (m.gtype[g2] == G_BOX) {
      box_plane(p0, n, k.gpos[g2], k.gmat[g2], m.gsize[g2], p, out);
    }
  }
}

// ------------------------------------------------------------------ constraint rows
template <class S>
struct Row {
  std::vector<S> J;   // nv
  std::vector<int> nz;  // dofs of the contact's two bodies (J vanishes elsewhere)
  S aref, D;
};

// MuJoCo impedance d(r) as a polynomial spline of the violation (Sec. 2.1,
// Fig. 2; parameters d0, dw, width, midpoint, power).  reading: x = min(1,
// |r|/width); y = x^p / m^(p-1) for x <= m, else 1 - (1-x)^p / (1-m)^(p-1);
// d = d0 + y (dw - d0).
template <class S>
static S spline_imp(S x, double d0, double dw, double mid, double pw) {
  S y;
  if (val(x) >= 1.0) return S(dw);
  if (val(x) <= mid) y = pow_(x, pw) / std::pow(mid, pw - 1.0);
  else y = 1.0 - pow_(1.0 - x, pw) / std::pow(1.0 - mid, pw - 1.0);
  return d0 + y * (dw - d0);
}

template <class S> static S softplus(S z, double beta) {
  S bz = z * beta;
  if (val(bz) > 30.0) return z + log1p_(exp_(-bz)) / beta;
  return log1p_(exp_(bz)) / beta;
}

// Constraint rows of the active contacts (Sec. 2.1): pyramidal cone with 4
// edge rows J_n +- mu J_t per contact (reading: order +t1, -t1, +t2, -t2, all
// sharing r); reference acceleration a_ref = -b (J v) - k r with
// b = 2/(d_w t_c), k = d(r)/(d_w^2 t_c^2 phi^2) (eq. for a_ref); regularizer
// R = A (1-d)/d and D = 1/R, with the diagonal approximation
// A = (1 + mu^2)(w_b1 + w_b2) from the bodies' translational inverse weights
// (reading).  With cfd (Sec. 4): rows for every contact with r < w_c, the
// impedance continued for r >= 0 by the CFD spline from d_0 at r = 0 to d_c at
// r = w_c, and the position term k*relu(-r) replaced by k*softplus(-r).
// reading (capacity): at most kMaxContacts contacts make rows, taken in
// candidate (pair) order; further ones are dropped and flagged.
constexpr int kMaxContacts = 256;

template <class S>
static void make_rows(const Model& m, const Kin<S>& k, const std::vector<Contact<S>>& cons, const S* v,
                      bool cfd, double beta, std::vector<Row<S>>& rows, bool* overflow = nullptr) {
  rows.clear();
  int nv = m.nv;
  int n_on = 0;
  std::vector<S> J1(3 * nv), J2(3 * nv);
  for (const Contact<S>& ct : cons) {
    int p = ct.pair;
    const double* si = &m.psolimp[5 * p];
    const double* cf = &m.pcfd[5 * p];
    double r = val(ct.r);
    bool on = cfd ? (r < cf[2]) : (r < 0.0);
    if (!on) continue;
    if (n_on == kMaxContacts) { if (overflow) *overflow = true; continue; }
    ++n_on;
    int b1 = m.gbody[m.pg1[p]], b2 = m.gbody[m.pg2[p]];
    std::vector<int> nzd;
    if (b1 >= 0) nzd = m.bdofs[b1];
    if (b2 >= 0) nzd.insert(nzd.end(), m.bdofs[b2].begin(), m.bdofs[b2].end());
    std::sort(nzd.begin(), nzd.end());
    nzd.erase(std::unique(nzd.begin(), nzd.end()), nzd.end());
    for (int i = 0; i < 3 * nv; ++i) { J1[i] = S(0.0); J2[i] = S(0.0); }
    if (b1 >= 0) point_jac(m, k, b1, ct.pos, J1.data(), (S*)nullptr);
    if (b2 >= 0) point_jac(m, k, b2, ct.pos, J2.data(), (S*)nullptr);
    std::vector<S> Jn(nv), Jt1(nv), Jt2(nv);
    for (int i = 0; i < nv; ++i) {
      S d0 = J2[i] - J1[i], d1 = J2[nv + i] - J1[nv + i], d2 = J2[2 * nv + i] - J1[2 * nv + i];
      Jn[i] = ct.n.x[0] * d0 + ct.n.x[1] * d1 + ct.n.x[2] * d2;
      Jt1[i] = ct.t1.x[0] * d0 + ct.t1.x[1] * d1 + ct.t1.x[2] * d2;
      Jt2[i] = ct.t2.x[0] * d0 + ct.t2.x[1] * d1 + ct.t2.x[2] * d2;
    }
    S d;
    if (r < 0.0) d = spline_imp(S(-1.0) * ct.r / si[2], si[0], si[1], si[3], si[4]);
    else d = spline_imp(ct.r / cf[2], cf[1], cf[0], cf[3], cf[4]);
    double tc = m.psolref[2 * p], dr = m.psolref[2 * p + 1], dw = si[1];
    double bcoef = 2.0 / (dw * tc);
    S kcoef = d / (dw * dw * tc * tc * dr * dr);
    double mu = m.pmu[p];
    double invw = (b1 >= 0 ? m.binvw[b1] : 0.0) + (b2 >= 0 ? m.binvw[b2] : 0.0);
    double Ahat = (1.0 + mu * mu) * invw;
    S D = d / (Ahat * (1.0 - d));
    S pterm = cfd ? kcoef * softplus(S(-1.0) * ct.r, beta) : S(-1.0) * kcoef * ct.r;
    for (int e = 0; e < 4; ++e) {
      Row<S> row;
      row.J.resize(nv);
      row.nz = nzd;
      const std::vector<S>& Jt = (e < 2) ? Jt1 : Jt2;
      double sg = (e % 2 == 0) ? mu : -mu;
      S jv = S(0.0);
      for (int i = 0; i < nv; ++i) { row.J[i] = Jn[i] + Jt[i] * sg; jv += row.J[i] * v[i]; }
      row.aref = S(-bcoef) * jv + pterm;
      row.D = D;
      rows.push_back(row);
    }
  }
}

// ------------------------------------------------------------------ linear algebra
template <class S>
static bool cholesky(std::vector<S>& A, int n) {  // in place, lower triangle
  for (int j = 0; j < n; ++j) {
    S s = A[j * n + j];
    for (int k2 = 0; k2 < j; ++k2) s -= A[j * n + k2] * A[j * n + k2];
    if (!(val(s) > 0.0)) return false;
    A[j * n + j] = sqrt_(s);
    for (int i = j + 1; i < n; ++i) {
      S t = A[i * n + j];
      for (int k2 = 0; k2 < j; ++k2) t -= A[i * n + k2] * A[j * n + k2];
      A[i * n + j] = t / A[j * n + j];
    }
  }
  return true;
}
template <class S>
static void chol_solve(const std::vector<S>& L, int n, std::vector<S>& x) {
  for (int i = 0; i < n; ++i) {
    S s = x[i];
    for (int k2 = 0; k2 < i; ++k2) s -= L[i * n + k2] * x[k2];
    x[i] = s / L[i * n + i];
  }
  for (int i = n - 1; i >= 0; --i) {
    S s = x[i];
    for (int k2 = i + 1; k2 < n; ++k2) s -= L[k2 * n + i] * x[k2];
    x[i] = s / L[i * n + i];
  }
}

// ------------------------------------------------------------------ Newton solve
// Exact Newton method for the convex primal problem (Sec. 2.1, eq.
// primal-problem) with a pyramidal cone: minimize
//   f(x) = 1/2 (x - a0)^T M (x - a0) + sum_e 1/2 D_e min(0, J_e x - aref_e)^2,
// a0 = M^-1 (tau - c).  reading: started at a0; each iteration takes the
// Newton direction of the current active set and the exact minimizer of the
// convex piecewise quadratic along it (breakpoints sorted, segments scanned),
// and stops when the active set no longer changes.
template <class T>
struct NewtonOut {
  std::vector<T> x;
  std::vector<char> active;
  int iters;
  bool ok;
  long long active_contacts = 0;    // contacts with an active edge, summed over iterations
  long long contact_segments = 0;   // contacts times line-search segments scanned
  long long active_box = 0, segments_box = 0;  // the same for contacts between two bodies
};

template <class T>
static T line_search(const std::vector<T>& M, const std::vector<T>& a0, const std::vector<Row<T>>& rows,
                     const std::vector<T>& x, const std::vector<T>& dl, int nv, long long* contact_segments,
                     long long* segments_box) {
  FlopPhase phase(kPhLineSearch);
  T dMd = 0.0, xMd = 0.0;
  for (int i = 0; i < nv; ++i) {
    const T dxi = x[i] - a0[i];
    for (int j = 0; j < nv; ++j) { dMd += dl[i] * M[i * nv + j] * dl[j]; xMd += dxi * M[i * nv + j] * dl[j]; }
  }
  size_t nr = rows.size();
  std::vector<T> s(nr), t(nr);
  std::vector<double> bp;
  for (size_t e = 0; e < nr; ++e) {
    T jx = 0.0, jd = 0.0;
    for (int i = 0; i < nv; ++i) { jx += rows[e].J[i] * x[i]; jd += rows[e].J[i] * dl[i]; }
    s[e] = jx - rows[e].aref; t[e] = jd;
    if (val(jd) != 0.0) {
      const double b = val(-(s[e] / jd));
      if (b > 0.0) bp.push_back(b);
    }
  }
  std::sort(bp.begin(), bp.end());
  double lo = 0.0;
  for (size_t seg = 0; seg <= bp.size(); ++seg) {
    bool last = seg == bp.size();
    double hi = last ? 0.0 : bp[seg];
    const T tlo = value_as<T>(lo);
    T mid = last ? tlo + 1.0 : T(0.5) * (tlo + value_as<T>(hi));
    T c2 = dMd, c1 = xMd;
    *contact_segments += (long long)(nr / 4);
    for (size_t c = 0; c + 3 < nr; c += 4) *segments_box += rows[c].nz.size() > 6 ? 1 : 0;
    for (size_t e = 0; e < nr; ++e)
      if (val(s[e] + mid * t[e]) < 0.0) { c2 += rows[e].D * t[e] * t[e]; c1 += rows[e].D * t[e] * s[e]; }
    T ar = -(c1 / c2);
    if (last || val(ar) <= hi) return val(ar) < lo ? T(lo) : ar;
    lo = hi;
  }
  return T(lo);
}

template <class T>
static NewtonOut<T> newton(const std::vector<T>& M, const std::vector<T>& a0, const std::vector<Row<T>>& rows, int nv,
                           int maxit) {
  FlopPhase phase(kPhNewton);
  NewtonOut<T> o;
  o.x = a0; o.iters = 0; o.ok = true;
  size_t nr = rows.size();
  auto act = [&](const std::vector<T>& x) {
    std::vector<char> a(nr);
    for (size_t e = 0; e < nr; ++e) {
      T jx = 0.0;
      for (int i = 0; i < nv; ++i) jx += rows[e].J[i] * x[i];
      a[e] = val(jx - rows[e].aref) < 0.0;
    }
    return a;
  };
  o.active = act(o.x);
  bool any = false;
  for (char c : o.active) any = any || c;
  if (!any) return o;  // no force: x = a0 is optimal
  for (int it = 0; it < maxit; ++it) {
    for (size_t c = 0; c + 3 < nr; c += 4)
    {
      const bool on = o.active[c] | o.active[c + 1] | o.active[c + 2] | o.active[c + 3];
      o.active_contacts += on ? 1 : 0;
      o.active_box += (on && rows[c].nz.size() > 6) ? 1 : 0;
    }
    std::vector<T> g(nv, T(0.0)), H = M, dx(nv);
    for (int j = 0; j < nv; ++j) dx[j] = o.x[j] - a0[j];
    for (int i = 0; i < nv; ++i)
      for (int j = 0; j < nv; ++j) g[i] += M[i * nv + j] * dx[j];
    for (size_t e = 0; e < nr; ++e) {
      if (!o.active[e]) continue;
      T jx = 0.0;
      for (int i = 0; i < nv; ++i) jx += rows[e].J[i] * o.x[i];
      T se = jx - rows[e].aref;
      for (int i : rows[e].nz) {
        g[i] += rows[e].D * se * rows[e].J[i];
        for (int j : rows[e].nz) H[i * nv + j] += rows[e].D * rows[e].J[i] * rows[e].J[j];
      }
    }
    if (!cholesky(H, nv)) { o.ok = false; return o; }
    std::vector<T> dl(nv);
    for (int i = 0; i < nv; ++i) dl[i] = -g[i];
    chol_solve(H, nv, dl);
    T alpha = line_search(M, a0, rows, o.x, dl, nv, &o.contact_segments, &o.segments_box);
    for (int i = 0; i < nv; ++i) o.x[i] += alpha * dl[i];
    o.iters = it + 1;
    std::vector<char> na = act(o.x);
    bool same = na == o.active;
    o.active = na;
    if (same) return o;
  }
  o.ok = false;
  return o;
}

// ------------------------------------------------------------------ right-hand side
struct Opts {
  double rtol = 1e-6, atol = 1e-8, h0 = 1e-3, safety = 0.9, facmin = 0.2, facmax = 10.0;
  double kP = 0.2, kI = 0.4, err_order = 5.0, err_floor = 1e-6;
  long long max_attempts = 1000000;
  int newton_maxit = 100;
  bool cfd = false;
  double beta = 1e4;
  int h_levels = 0;
  int tableau = 0;
};

// reading: the controller's proposed step is rounded down to a grid of
// `levels` mantissa values per octave, h = floor(m * 2 levels) / (2 levels) * 2^e
// with h = m * 2^e, m in [0.5, 1) (exact in binary floating point).  Step
// sequences then do not depend on rounding-level differences of the error
// estimate between implementations.
static double quantize_step(double h, int levels) {
  if (levels <= 0 || !(h > 0.0) || !std::isfinite(h)) return h;
  int e;
  double m = std::frexp(h, &e);
  double k = std::floor(m * (2.0 * levels));
  return std::ldexp(k / (2.0 * levels), e);
}

struct Stats {
  long long rhs = 0, newton_it = 0;
  int status = 0;
  int nrows = 0, nactive = 0;
  // work units: contacts per right-hand side, contacts with an active edge
  // per Newton iteration, contacts per line-search segment scanned (summed)
  long long contacts = 0, newton_contacts = 0, ls_contacts = 0;
  long long contacts_box = 0, newton_contacts_box = 0, ls_contacts_box = 0;  // between two bodies
};

// F(t, x) = (v, qacc) with qacc the minimizer of the primal problem, i.e. the
// acceleration of eq. EOM under the soft contact forces (Sec. 2 and App. C.2
// write the simulator as this ODE).  For S = Dual the tangent of qacc follows
// from the optimality system H x* = (tau - c) + sum_A D_e aref_e J_e^T at the
// converged active set A, i.e. the derivative of the exact solution; the
// value is the Newton iterate.
template <class S>
static void rhs(const Model& m, const S* y, const S* u, bool cfd, double beta, int maxit, S* kout,
                Stats* st, std::vector<double>* forces = nullptr) {
  FlopPhase phase(kPhRhs);
  int nv = m.nv;
  const S* q = y;
  const S* v = y + m.nq;
  Kin<S> kin;
  kinematics(m, q, v, kin);
  std::vector<S> M(nv * nv), c(nv);
  mass_bias(m, kin, M.data(), c.data());
  std::vector<S> f0(nv);
  for (int i = 0; i < nv; ++i) f0[i] = S(0.0) - c[i];
  for (int i = 0; i < m.nu; ++i) f0[m.ctrl[i]] += u[i];
  std::vector<S> L = M;
  if (!cholesky(L, nv)) { st->status |= ORC_NONFINITE; }
  std::vector<S> a0 = f0;
  chol_solve(L, nv, a0);
  std::vector<Contact<S>> cons;
  collide(m, kin, cons, cfd);
  std::vector<Row<S>> rows;
  bool overflow = false;
  make_rows(m, kin, cons, v, cfd, beta, rows, &overflow);
  if (overflow) st->status |= ORC_CONTACT_OVERFLOW;
  st->rhs += 1;
  st->contacts += (long long)(rows.size() / 4);
  for (size_t c = 0; c + 3 < rows.size(); c += 4) st->contacts_box += rows[c].nz.size() > 6 ? 1 : 0;
  st->nrows = (int)rows.size();
  for (int i = 0; i < nv; ++i) kout[i] = v[i];
  if (forces) forces->assign(rows.size(), 0.0);
  if (rows.empty()) { for (int i = 0; i < nv; ++i) kout[nv + i] = a0[i]; st->nactive = 0; return; }
  using T = typename ValueOf<S>::type;
  std::vector<T> Md(nv * nv), a0d(nv);
  for (int i = 0; i < nv * nv; ++i) Md[i] = value_as<T>(M[i]);
  for (int i = 0; i < nv; ++i) a0d[i] = value_as<T>(a0[i]);
  std::vector<Row<T>> rd(rows.size());
  for (size_t e = 0; e < rows.size(); ++e) {
    rd[e].J.resize(nv);
    rd[e].nz = rows[e].nz;
    for (int i = 0; i < nv; ++i) rd[e].J[i] = value_as<T>(rows[e].J[i]);
    rd[e].aref = value_as<T>(rows[e].aref); rd[e].D = value_as<T>(rows[e].D);
  }
  NewtonOut<T> no = newton(Md, a0d, rd, nv, maxit);
  st->newton_it += no.iters;
  st->newton_contacts += no.active_contacts;
  st->ls_contacts += no.contact_segments;
  st->newton_contacts_box += no.active_box;
  st->ls_contacts_box += no.segments_box;
  if (!no.ok) st->status |= ORC_SOLVER_MAXIT;
  int na = 0;
  for (char a : no.active) na += a;
  st->nactive = na;
  if (forces)
    for (size_t e = 0; e < rows.size(); ++e) {
      T jx = 0.0;
      for (int i = 0; i < nv; ++i) jx += rd[e].J[i] * no.x[i];
      (*forces)[e] = no.active[e] ? val(rd[e].D * (rd[e].aref - jx)) : 0.0;
    }
  if (!is_dual<S>() || na == 0) {
    for (int i = 0; i < nv; ++i) { kout[nv + i] = na == 0 ? a0[i] : FromValue<S>::get(no.x[i]); set_val(kout[nv + i], val(no.x[i])); }
    return;
  }
  std::vector<S> H = M, b = f0;
  for (size_t e = 0; e < rows.size(); ++e) {
    if (!no.active[e]) continue;
    for (int i : rows[e].nz) {
      b[i] += rows[e].D * rows[e].aref * rows[e].J[i];
      for (int j : rows[e].nz) H[i * nv + j] += rows[e].D * rows[e].J[i] * rows[e].J[j];
    }
  }
  if (!cholesky(H, nv)) st->status |= ORC_NONFINITE;
  chol_solve(H, nv, b);
  for (int i = 0; i < nv; ++i) { kout[nv + i] = b[i]; set_val(kout[nv + i], val(no.x[i])); }
}

// Straight-through rule at the ODE level (Sec. 4): the value is F (no CFD),
// the tangent is that of the CFD field F~ evaluated at the same state.
template <class S>
static void rhs_st(const Model& m, const S* y, const S* u, const Opts& o, S* kout, Stats* st) {
  if (!o.cfd || !is_dual<S>()) { rhs(m, y, u, false, o.beta, o.newton_maxit, kout, st); return; }
  rhs(m, y, u, true, o.beta, o.newton_maxit, kout, st);
  int nx = m.nq + m.nv;
  std::vector<double> yd(nx), ud(std::max(m.nu, 1)), kd(2 * m.nv);
  for (int i = 0; i < nx; ++i) yd[i] = val(y[i]);
  for (int i = 0; i < m.nu; ++i) ud[i] = val(u[i]);
  Stats s2;
  rhs(m, yd.data(), ud.data(), false, o.beta, o.newton_maxit, kd.data(), &s2);
  st->status |= s2.status; st->newton_it += s2.newton_it; st->rhs += 1;
  for (int i = 0; i < 2 * m.nv; ++i) set_val(kout[i], kd[i]);
}

// ------------------------------------------------------------------ integration
// Dormand-Prince 5(4) (cited in App. C.2), the FSAL tableau of Dormand and
// Prince (1980).
static const double RK_C[7] = {0.0, 1.0 / 5.0, 3.0 / 10.0, 4.0 / 5.0, 8.0 / 9.0, 1.0, 1.0};
static const double RK_A[7][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 5.0, 0, 0, 0, 0, 0},
    {3.0 / 40.0, 9.0 / 40.0, 0, 0, 0, 0},
    {44.0 / 45.0, -56.0 / 15.0, 32.0 / 9.0, 0, 0, 0},
    {19372.0 / 6561.0, -25360.0 / 2187.0, 64448.0 / 6561.0, -212.0 / 729.0, 0, 0},
    {9017.0 / 3168.0, -355.0 / 33.0, 46732.0 / 5247.0, 49.0 / 176.0, -5103.0 / 18656.0, 0},
    {35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0, -2187.0 / 6784.0, 11.0 / 84.0}};
static const double RK_B[7] = {35.0 / 384.0, 0.0, 500.0 / 1113.0, 125.0 / 192.0, -2187.0 / 6784.0, 11.0 / 84.0, 0.0};
static const double RK_BH[7] = {5179.0 / 57600.0, 0.0, 7571.0 / 16695.0, 393.0 / 640.0, -92097.0 / 339200.0,
                                187.0 / 2100.0, 1.0 / 40.0};

// Tsitouras 5(4) (Tsit5, the solver of the paper's experiments, App. E.1): the
// FSAL pair of Tsitouras (2011), whose coefficients satisfy only the first
// column simplifying assumption.  b-hat = b - btilde with btilde the published
// error weights.
static const double T5_C[7] = {0.0, 0.161, 0.327, 0.9, 0.9800255409045097, 1.0, 1.0};
static const double T5_A[7][6] = {
    {0, 0, 0, 0, 0, 0},
    {0.161, 0, 0, 0, 0, 0},
    {-0.008480655492356989, 0.335480655492357, 0, 0, 0, 0},
    {2.897153057105493, -6.359448489975075, 4.3622954328695815, 0, 0, 0},
    {5.325864828439257, -11.748883564062828, 7.4955393428898365, -0.09249506636175525, 0, 0},
    {5.86145544294642, -12.92096931784711, 8.159367898576159, -0.071584973281401, -0.028269050394068383, 0},
    {0.09646076681806523, 0.01, 0.4798896504144996, 1.379008574103742, -3.290069515436081, 2.324710524099774}};
static const double T5_B[7] = {0.09646076681806523, 0.01, 0.4798896504144996, 1.379008574103742,
                               -3.290069515436081, 2.324710524099774, 0.0};
static const double T5_BT[7] = {-0.00178001105222577714, -0.0008164344596567469, 0.007880878010261995,
                                -0.1447110071732629, 0.5823571654525552, -0.45808210592918697,
                                0.015151515151515152};
struct Tab { const double (*A)[6]; const double* B; double BH[7]; };
static Tab tableau_of(int which) {
  Tab t;
  if (which == 1) {
    t.A = T5_A; t.B = T5_B;
    for (int i = 0; i < 7; ++i) t.BH[i] = T5_B[i] - T5_BT[i];
  } else {
    t.A = RK_A; t.B = RK_B;
    for (int i = 0; i < 7; ++i) t.BH[i] = RK_BH[i];
  }
  return t;
}

// q (+) dq: positions integrate the tangent; free-joint quaternions are
// integrated exactly, quat <- quat * exp(dtheta/2) with dtheta the body-frame
// rotation vector, and renormalized (App. C.2: quaternion-aware solvers).
template <class S>
static void qplus(const Model& m, const S* q, const S* dq, S* out) {
  for (int j = 0; j < m.nj; ++j) {
    int qa = m.jqadr[j], da = m.jdadr[j];
    if (m.jtype[j] == J_FREE) {
      for (int i = 0; i < 3; ++i) out[qa + i] = q[qa + i] + dq[da + i];
      Q4<S> qq; qq.w = q[qa + 3]; qq.x = q[qa + 4]; qq.y = q[qa + 5]; qq.z = q[qa + 6];
      Q4<S> e = qexp_rotvec(v3<S>(dq[da + 3], dq[da + 4], dq[da + 5]));
      Q4<S> r = qnormalize(qmul(qq, e));
      out[qa + 3] = r.w; out[qa + 4] = r.x; out[qa + 5] = r.y; out[qa + 6] = r.z;
    } else {
      out[qa] = q[qa] + dq[da];
    }
  }
}

struct Log {
  std::vector<double> tape;     // (t, h, y[nx]) per accepted step
  std::vector<double> steplog;  // (t, h, err, accepted) per attempt
  long long n_acc = 0, n_rej = 0;
  bool keep_tape = false, keep_log = false;
};

// One Dormand-Prince attempt from (y, k1) with step h.  Writes the 5th-order
// solution, the FSAL stage k7 = F(y_new), and returns the error norm.
// reading: the error estimate is taken in the ambient coordinates of q and v:
// for scalar coordinates e = h sum_i (b_i - bh_i) k_i, for a quaternion the
// difference of the two (+)-integrated quaternions; eps is the RMS over all
// nq + nv components of e_j / (atol + rtol max(|y_j|, |y_new_j|)).
template <class S>
static double dopri_attempt(const Model& m, const S* y, const S* uk, const std::vector<S>& k1, double h,
                            const Opts& o, bool want_err, S* ynew, std::vector<S>& k7, Stats* st,
                            std::vector<std::vector<S>>* stages = nullptr) {
  FlopPhase phase(kPhStep);
  const Tab tb = tableau_of(o.tableau);
  int nq = m.nq, nv = m.nv, nx = nq + nv;
  std::vector<std::vector<S>> K(7, std::vector<S>(2 * nv));
  K[0] = k1;
  std::vector<S> Y(nx), dq(nv);
  for (int i = 1; i < 7; ++i) {
    for (int d = 0; d < nv; ++d) {
      S sq = S(0.0), sv = S(0.0);
      for (int j = 0; j < i; ++j) { sq += K[j][d] * tb.A[i][j]; sv += K[j][nv + d] * tb.A[i][j]; }
      dq[d] = sq * h;
      Y[nq + d] = y[nq + d] + sv * h;
    }
    qplus(m, y, dq.data(), Y.data());
    rhs_st(m, Y.data(), uk, o, K[i].data(), st);
  }
  for (int i = 0; i < nx; ++i) ynew[i] = Y[i];  // stage 7 is evaluated at y_new (FSAL)
  k7 = K[6];
  if (stages) *stages = K;
  if (!want_err) return 0.0;
  using T = typename ValueOf<S>::type;
  std::vector<T> e(nx, T(0.0)), dqh(nv);
  std::vector<T> yhat(nq);
  for (int d = 0; d < nv; ++d) {
    T sh = 0.0, sa = 0.0;
    for (int i = 0; i < 7; ++i) {
      sh += value_as<T>(K[i][d]) * tb.BH[i];
      sa += value_as<T>(K[i][nv + d]) * (tb.B[i] - tb.BH[i]);
    }
    dqh[d] = sh * h;
    e[nq + d] = sa * h;
  }
  std::vector<T> yv(nq);
  for (int i = 0; i < nq; ++i) yv[i] = value_as<T>(y[i]);
  qplus(m, yv.data(), dqh.data(), yhat.data());
  for (int i = 0; i < nq; ++i) e[i] = value_as<T>(ynew[i]) - yhat[i];
  // scalar coordinates: use the difference form h sum (b - bh) k directly
  for (int j = 0; j < m.nj; ++j) {
    int qa = m.jqadr[j], da = m.jdadr[j];
    int nlin = m.jtype[j] == J_FREE ? 3 : 1;
    for (int i = 0; i < nlin; ++i) {
      T se = 0.0;
      for (int s = 0; s < 7; ++s) se += value_as<T>(K[s][da + i]) * (tb.B[s] - tb.BH[s]);
      e[qa + i] = se * h;
    }
  }
  T acc = 0.0;
  for (int i = 0; i < nx; ++i) {
    T sc = T(o.atol) + T(o.rtol) * value_as<T>(std::max(std::fabs(val(y[i])), std::fabs(val(ynew[i]))));
    T r = e[i] / sc;
    acc += r * r;
  }
  return val(sqrt_(acc / T((double)nx)));
}

static bool finite_vec(const double* x, int n) {
  for (int i = 0; i < n; ++i) if (!std::isfinite(x[i])) return false;
  return true;
}

// The step-size controller (App. E.1 names Diffrax's PID controller with
// P = 0.2, I = 0.4, D = 0).  reading (PI form, D = 0): the step factor is
// fac = safety * e^(-(kP + kI)/K) * e_prev^(kP/K) with K = err_order = 5,
// clipped to [facmin, facmax]; e = max(eps, err_floor) (a non-finite eps, a
// failed trial solve, counts as 1e300); e_prev starts at 1 and takes e on
// acceptance.  The next proposed step is fac h after an acceptance and
// min(1, fac) h after a rejection, optionally rounded down to the step grid.
static double next_step(const Opts& o, double err, double eprev, double h, bool accepted, double* eprev_out) {
  const double et = std::isfinite(err) ? std::max(err, o.err_floor) : 1e300;
  double fac = o.safety * std::pow(et, -(o.kP + o.kI) / o.err_order) * std::pow(eprev, o.kP / o.err_order);
  fac = std::min(o.facmax, std::max(o.facmin, fac));
  if (accepted) {
    *eprev_out = et;
    return quantize_step(fac * h, o.h_levels);
  }
  *eprev_out = eprev;
  return quantize_step(std::min(1.0, fac) * h, o.h_levels);
}

// Adaptive rollout over piecewise-constant control intervals (Sec. 3.1: an
// embedded pair accepts a step when its error estimate is within tolerance,
// otherwise retries with a controller-chosen step; App. E.1 names the PID
// controller with P = 0.2, I = 0.4, D = 0).  reading (PI form, D = 0):
// fac = safety * e^(-(kP+kI)/K) * e_prev^(kP/K), K = err_order = 5, clipped to
// [facmin, facmax], e = max(eps, err_floor), e_prev starting at 1 and updated
// on acceptance; accept iff eps <= 1; after a rejection h <- min(1, fac) h.
// Steps stop on interval ends: if t + 1.01 h >= t_end the step becomes
// t_end - t (and t is set to t_end); the controller's h carries across
// intervals and FSAL is re-evaluated after each interval end (u jumps).
// With `forced`, the listed (t_n, h_n) are replayed with every step accepted.
template <class S>
static int rollout(const Model& m, const S* x0, const S* u, int n_int, double dt, const Opts& o,
                   const double* forced, int n_forced, S* xout, Log* lg, Stats* st) {
  int nq = m.nq, nv = m.nv, nx = nq + nv;
  std::vector<S> y(x0, x0 + nx), yn(nx), k1(2 * nv), k7(2 * nv);
  double t = 0.0, hprop = quantize_step(std::min(o.h0, dt), o.h_levels), eprev = 1.0;
  long long attempts = 0;
  int fi = 0;
  std::vector<double> yv(nx);
  for (int i = 0; i < nx; ++i) yv[i] = val(y[i]);
  if (!finite_vec(yv.data(), nx)) { st->status |= ORC_NONFINITE; }
  std::vector<S> uz(1, S(0.0));
  for (int kk = 0; kk < n_int && (st->status & ~ORC_CONTACT_OVERFLOW) == 0; ++kk) {
    const S* uk = m.nu > 0 ? u + (size_t)kk * m.nu : uz.data();
    double tend = (double)(kk + 1) * dt;
    bool have_k1 = false;
    while (t < tend) {
      if (!have_k1) { rhs_st(m, y.data(), uk, o, k1.data(), st); have_k1 = true; }
      double h;
      bool landing;
      if (forced) {
        if (fi >= n_forced) { st->status |= ORC_MAX_STEPS; break; }
        h = forced[2 * fi + 1];
        landing = t + h >= tend - 0.005 * h;
        ++fi;
      } else {
        landing = t + 1.01 * hprop >= tend;
        h = landing ? tend - t : hprop;
      }
      if (attempts >= o.max_attempts) { st->status |= ORC_MAX_STEPS; break; }
      ++attempts;
      const int status_before = st->status;
      double err = dopri_attempt(m, y.data(), uk, k1, h, o, !forced || !is_dual<S>(), yn.data(), k7, st);
      // reading: a contact solve that fails at a trial stage rejects the
      // attempt (as an infinite error estimate); it is fatal only at an
      // accepted state or in a replay
      if (!forced && (st->status & (ORC_NONFINITE | ORC_SOLVER_MAXIT))) {
        st->status = status_before;
        err = HUGE_VAL;
      }
      bool accept = forced ? true : (err <= 1.0);
      const double hnext = next_step(o, err, eprev, h, accept, &eprev);
      if (lg && lg->keep_log) { lg->steplog.push_back(t); lg->steplog.push_back(h); lg->steplog.push_back(err);
                                lg->steplog.push_back(accept ? 1.0 : 0.0); }
      if (accept) {
        if (lg) {
          lg->n_acc++;
          if (lg->keep_tape) { lg->tape.push_back(t); lg->tape.push_back(h); for (int i = 0; i < nx; ++i) lg->tape.push_back(val(y[i])); }
        }
        y = yn;
        k1 = k7;
        t = landing ? tend : t + h;
        hprop = hnext;
        for (int i = 0; i < nx; ++i) yv[i] = val(y[i]);
        if (!finite_vec(yv.data(), nx)) { st->status |= ORC_NONFINITE; break; }
      } else {
        if (lg) lg->n_rej++;
        hprop = hnext;
      }
      if (!forced && hprop < 1e-12 * std::max(1.0, std::fabs(t))) { st->status |= ORC_DT_UNDERFLOW; break; }
    }
  }
  for (int i = 0; i < nx; ++i) xout[i] = y[i];
  return st->status;
}

}  // namespace orc

using namespace orc;

// ------------------------------------------------------------------ C API
static Opts to_opts(const orc_opts* p) {
  Opts o;
  if (!p) return o;
  o.rtol = p->rtol; o.atol = p->atol; o.h0 = p->h0; o.safety = p->safety; o.facmin = p->facmin;
  o.facmax = p->facmax; o.kP = p->kP; o.kI = p->kI; o.err_order = p->err_order; o.err_floor = p->err_floor;
  o.max_attempts = p->max_attempts; o.newton_maxit = p->newton_maxit; o.cfd = p->cfd != 0;
  o.beta = p->softplus_beta; o.h_levels = p->h_levels; o.tableau = p->tableau == 1 ? 1 : 0;
  return o;
}

extern "C" void* orc_model_new(const orc_model_def* d) {
  Model* m = new Model();
  m->nb = d->nb; m->nj = d->nj; m->ng = d->ng; m->np = d->npair; m->nu = d->nu;
  m->grav = v3<double>(d->gravity[0], d->gravity[1], d->gravity[2]);
  m->bjnt0.assign(m->nb, 0); m->bjntn.assign(m->nb, 0);
  for (int b = 0; b < m->nb; ++b) {
    m->bparent.push_back(d->body_parent[b]);
    m->bpos.push_back(v3<double>(d->body_pos[3 * b], d->body_pos[3 * b + 1], d->body_pos[3 * b + 2]));
    Q4<double> q; q.w = d->body_quat[4 * b]; q.x = d->body_quat[4 * b + 1]; q.y = d->body_quat[4 * b + 2]; q.z = d->body_quat[4 * b + 3];
    m->bquat.push_back(q);
    double mass, I[3];
    primitive_inertia(d->body_iner_type[b], &d->body_iner_size[3 * b], d->body_mass[b], &mass, I);
    Q4<double> iq; iq.w = d->body_iner_quat[4 * b]; iq.x = d->body_iner_quat[4 * b + 1];
    iq.y = d->body_iner_quat[4 * b + 2]; iq.z = d->body_iner_quat[4 * b + 3];
    M3<double> Ri = qmat(qnormalize(iq)), Dg = eye3<double>();
    for (int i = 0; i < 3; ++i) Dg.a[i][i] = I[i];
    m->bmass.push_back(mass);
    m->biner.push_back(matmul(matmul(Ri, Dg), transpose(Ri)));
  }
  int qa = 0, da = 0;
  for (int j = 0; j < m->nj; ++j) {
    int b = d->jnt_body[j];
    if (m->bjntn[b] == 0) m->bjnt0[b] = j;
    m->bjntn[b]++;
    m->jbody.push_back(b); m->jtype.push_back(d->jnt_type[j]);
    m->jaxis.push_back(v3<double>(d->jnt_axis[3 * j], d->jnt_axis[3 * j + 1], d->jnt_axis[3 * j + 2]));
    m->jpos.push_back(v3<double>(d->jnt_pos[3 * j], d->jnt_pos[3 * j + 1], d->jnt_pos[3 * j + 2]));
    m->jqadr.push_back(qa); m->jdadr.push_back(da);
    qa += d->jnt_type[j] == J_FREE ? 7 : 1;
    da += d->jnt_type[j] == J_FREE ? 6 : 1;
  }
  m->nq = qa; m->nv = da;
  m->bdofs.assign(m->nb, {});
  for (int b = 0; b < m->nb; ++b) {
    for (int c = b; c >= 0; c = m->bparent[c])
      for (int j = m->bjnt0[c]; j < m->bjnt0[c] + m->bjntn[c]; ++j) {
        const int n = m->jtype[j] == J_FREE ? 6 : 1;
        for (int i = 0; i < n; ++i) m->bdofs[b].push_back(m->jdadr[j] + i);
      }
    std::sort(m->bdofs[b].begin(), m->bdofs[b].end());
  }
  for (int g = 0; g < m->ng; ++g) {
    m->gbody.push_back(d->geom_body[g]); m->gtype.push_back(d->geom_type[g]);
    m->gsize.push_back(v3<double>(d->geom_size[3 * g], d->geom_size[3 * g + 1], d->geom_size[3 * g + 2]));
    m->gpos.push_back(v3<double>(d->geom_pos[3 * g], d->geom_pos[3 * g + 1], d->geom_pos[3 * g + 2]));
    Q4<double> q; q.w = d->geom_quat[4 * g]; q.x = d->geom_quat[4 * g + 1]; q.y = d->geom_quat[4 * g + 2]; q.z = d->geom_quat[4 * g + 3];
    m->gquat.push_back(q);
  }
  m->ncmax = 0;
  for (int p = 0; p < m->np; ++p) {
    m->pg1.push_back(d->pair_g1[p]); m->pg2.push_back(d->pair_g2[p]); m->pmu.push_back(d->pair_mu[p]);
    for (int i = 0; i < 2; ++i) m->psolref.push_back(d->pair_solref[2 * p + i]);
    for (int i = 0; i < 5; ++i) { m->psolimp.push_back(d->pair_solimp[5 * p + i]); m->pcfd.push_back(d->pair_cfd[5 * p + i]); }
    int t1 = d->geom_type[d->pair_g1[p]], t2 = d->geom_type[d->pair_g2[p]];
    int nc = t1 == G_BOX ? 8 : t2 == G_SPHERE ? 1 : t2 == G_CAPSULE ? 2 : 4;
    m->pncon.push_back(nc); m->pcadr.push_back(m->ncmax); m->ncmax += nc;
  }
  for (int i = 0; i < m->nu; ++i) m->ctrl.push_back(d->ctrl_dof[i]);
  // Translational inverse weight of each body at the reference configuration
  // (joints at zero, free joints at the origin with identity orientation):
  // w_b = trace(Jp_b M^-1 Jp_b^T) / 3 (reading for the diagonal approximation).
  std::vector<double> q0(m->nq, 0.0);
  for (int j = 0; j < m->nj; ++j) if (m->jtype[j] == J_FREE) q0[m->jqadr[j] + 3] = 1.0;
  Kin<double> k;
  kinematics(*m, q0.data(), (const double*)nullptr, k);
  int nv = m->nv;
  std::vector<double> M(nv * nv), c(nv), Jp(3 * nv);
  std::vector<double> zv(nv, 0.0);
  kinematics(*m, q0.data(), zv.data(), k);
  mass_bias(*m, k, M.data(), c.data());
  std::vector<double> L = M;
  cholesky(L, nv);
  for (int b = 0; b < m->nb; ++b) {
    point_jac(*m, k, b, k.xpos[b], Jp.data(), (double*)nullptr);
    double tr = 0.0;
    for (int r = 0; r < 3; ++r) {
      std::vector<double> x(Jp.begin() + r * nv, Jp.begin() + (r + 1) * nv);
      chol_solve(L, nv, x);
      for (int i = 0; i < nv; ++i) tr += Jp[r * nv + i] * x[i];
    }
    m->binvw.push_back(tr / 3.0);
  }
  return m;
}

extern "C" void orc_model_free(void* m) { delete static_cast<Model*>(m); }

extern "C" void orc_model_sizes(const void* mp, int* out) {
  const Model& m = *static_cast<const Model*>(mp);
  out[0] = m.nq; out[1] = m.nv; out[2] = m.nu; out[3] = m.ncmax;
}

extern "C" void orc_model_inertia(const void* mp, double* mass, double* inertia, double* invw) {
  const Model& m = *static_cast<const Model*>(mp);
  for (int b = 0; b < m.nb; ++b) {
    mass[b] = m.bmass[b]; invw[b] = m.binvw[b];
    for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) inertia[9 * b + 3 * i + j] = m.biner[b].a[i][j];
  }
}

extern "C" int orc_kinematics(const void* mp, const double* q, const double* v, double* xpos, double* xmat,
                              double* M, double* c, double* twist) {
  const Model& m = *static_cast<const Model*>(mp);
  Kin<double> k;
  kinematics(m, q, v, k);
  for (int b = 0; b < m.nb; ++b) {
    for (int i = 0; i < 3; ++i) {
      if (xpos) xpos[3 * b + i] = k.xpos[b].x[i];
      if (twist) { twist[6 * b + i] = k.w[b].x[i]; twist[6 * b + 3 + i] = k.vel[b].x[i]; }
      for (int j = 0; j < 3; ++j) if (xmat) xmat[9 * b + 3 * i + j] = k.xmat[b].a[i][j];
    }
  }
  if (M && c) mass_bias(m, k, M, c);
  return 0;
}

extern "C" int orc_contacts(const void* mp, const double* q, double* out) {
  return orc_contacts_cfd(mp, q, 0, out);
}

extern "C" int orc_contacts_cfd(const void* mp, const double* q, int cfd, double* out) {
  const Model& m = *static_cast<const Model*>(mp);
  Kin<double> k;
  kinematics(m, q, (const double*)nullptr, k);
  std::vector<Contact<double>> cons;
  collide(m, k, cons, cfd != 0);
  for (size_t i = 0; i < cons.size(); ++i) {
    double* o = out + 13 * i;
    o[0] = cons[i].r;
    for (int r = 0; r < 3; ++r) { o[1 + r] = cons[i].pos.x[r]; o[4 + r] = cons[i].n.x[r]; o[7 + r] = cons[i].t1.x[r]; o[10 + r] = cons[i].t2.x[r]; }
  }
  return (int)cons.size();
}

extern "C" void orc_point_jac(const void* mp, const double* q, int body, const double* point, double* jac) {
  const Model& m = *static_cast<const Model*>(mp);
  Kin<double> k;
  kinematics(m, q, (const double*)nullptr, k);
  point_jac(m, k, body, v3<double>(point[0], point[1], point[2]), jac, (double*)nullptr);
}

extern "C" int orc_rhs(const void* mp, const double* x, const double* u, int cfd, double* xdot, int* info,
                       double* forces) {
  const Model& m = *static_cast<const Model*>(mp);
  Stats st;
  double uz = 0.0;
  std::vector<double> f;
  rhs(m, x, m.nu ? u : &uz, cfd != 0, 1e4, 100, xdot, &st, forces ? &f : nullptr);
  if (forces) for (size_t i = 0; i < f.size(); ++i) forces[i] = f[i];
  if (info) { info[0] = st.nrows; info[1] = st.nactive; info[2] = (int)st.newton_it; info[3] = st.status; }
  return st.status;
}

extern "C" int orc_rows(const void* mp, const double* x, const double* u, int cfd, double beta, double* M, double* a0,
                        double* J, double* aref, double* D) {
  const Model& m = *static_cast<const Model*>(mp);
  int nv = m.nv;
  Kin<double> kin;
  kinematics(m, x, x + m.nq, kin);
  std::vector<double> c(nv);
  mass_bias(m, kin, M, c.data());
  std::vector<double> f0(nv);
  for (int i = 0; i < nv; ++i) f0[i] = -c[i];
  for (int i = 0; i < m.nu; ++i) f0[m.ctrl[i]] += u[i];
  std::vector<double> L(M, M + nv * nv);
  cholesky(L, nv);
  chol_solve(L, nv, f0);
  for (int i = 0; i < nv; ++i) a0[i] = f0[i];
  std::vector<Contact<double>> cons;
  collide(m, kin, cons, cfd != 0);
  std::vector<Row<double>> rows;
  make_rows(m, kin, cons, x + m.nq, cfd != 0, beta, rows);
  for (size_t e = 0; e < rows.size(); ++e) {
    for (int i = 0; i < nv; ++i) J[e * nv + i] = rows[e].J[i];
    aref[e] = rows[e].aref; D[e] = rows[e].D;
  }
  return (int)rows.size();
}

extern "C" int orc_rhs_jvp(const void* mp, const double* x, const double* u, int stflag, double beta, int n_dir,
                           const double* dx, const double* du, double* xdot, double* dxdot) {
  const Model& m = *static_cast<const Model*>(mp);
  int nx = m.nq + m.nv, nv = m.nv;
  if (n_dir > kDir) return -1;
  std::vector<DualT> X(nx), U(std::max(m.nu, 1)), K(2 * nv);
  for (int i = 0; i < nx; ++i) { X[i] = DualT(x[i]); for (int d = 0; d < n_dir; ++d) X[i].d[d] = dx[d * nx + i]; }
  for (int i = 0; i < m.nu; ++i) { U[i] = DualT(u[i]); for (int d = 0; d < n_dir; ++d) U[i].d[d] = du[d * m.nu + i]; }
  Opts o; o.cfd = stflag != 0; o.beta = beta;
  Stats st;
  rhs_st(m, X.data(), U.data(), o, K.data(), &st);
  for (int i = 0; i < 2 * nv; ++i) { xdot[i] = K[i].v; for (int d = 0; d < n_dir; ++d) dxdot[d * 2 * nv + i] = K[i].d[d]; }
  return st.status;
}

extern "C" int orc_rollout(const void* mp, const double* x0, const double* u, int n_int, double dt_int,
                           const orc_opts* op, const double* forced, int n_forced, double* x_out,
                           long long* counters, int tape_cap, double* tape, int log_cap, double* steplog) {
  const Model& m = *static_cast<const Model*>(mp);
  Opts o = to_opts(op);
  Log lg;
  lg.keep_tape = tape != nullptr; lg.keep_log = steplog != nullptr;
  Stats st;
  rollout<double>(m, x0, u, n_int, dt_int, o, forced, n_forced, x_out, &lg, &st);
  int nx = m.nq + m.nv;
  if (tape) {
    size_t n = std::min((size_t)tape_cap, lg.tape.size() / (2 + nx));
    std::copy(lg.tape.begin(), lg.tape.begin() + n * (2 + nx), tape);
  }
  if (steplog) {
    size_t n = std::min((size_t)log_cap, lg.steplog.size() / 4);
    std::copy(lg.steplog.begin(), lg.steplog.begin() + 4 * n, steplog);
  }
  if (counters) { counters[0] = lg.n_acc; counters[1] = lg.n_rej; counters[2] = st.rhs; counters[3] = st.newton_it; counters[4] = st.status; }
  return st.status;
}

// ------------------------------------------------------------------ optimize-then-discretize adjoint
// The continuous adjoint equations (App. C.2, eq. adjoint-equations; with the
// straight-through rule, App. C.4: the Jacobian of the CFD field F~ taken at
// the trajectory of F): for a loss on the final state, a(T) = dL/dx(T) and
// da/dt = -(dF/dx)^T a, and the controls' gradient a_u = integral over each
// interval of (dF/du)^T a; dL/dx(0) = a(0).  They are solved backwards in
// time with the same adaptive Dormand-Prince pair and PI controller as the
// forward ODE, with its own steps.
// reading: the state is taken in its raw coordinates, x = (q, v) with the
// quaternions as 4-vectors, dq/dt = v for positions and hinge/slide joints and
// (1/2) q (x) (0, omega) for a free joint's quaternion (omega in the body
// frame); the returned quaternion gradient is projected onto the tangent
// space of the unit sphere at q(0), as the discrete adjoint's is (its (+) map
// normalizes).
// reading: x(t) between the forward's accepted steps is that step's
// fourth-order continuous extension (Hairer, Norsett and Wanner's dense output
// of the Dormand-Prince pair), applied to the tangent increment and mapped
// through (+), rather than the forward ODE solved backwards together with the
// adjoint (unstable for dissipative contacts); the continuous extension's
// coefficients are those of that published scheme.
// reading: the adjoint's error estimate is the RMS over the nq + nv components
// of a, scaled by atol + rtol max(|a_j|, |a_new_j|) (the forward's norm); its
// first step is the forward's last step size; its steps land on the control
// interval ends as the forward's do.
// reading: the adjoint's steps are floored at 1e-12 max(1, |t|), and a step at
// the floor is accepted whatever its error estimate: where a contact switches
// on, dF/dx jumps (by the damping and stiffness terms, up to ~1e4 here), and
// no step size resolves a jump to a tight tolerance; a floor step carries
// that jump's error, of order the floor times the jump.
static const double RK_D[7] = {-12715105075.0 / 11282082432.0, 0.0, 87487479700.0 / 32700410799.0,
                               -10690763975.0 / 1880347072.0, 701980252875.0 / 199316789632.0,
                               -1453857185.0 / 822651844.0, 69997945.0 / 29380423.0};

// weights of the stage slopes in the continuous extension: the increment over
// the fraction th of a step of size h is h sum_i w_i(th) k_i, with
// w(th) = th b + th (1 - th) (e_1 - b) + th^2 (1 - th) (2 b - e_1 - e_7)
//         + th^2 (1 - th)^2 d
static void dense_weights(double th, double* w) {
  for (int i = 0; i < 7; ++i) {
    const double e1 = i == 0 ? 1.0 : 0.0, e7 = i == 6 ? 1.0 : 0.0;
    w[i] = th * RK_B[i] + th * (1.0 - th) * (e1 - RK_B[i]) + th * th * (1.0 - th) * (2.0 * RK_B[i] - e1 - e7) +
           th * th * (1.0 - th) * (1.0 - th) * RK_D[i];
  }
}

// rates of the raw coordinates from the tangent-form right-hand side k = (v, qacc)
template <class S>
static void raw_rates(const Model& m, const S* x, const S* k, S* out) {
  for (int j = 0; j < m.nj; ++j) {
    const int qa = m.jqadr[j], da = m.jdadr[j];
    if (m.jtype[j] == J_FREE) {
      for (int i = 0; i < 3; ++i) out[qa + i] = k[da + i];
      Q4<S> q; q.w = x[qa + 3]; q.x = x[qa + 4]; q.y = x[qa + 5]; q.z = x[qa + 6];
      Q4<S> w; w.w = S(0.0); w.x = k[da + 3]; w.y = k[da + 4]; w.z = k[da + 5];
      const Q4<S> r = qmul(q, w);
      out[qa + 3] = r.w * 0.5; out[qa + 4] = r.x * 0.5; out[qa + 5] = r.y * 0.5; out[qa + 6] = r.z * 0.5;
    } else {
      out[qa] = k[da];
    }
  }
  for (int d = 0; d < m.nv; ++d) out[m.nq + d] = k[m.nv + d];
}

// g = (dF/dx)^T lam and gu = (dF/du)^T lam at (x, u) in raw coordinates,
// from the forward-mode tangents of F (of F~ with CFD on), kDir directions at
// a time
static void raw_vjp(const Model& m, const double* x, const double* u, const Opts& o, const double* lam, double* g,
                    double* gu, Stats* st) {
  const int nx = m.nq + m.nv, nd = nx + m.nu;
  std::vector<DualT> X(nx), U(std::max(m.nu, 1)), K(2 * m.nv), R(nx);
  for (int d0 = 0; d0 < nd; d0 += kDir) {
    for (int i = 0; i < nx; ++i) { X[i] = DualT(x[i]); if (i >= d0 && i < d0 + kDir) X[i].d[i - d0] = 1.0; }
    for (int i = 0; i < m.nu; ++i) {
      U[i] = DualT(u[i]);
      if (nx + i >= d0 && nx + i < d0 + kDir) U[i].d[nx + i - d0] = 1.0;
    }
    rhs_st(m, X.data(), U.data(), o, K.data(), st);
    raw_rates(m, X.data(), K.data(), R.data());
    for (int c = d0; c < std::min(nd, d0 + kDir); ++c) {
      double s = 0.0;
      for (int r = 0; r < nx; ++r) s += R[r].d[c - d0] * lam[r];
      if (c < nx) g[c] = s; else gu[c - nx] = s;
    }
  }
}

// One world: the forward rollout (kept: accepted steps), then the adjoint
// solved backwards.  counters: adjoint attempts, adjoint accepted steps.
static int otd_world(const Model& m, const double* x0, const double* u, int n_int, double dt, const Opts& o,
                     const double* xbar, double* x_out, double* x0bar, double* ubar, long long* counters) {
  const int nq = m.nq, nv = m.nv, nx = nq + nv, nu = m.nu;
  Log lg;
  lg.keep_tape = true;
  Stats st;
  rollout<double>(m, x0, u, n_int, dt, o, nullptr, 0, x_out, &lg, &st);
  const size_t nut = (size_t)n_int * nu;
  if (o.tableau != 0) st.status |= ORC_UNSUPPORTED;  // the continuous extension is the Dormand-Prince pair's
  if (st.status & ~ORC_CONTACT_OVERFLOW) {
    for (int i = 0; i < nx; ++i) x0bar[i] = NAN;
    for (size_t i = 0; i < nut; ++i) ubar[i] = NAN;
    return st.status;
  }
  const int N = (int)lg.n_acc;
  const size_t rl = 2 + nx;
  auto t_of = [&](int n) { return lg.tape[n * rl]; };
  auto h_of = [&](int n) { return lg.tape[n * rl + 1]; };
  std::vector<double> uz(1, 0.0);
  auto u_of = [&](int kk) { return nu > 0 ? u + (size_t)kk * nu : uz.data(); };
  auto interval_of = [&](int n) {
    int kk = (int)std::floor((t_of(n) + 0.5 * h_of(n)) / dt);
    return std::min(std::max(kk, 0), n_int - 1);
  };
  // stage slopes of accepted step n, solved again (the forward's right-hand
  // sides are functions of the state: the same values)
  std::vector<std::vector<std::vector<double>>> slopes(N);
  auto step_slopes = [&](int n) -> const std::vector<std::vector<double>>& {
    if (slopes[n].empty()) {
      const double* y = &lg.tape[n * rl + 2];
      const double* uk = u_of(interval_of(n));
      std::vector<double> k1(2 * nv), yn(nx), k7(2 * nv);
      Stats s2;
      rhs_st(m, y, uk, o, k1.data(), &s2);
      dopri_attempt(m, y, uk, k1, h_of(n), o, false, yn.data(), k7, &s2, &slopes[n]);
    }
    return slopes[n];
  };
  // x(tau) from the continuous extension of the step that holds tau
  auto dense = [&](double tau, double* xo) {
    int n = N - 1;
    for (int i = 0; i < N; ++i)
      if (tau < t_of(i) + h_of(i)) { n = i; break; }
    const double h = h_of(n);
    const double th = std::min(1.0, std::max(0.0, (tau - t_of(n)) / h));
    double w[7];
    dense_weights(th, w);
    const std::vector<std::vector<double>>& K = step_slopes(n);
    const double* y = &lg.tape[n * rl + 2];
    std::vector<double> dq(nv);
    for (int d = 0; d < nv; ++d) {
      double sq = 0.0, sv = 0.0;
      for (int i = 0; i < 7; ++i) { sq += w[i] * K[i][d]; sv += w[i] * K[i][nv + d]; }
      dq[d] = h * sq;
      xo[nq + d] = y[nq + d] + h * sv;
    }
    qplus(m, y, dq.data(), xo);
  };
  // start of the last accepted forward step that begins before t: the
  // adjoint's steps end on the forward's step boundaries, never across them
  // (reading of App. C.2: the adjoint chooses its own steps, within each step
  // of the forward whose continuous extension it reads, so that the short
  // steps the forward took through a contact phase are never skipped)
  auto step_start = [&](double t) {
    double s = 0.0;
    for (int i = 0; i < N; ++i)
      if (t_of(i) < t) s = t_of(i);
    return s;
  };
  std::vector<double> lam(xbar, xbar + nx), lamn(nx), Lam(nx), xs(nx), e(nx);
  std::vector<std::vector<double>> G(7, std::vector<double>(nx)), GU(7, std::vector<double>(std::max(nu, 1)));
  for (size_t i = 0; i < nut; ++i) ubar[i] = 0.0;
  double hprop = N > 0 ? h_of(N - 1) : std::min(o.h0, dt), eprev = 1.0;
  long long attempts = 0, accepted = 0;
  int status = 0;
  for (int kk = n_int - 1; kk >= 0 && !status; --kk) {
    const double* uk = u_of(kk);
    const double tlo = (double)kk * dt;
    double t = (double)(kk + 1) * dt;
    bool have_g1 = false;
    while (t > tlo) {
      const double lo = std::max(tlo, step_start(t));
      const bool landing = t - 1.01 * hprop <= lo;
      const double H = landing ? t - lo : hprop;
      if (attempts >= o.max_attempts) { status |= ORC_MAX_STEPS; break; }
      ++attempts;
      for (int i = 0; i < 7; ++i) {
        if (i == 0 && have_g1) continue;
        for (int r = 0; r < nx; ++r) {
          double s = 0.0;
          for (int j = 0; j < i; ++j) s += RK_A[i][j] * G[j][r];
          Lam[r] = lam[r] + H * s;
        }
        dense(t - RK_C[i] * H, xs.data());
        Stats s2;
        raw_vjp(m, xs.data(), uk, o, Lam.data(), G[i].data(), GU[i].data(), &s2);
        if (s2.status & (ORC_NONFINITE | ORC_SOLVER_MAXIT)) status |= s2.status & (ORC_NONFINITE | ORC_SOLVER_MAXIT);
      }
      if (status) break;
      double acc = 0.0;
      for (int r = 0; r < nx; ++r) {
        double s5 = 0.0, se = 0.0;
        for (int i = 0; i < 7; ++i) { s5 += RK_B[i] * G[i][r]; se += (RK_B[i] - RK_BH[i]) * G[i][r]; }
        lamn[r] = lam[r] + H * s5;
        e[r] = H * se;
        const double sc = o.atol + o.rtol * std::max(std::fabs(lam[r]), std::fabs(lamn[r]));
        acc += (e[r] / sc) * (e[r] / sc);
      }
      if (!finite_vec(lamn.data(), nx)) { status |= ORC_NONFINITE; break; }
      const double err = std::sqrt(acc / nx);
      const double hmin = 1e-12 * std::max(1.0, std::fabs(t));
      const bool accept = err <= 1.0 || H <= hmin;
      const double hnext = next_step(o, err, eprev, H, accept, &eprev);
      if (accept) {
        for (int i = 0; i < nu; ++i) {
          double s = 0.0;
          for (int j = 0; j < 7; ++j) s += RK_B[j] * GU[j][i];
          ubar[(size_t)kk * nu + i] += H * s;
        }
        lam = lamn;
        G[0] = G[6];
        GU[0] = GU[6];
        have_g1 = true;
        t = landing ? lo : t - H;
        ++accepted;
      }
      hprop = std::max(hnext, hmin);
    }
  }
  for (int i = 0; i < nx; ++i) x0bar[i] = lam[i];
  for (int j = 0; j < m.nj; ++j) {  // quaternion gradients: tangent part at q(0)
    if (m.jtype[j] != J_FREE) continue;
    const int qa = m.jqadr[j] + 3;
    double nn = 0.0, dp = 0.0;
    for (int i = 0; i < 4; ++i) nn += x0[qa + i] * x0[qa + i];
    for (int i = 0; i < 4; ++i) dp += x0bar[qa + i] * x0[qa + i];
    for (int i = 0; i < 4; ++i) x0bar[qa + i] -= dp / nn * x0[qa + i];
  }
  if (status) {
    for (int i = 0; i < nx; ++i) x0bar[i] = NAN;
    for (size_t i = 0; i < nut; ++i) ubar[i] = NAN;
  }
  if (counters) { counters[0] = attempts; counters[1] = accepted; counters[2] = N; counters[3] = status; }
  return status;
}

// Operation count of a forward rollout: the same rollout in the counting
// scalar (values equal those of orc_rollout), per phase of the method.
extern "C" int orc_flop_count(const void* mp, const double* x0, const double* u, int n_int, double dt_int,
                              const orc_opts* op, long long* out) {
  const Model& m = *static_cast<const Model*>(mp);
  Opts o = to_opts(op);
  const int nx = m.nq + m.nv;
  std::vector<Flop> X(nx), U, Y(nx);
  for (int i = 0; i < nx; ++i) X[i] = Flop::data(x0[i]);
  for (size_t i = 0; i < (size_t)n_int * m.nu; ++i) U.push_back(Flop::data(u[i]));
  if (U.empty()) U.assign(1, Flop(0.0));
  Log lg;
  Stats st;
  FlopTally& t = flop_tally();
  const FlopTally before = t;
  rollout<Flop>(m, X.data(), U.data(), n_int, dt_int, o, nullptr, 0, Y.data(), &lg, &st);
  for (int p = 0; p < kPhases; ++p) out[p] = t.n[p] - before.n[p];
  out[5] = lg.n_acc + lg.n_rej;
  out[6] = st.rhs;
  out[7] = st.newton_it;
  out[8] = st.contacts;
  out[9] = st.newton_contacts;
  out[10] = st.ls_contacts;
  out[11] = lg.n_acc;
  out[12] = st.status;
  out[13] = st.contacts_box;
  out[14] = st.newton_contacts_box;
  out[15] = st.ls_contacts_box;
  return st.status;
}

extern "C" void orc_dense_weights(double theta, double* w) { dense_weights(theta, w); }

// The forward trajectory x(tau) of one world at n_tau times, from the
// continuous extension of its accepted steps (forced: replayed steps, as for
// orc_rollout).
extern "C" int orc_dense_states(const void* mp, const double* x0, const double* u, int n_int, double dt_int,
                                const orc_opts* op, const double* forced, int n_forced, int n_tau, const double* tau,
                                double* out) {
  const Model& m = *static_cast<const Model*>(mp);
  Opts o = to_opts(op);
  const int nq = m.nq, nv = m.nv, nx = nq + nv, nu = m.nu;
  Log lg;
  lg.keep_tape = true;
  Stats st;
  std::vector<double> xo(nx);
  rollout<double>(m, x0, u, n_int, dt_int, o, forced, n_forced, xo.data(), &lg, &st);
  if (st.status & ~ORC_CONTACT_OVERFLOW) return st.status;
  const int N = (int)lg.n_acc;
  const size_t rl = 2 + nx;
  std::vector<double> uz(1, 0.0);
  for (int k = 0; k < n_tau; ++k) {
    int n = N - 1;
    for (int i = 0; i < N; ++i)
      if (tau[k] < lg.tape[i * rl] + lg.tape[i * rl + 1]) { n = i; break; }
    const double t0 = lg.tape[n * rl], h = lg.tape[n * rl + 1];
    const double* y = &lg.tape[n * rl + 2];
    int kk = std::min(std::max((int)std::floor((t0 + 0.5 * h) / dt_int), 0), n_int - 1);
    const double* uk = nu > 0 ? u + (size_t)kk * nu : uz.data();
    std::vector<double> k1(2 * nv), yn(nx), k7(2 * nv);
    std::vector<std::vector<double>> K;
    Stats s2;
    rhs_st(m, y, uk, o, k1.data(), &s2);
    dopri_attempt(m, y, uk, k1, h, o, false, yn.data(), k7, &s2, &K);
    double w[7];
    dense_weights(std::min(1.0, std::max(0.0, (tau[k] - t0) / h)), w);
    std::vector<double> dq(nv);
    double* xk = out + (size_t)k * nx;
    for (int d = 0; d < nv; ++d) {
      double sq = 0.0, sv = 0.0;
      for (int i = 0; i < 7; ++i) { sq += w[i] * K[i][d]; sv += w[i] * K[i][nv + d]; }
      dq[d] = h * sq;
      xk[nq + d] = y[nq + d] + h * sv;
    }
    qplus(m, y, dq.data(), xk);
  }
  return 0;
}

// Operation count of the oracle's Cholesky factorization and solve of an n x n
// matrix (row-major; zero entries are taken as structural zeros, the others
// as data), for checking the counting rules against closed forms.
extern "C" long long orc_flop_cholesky(const double* A, int n) {
  std::vector<Flop> L(n * n), x(n);
  for (int i = 0; i < n * n; ++i) L[i] = A[i] == 0.0 ? Flop(0.0) : Flop::data(A[i]);
  for (int i = 0; i < n; ++i) x[i] = Flop::data(1.0 + i);
  FlopPhase phase(kPhOther);
  const long long before = flop_tally().n[kPhOther];
  if (!cholesky(L, n)) return -1;
  chol_solve(L, n, x);
  return flop_tally().n[kPhOther] - before;
}

// forward-mode pass with frozen steps: y tangents for up to kDir directions
static int jvp_pass(const Model& m, const double* x0, const double* u, int n_int, double dt, const Opts& o,
                    const std::vector<double>& forced, int n_dir, const double* dx0, const double* du,
                    double* xout, double* tx, Stats* st) {
  int nx = m.nq + m.nv;
  size_t nut = (size_t)n_int * m.nu;
  std::vector<DualT> X(nx), U(std::max<size_t>(nut, 1)), XO(nx);
  for (int i = 0; i < nx; ++i) { X[i] = DualT(x0[i]); for (int d = 0; d < n_dir; ++d) X[i].d[d] = dx0 ? dx0[d * nx + i] : 0.0; }
  for (size_t i = 0; i < nut; ++i) { U[i] = DualT(u[i]); for (int d = 0; d < n_dir; ++d) U[i].d[d] = du ? du[d * nut + i] : 0.0; }
  rollout<DualT>(m, X.data(), U.data(), n_int, dt, o, forced.data(), (int)forced.size() / 2, XO.data(), nullptr, st);
  for (int i = 0; i < nx; ++i) { if (xout) xout[i] = XO[i].v; for (int d = 0; d < n_dir; ++d) tx[d * nx + i] = XO[i].d[d]; }
  return st->status;
}

static std::vector<double> accepted_steps(const Model& m, const double* x0, const double* u, int n_int, double dt,
                                          const Opts& o, double* xout, Stats* st, Log* lgout) {
  Log lg;
  lg.keep_tape = true;
  int nx = m.nq + m.nv;
  std::vector<double> xo(nx);
  rollout<double>(m, x0, u, n_int, dt, o, nullptr, 0, xo.data(), &lg, st);
  if (xout) std::copy(xo.begin(), xo.end(), xout);
  std::vector<double> f;
  for (size_t i = 0; i < lg.tape.size(); i += 2 + nx) { f.push_back(lg.tape[i]); f.push_back(lg.tape[i + 1]); }
  if (lgout) { lgout->n_acc = lg.n_acc; lgout->n_rej = lg.n_rej; }
  return f;
}

extern "C" int orc_rollout_jvp(const void* mp, const double* x0, const double* u, int n_int, double dt_int,
                               const orc_opts* op, int n_dir, const double* dx0, const double* du, double* x_out,
                               double* tx, long long* counters) {
  const Model& m = *static_cast<const Model*>(mp);
  if (n_dir > kDir) return -1;
  Opts o = to_opts(op);
  Stats st;
  Log lg;
  std::vector<double> f = accepted_steps(m, x0, u, n_int, dt_int, o, x_out, &st, &lg);
  if (st.status) return st.status;
  Stats st2;
  jvp_pass(m, x0, u, n_int, dt_int, o, f, n_dir, dx0, du, nullptr, tx, &st2);
  if (counters) { counters[0] = lg.n_acc; counters[1] = lg.n_rej; counters[2] = st.rhs; counters[3] = st.newton_it; counters[4] = st.status | st2.status; }
  return st.status | st2.status;
}

template <class F>
static void parallel_for(int n, int n_threads, F fn) {
  if (n_threads <= 1) { for (int i = 0; i < n; ++i) fn(i); return; }
  std::atomic<int> next(0);
  std::vector<std::thread> th;
  for (int t = 0; t < n_threads; ++t)
    th.emplace_back([&]() { for (int i = next++; i < n; i = next++) fn(i); });
  for (auto& x : th) x.join();
}

extern "C" int orc_rollout_batch(const void* mp, int W, const double* x0, const double* u, int n_int, double dt_int,
                                 const orc_opts* op, double* x_out, long long* counters, int n_threads) {
  const Model& m = *static_cast<const Model*>(mp);
  Opts o = to_opts(op);
  int nx = m.nq + m.nv;
  size_t nut = (size_t)n_int * m.nu;
  parallel_for(W, n_threads, [&](int w) {
    Log lg; Stats st;
    rollout<double>(m, x0 + (size_t)w * nx, u + w * nut, n_int, dt_int, o, nullptr, 0, x_out + (size_t)w * nx, &lg, &st);
    long long* c = counters + 5 * (size_t)w;
    c[0] = lg.n_acc; c[1] = lg.n_rej; c[2] = st.rhs; c[3] = st.newton_it; c[4] = st.status;
  });
  return 0;
}

// Gradient J^T xbar of the final state w.r.t. (x0, u) of one world along the
// frozen accepted-step sequence f = (t_n, h_n): the full Jacobian is formed by
// forward-mode passes of kDir unit directions.
static int grad_world(const Model& m, const double* xw, const double* uw, int n_int, double dt, const Opts& o,
                      const std::vector<double>& f, const double* xb, double* x0b, double* ub, long long* nrhs) {
  int nx = m.nq + m.nv;
  size_t nut = (size_t)n_int * m.nu;
  size_t nin = nx + nut;
  int status = 0;
  std::vector<double> dx0(kDir * nx), du(kDir * std::max<size_t>(nut, 1)), tx(kDir * nx);
  for (size_t c0 = 0; c0 < nin && !status; c0 += kDir) {
    int nd = (int)std::min<size_t>(kDir, nin - c0);
    std::fill(dx0.begin(), dx0.end(), 0.0);
    std::fill(du.begin(), du.end(), 0.0);
    for (int d = 0; d < nd; ++d) {
      size_t idx = c0 + d;
      if (idx < (size_t)nx) dx0[d * nx + idx] = 1.0; else du[d * nut + (idx - nx)] = 1.0;
    }
    Stats s2;
    jvp_pass(m, xw, uw, n_int, dt, o, f, nd, dx0.data(), du.data(), nullptr, tx.data(), &s2);
    status |= s2.status; *nrhs += s2.rhs;
    for (int d = 0; d < nd; ++d) {
      double g = 0.0;
      for (int i = 0; i < nx; ++i) g += xb[i] * tx[d * nx + i];
      size_t idx = c0 + d;
      if (idx < (size_t)nx) x0b[idx] = g; else ub[idx - nx] = g;
    }
  }
  return status;
}

// Forward-mode tangents of one rollout along a given frozen step sequence.
extern "C" int orc_rollout_jvp_forced(const void* mp, const double* x0, const double* u, int n_int, double dt_int,
                                      const orc_opts* op, const double* forced, int n_forced, int n_dir,
                                      const double* dx0, const double* du, double* x_out, double* tx) {
  const Model& m = *static_cast<const Model*>(mp);
  if (n_dir > kDir) return -1;
  Opts o = to_opts(op);
  std::vector<double> f(forced, forced + 2 * (size_t)n_forced);
  Stats st;
  return jvp_pass(m, x0, u, n_int, dt_int, o, f, n_dir, dx0, du, x_out, tx, &st);
}

// Gradients of every world of a batch along the world's own adaptive run.
extern "C" int orc_grad_batch(const void* mp, int W, const double* x0, const double* u, int n_int, double dt_int,
                              const orc_opts* op, const double* xbar, double* x_out, double* x0bar, double* ubar,
                              long long* counters, int n_threads) {
  const Model& m = *static_cast<const Model*>(mp);
  Opts o = to_opts(op);
  int nx = m.nq + m.nv;
  size_t nut = (size_t)n_int * m.nu;
  parallel_for(W, n_threads, [&](int w) {
    const double* xw = x0 + (size_t)w * nx;
    const double* uw = u + w * nut;
    Stats st; Log lg;
    std::vector<double> f = accepted_steps(m, xw, uw, n_int, dt_int, o, x_out + (size_t)w * nx, &st, &lg);
    long long nit = st.newton_it, nrhs = st.rhs;
    int status = st.status;
    if (!status) status |= grad_world(m, xw, uw, n_int, dt_int, o, f, xbar + (size_t)w * nx, x0bar + (size_t)w * nx,
                                      ubar + w * nut, &nrhs);
    long long* c = counters + 5 * (size_t)w;
    c[0] = lg.n_acc; c[1] = lg.n_rej; c[2] = nrhs; c[3] = nit; c[4] = status;
  });
  return 0;
}

// The same along given accepted-step sequences: world w replays its
// forced_n[w] steps forced[w][i] = (t_i, h_i) (the controller is off), and its
// end state and gradient are those of that frozen discretization.
extern "C" int orc_grad_forced_batch(const void* mp, int W, const double* x0, const double* u, int n_int,
                                     double dt_int, const orc_opts* op, const double* forced, const int* forced_n,
                                     int forced_cap, const double* xbar, double* x_out, double* x0bar, double* ubar,
                                     long long* counters, int n_threads) {
  const Model& m = *static_cast<const Model*>(mp);
  Opts o = to_opts(op);
  int nx = m.nq + m.nv;
  size_t nut = (size_t)n_int * m.nu;
  parallel_for(W, n_threads, [&](int w) {
    const double* xw = x0 + (size_t)w * nx;
    const double* uw = u + w * nut;
    std::vector<double> f(forced + (size_t)w * forced_cap * 2, forced + ((size_t)w * forced_cap + forced_n[w]) * 2);
    Stats st; Log lg;
    rollout<double>(m, xw, uw, n_int, dt_int, o, f.data(), forced_n[w], x_out + (size_t)w * nx, &lg, &st);
    long long nrhs = st.rhs;
    int status = st.status;
    if (!status) status |= grad_world(m, xw, uw, n_int, dt_int, o, f, xbar + (size_t)w * nx, x0bar + (size_t)w * nx,
                                      ubar + w * nut, &nrhs);
    long long* c = counters + 5 * (size_t)w;
    c[0] = lg.n_acc; c[1] = lg.n_rej; c[2] = nrhs; c[3] = st.newton_it; c[4] = status;
  });
  return 0;
}

// One Dormand-Prince attempt from state y with step h under the controls u
// (the first stage evaluated at y): the 5th-order state and the error norm.
extern "C" int orc_attempt(const void* mp, const double* y, const double* u, double h, const orc_opts* op,
                           double* ynew, double* err) {
  const Model& m = *static_cast<const Model*>(mp);
  Opts o = to_opts(op);
  int nv = m.nv;
  std::vector<double> k1(2 * nv), k7(2 * nv);
  double uz = 0.0;
  const double* uk = m.nu > 0 ? u : &uz;
  Stats st;
  rhs_st(m, y, uk, o, k1.data(), &st);
  *err = dopri_attempt(m, y, uk, k1, h, o, true, ynew, k7, &st);
  return st.status;
}

// The controller's next proposed step after an attempt with error norm err
// (eprev_out receives the controller's memory for the next attempt).
extern "C" double orc_next_step(const orc_opts* op, double err, double eprev, double h, int accepted,
                                double* eprev_out) {
  Opts o = to_opts(op);
  return next_step(o, err, eprev, h, accepted != 0, eprev_out);
}

extern "C" int orc_otd_grad_batch(const void* mp, int W, const double* x0, const double* u, int n_int,
                                  double dt_int, const orc_opts* op, const double* xbar, double* x_out,
                                  double* x0bar, double* ubar, long long* counters, int n_threads) {
  const Model& m = *static_cast<const Model*>(mp);
  Opts o = to_opts(op);
  const int nx = m.nq + m.nv;
  const size_t nut = (size_t)n_int * m.nu;
  parallel_for(W, n_threads, [&](int w) {
    otd_world(m, x0 + (size_t)w * nx, u + w * nut, n_int, dt_int, o, xbar + (size_t)w * nx,
              x_out + (size_t)w * nx, x0bar + (size_t)w * nx, ubar + w * nut, counters + 4 * (size_t)w);
  });
  return 0;
}
