// Contact geometry of box worlds and its reverse.
//
//  - plane-box: the smoothed four-deepest-vertex detection of App. C.1;
//  - box-box: the separating-axis test over the 15 candidate axes with face
//    clipping or one crossing-edge contact (primitive-vs-primitive detection
//    of Sec. 2.1).
//
// Every contact comes with a code: the discrete choices that made it (the
// separating axis, the reference and incident faces, which corner, edge
// crossing or corner line of the clipped face, the top-four vertex and
// whether the skin threshold was on).  The reverse sweep rebuilds the
// contact's construction from its code and the poses and differentiates
// point, depth and normal along it, the choices held fixed as in any
// derivative of a contact set.
#pragma once
#include "dmx_common.hpp"

namespace dmx {

DMX_DEV V3 colv(const double* R, int j) { return mk3(R[j], R[3 + j], R[6 + j]); }
DMX_DEV void col_add(double* Rb, int j, V3 v) { Rb[j] += v.x; Rb[3 + j] += v.y; Rb[6 + j] += v.z; }

// Tangent frame of a unit normal (a = e_x unless |n_x| >= 0.5, then e_y):
// t1 = normalized (a - (a.n) n), t2 = n x t1.
DMX_DEV void make_frame(V3 n, V3* t1, V3* t2) {
  const V3 a = fabs(n.x) < 0.5 ? mk3(1.0, 0.0, 0.0) : mk3(0.0, 1.0, 0.0);
  const V3 t = a - dot(a, n) * n;
  *t1 = (1.0 / sqrt(dot(t, t))) * t;
  *t2 = cross(n, *t1);
}
// cotangent of n from those of t1 and t2
DMX_DEV V3 make_frame_vjp(V3 n, V3 t1b, V3 t2b) {
  const V3 a = fabs(n.x) < 0.5 ? mk3(1.0, 0.0, 0.0) : mk3(0.0, 1.0, 0.0);
  const V3 t = a - dot(a, n) * n;
  const double inv = 1.0 / sqrt(dot(t, t));
  const V3 t1 = inv * t;
  V3 nb = cross(t1, t2b);  // t2 = n x t1
  const V3 t1t = t1b + cross(t2b, n);
  const V3 tb = inv * (t1t - dot(t1, t1t) * t1);
  nb -= dot(a, n) * tb + dot(n, tb) * a;  // t = a - (a.n) n
  return nb;
}

// ------------------------------------------------------------ contact codes
// bits 0-2 kind, 3-5 and 6-8 two indices, 9 a flag, 10-13 the separating
// axis (face 0-5 or edge 0-8), 14 set for an edge axis, 15-21 orientation
// signs of the construction.
enum { kRcCorner = 0, kRcCross = 1, kRcLine = 2, kRcVertex = 3, kRcEdges = 4 };
DMX_DEV int rc_kind(int c) { return c & 7; }
DMX_DEV int rc_i(int c) { return (c >> 3) & 7; }
DMX_DEV int rc_j(int c) { return (c >> 6) & 7; }
DMX_DEV bool rc_flag(int c) { return (c >> 9) & 1; }
DMX_DEV int rc_axis(int c) { return (c >> 10) & 15; }
DMX_DEV bool rc_bit(int c, int b) { return (c >> b) & 1; }

// ------------------------------------------------------------ plane-box
// Vertex k of the box (centre c, rotation R, half sizes h; coordinate signs
// from the bits of k: x bit 0, y bit 1, z bit 2) is x_k = c + R s_k and
// penetrates the plane (point p0, normal n) by e_k = -n.(x_k - p0).  With the
// skin 1 mm and tau = max(0, e_max - skin), w_k = smoothstep((e_k - (tau -
// skin)) / skin) (C^1 smoothstep t^2 (3 - 2t) on [0, 1]) and z_k = w_k e_k;
// the four largest z_k (ties to the lower vertex index) give r = -z_k at
// x_k + (z_k / 2) n.  Candidates with r >= margin are dropped.
// Code: vertex k, the deepest vertex, the threshold flag.
DMX_DEV V3 box_corner(const double* h, int k) {
  return mk3((k & 1) ? h[0] : -h[0], (k & 2) ? h[1] : -h[1], (k & 4) ? h[2] : -h[2]);
}
DMX_DEV double smoothstep(double u, double* du) {
  if (u <= 0.0) { *du = 0.0; return 0.0; }
  if (u >= 1.0) { *du = 0.0; return 1.0; }
  *du = 6.0 * u * (1.0 - u);
  return u * u * (3.0 - 2.0 * u);
}

constexpr double kPlaneSkin = 1e-3;

DMX_DEV int box_plane(const double* h, const double* p0, const double* pn, V3 c, const M3& R, double margin,
                      double* r_out, V3* p_out, int* code) {
  const V3 n = ld3(pn), q0 = ld3(p0);
  double e[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) e[k] = -dot(n, c + mul(R, box_corner(h, k)) - q0);
  int kmax = 0;
  double emax = e[0];
#pragma unroll
  for (int k = 1; k < 8; ++k)
    if (e[k] > emax) { emax = e[k]; kmax = k; }
  const bool tau_on = emax > kPlaneSkin;
  const double tau = tau_on ? emax - kPlaneSkin : 0.0;
  double z[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) { double du; z[k] = smoothstep((e[k] - (tau - kPlaneSkin)) / kPlaneSkin, &du) * e[k]; }
  int rk[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    rk[k] = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) rk[k] += (z[j] > z[k]) || (j < k && z[j] == z[k]);
  }
  // the candidates that pass the margin are a prefix of the rank order
  int cnt = 0;
#pragma unroll
  for (int slot = 0; slot < 4; ++slot) {
    int k = 0;
    double zk = z[0];
#pragma unroll
    for (int q = 1; q < 8; ++q)
      if (rk[q] == slot) { k = q; zk = z[q]; }
    if (-zk < margin) {
      if (r_out) {
        r_out[slot] = -zk;
        p_out[slot] = c + mul(R, box_corner(h, k)) + (0.5 * zk) * n;
      }
      if (code) code[slot] = kRcVertex | (k << 3) | (kmax << 6) | (tau_on ? 1 << 9 : 0);
      cnt = slot + 1;
    }
  }
  return cnt;
}

// cotangents of the box pose (c_bar += , R_bar += ) from those of one
// plane-box contact (r_bar, p_bar); the normal is the plane's
DMX_DEV void box_plane_vjp(const double* h, const double* p0, const double* pn, V3 c, const M3& R, int code,
                           double rb, V3 pb, V3* cb, double* Rb) {
  const V3 n = ld3(pn), q0 = ld3(p0);
  const V3 sk = box_corner(h, rc_i(code)), sm = box_corner(h, rc_j(code));
  const double ek = -dot(n, c + mul(R, sk) - q0);
  const double em = -dot(n, c + mul(R, sm) - q0);
  const bool tau_on = rc_flag(code);
  const double tau = tau_on ? em - kPlaneSkin : 0.0;
  double du;
  const double w = smoothstep((ek - (tau - kPlaneSkin)) / kPlaneSkin, &du);
  // r = -z, p = x_k + (z/2) n, z = w e_k
  const double zb = -rb + 0.5 * dot(n, pb);
  const double wb = zb * ek;
  const double ekb = zb * w + wb * du / kPlaneSkin;
  const double taub = -wb * du / kPlaneSkin;
  const V3 xk = pb - ekb * n;                                    // x_k bar
  const V3 xm = tau_on ? (-taub) * n : mk3(0.0, 0.0, 0.0);       // e_max = -n.(x_m - p0)
  // x = c + R s: c_bar += x_bar, R_bar += x_bar s^T
  *cb += xk + xm;
  const double xs[3][2] = {{xk.x, xm.x}, {xk.y, xm.y}, {xk.z, xm.z}};
  const double ss[3][2] = {{sk.x, sm.x}, {sk.y, sm.y}, {sk.z, sm.z}};
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) Rb[3 * i + j] += xs[i][0] * ss[j][0] + xs[i][1] * ss[j][1];
}

// ------------------------------------------------------------ box-box
struct BoxChoice {
  int edge;  // -1: face axis `face` (0-2 of box A, 3-5 of box B); else edge axis 3 i + j
  int face;
};
constexpr int kBoxBoxMax = 8;

// Separating-axis test over the 15 axes: the overlap of the projections on a
// unit axis L is o(L) = sum a_i |L.u_i| + sum b_j |L.w_j| - |L.(cB - cA)|
// (u, w the box axes, a, b the half sizes); the contact axis is the face axis
// of least overlap unless the least edge overlap (axes u_i x w_j shorter
// than 1e-6 skipped) is smaller by more than 5% of its magnitude plus 1e-6.
// Returns false if the boxes are apart by at least `margin` along some axis.
// Evaluated in the boxes' frames: with C_ij = u_i.w_j, dA = (u_i.d),
// dB = (w_j.d), a face axis u_i has o = a_i + sum_j b_j |C_ij| - |dA_i|; the
// edge axis u_i x w_j has length s = sqrt(1 - C_ij^2) and
// s o = a_(i+1) |C_(i+2)j| + a_(i+2) |C_(i+1)j| + b_(j+1) |C_i(j+2)|
//       + b_(j+2) |C_i(j+1)| - |dA_(i+2) C_(i+1)j - dA_(i+1) C_(i+2)j|.
DMX_DEV bool box_box_choose(const double* ha, const double* hb, V3 cA, const M3& RA, V3 cB, const M3& RB,
                            double margin, BoxChoice* ch) {
  double C[3][3], dA[3], dB[3];
  const V3 d = cB - cA;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const V3 u = colv(RA.a, i), w = colv(RB.a, i);
    dA[i] = dot(u, d);
    dB[i] = dot(w, d);
#pragma unroll
    for (int j = 0; j < 3; ++j) C[i][j] = dot(u, colv(RB.a, j));
  }
  int face = 0, edge = -1;
  double of = 1e300, oe = 1e300;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double o = ha[i] + hb[0] * fabs(C[i][0]) + hb[1] * fabs(C[i][1]) + hb[2] * fabs(C[i][2]) - fabs(dA[i]);
    if (o < of) { of = o; face = i; }
  }
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const double o = hb[j] + ha[0] * fabs(C[0][j]) + ha[1] * fabs(C[1][j]) + ha[2] * fabs(C[2][j]) - fabs(dB[j]);
    if (o < of) { of = o; face = 3 + j; }
  }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const double s2 = 1.0 - C[i][j] * C[i][j];
      if (!(s2 >= 1e-12)) continue;
      const int i1 = (i + 1) % 3, i2 = (i + 2) % 3, j1 = (j + 1) % 3, j2 = (j + 2) % 3;
      const double so = ha[i1] * fabs(C[i2][j]) + ha[i2] * fabs(C[i1][j]) + hb[j1] * fabs(C[i][j2]) +
                        hb[j2] * fabs(C[i][j1]) - fabs(dA[i2] * C[i1][j] - dA[i1] * C[i2][j]);
      const double o = so * rsqrt_nr(s2);
      if (o < oe) { oe = o; edge = 3 * i + j; }
    }
  const bool use_edge = edge >= 0 && oe < of - (0.05 * fabs(of) + 1e-6);
  ch->edge = use_edge ? edge : -1;
  ch->face = face;
  return fmin(of, oe) > -margin;
}

// The face case's frame: reference box (the axis owner) and incident box,
// the reference normal's sign (toward the incident box) and the incident
// face (the incident axis most anti-parallel to the reference normal).
struct FaceFrame {
  bool refA;
  int face, ax, fj, j1, j2, k1, k2;
  double ns, sg;  // nR = ns u_R[ax]; incident face centre c_I + sg h_I[fj] u_I[fj]
};
DMX_DEV void face_frame_finish(FaceFrame& f) {
  f.j1 = (f.fj + 1) % 3; f.j2 = (f.fj + 2) % 3;
  f.k1 = (f.ax + 1) % 3; f.k2 = (f.ax + 2) % 3;
}
DMX_DEV FaceFrame face_frame(int face, V3 cA, const M3& RA, V3 cB, const M3& RB) {
  FaceFrame f;
  f.face = face;
  f.refA = face < 3;
  f.ax = face % 3;
  const double* RR = f.refA ? RA.a : RB.a;
  const double* RI = f.refA ? RB.a : RA.a;
  const V3 cR = f.refA ? cA : cB, cI = f.refA ? cB : cA;
  const V3 u = colv(RR, f.ax);
  f.ns = dot(u, cI - cR) < 0.0 ? -1.0 : 1.0;
  const V3 nR = f.ns * u;
  f.fj = 0;
  double best = -1.0;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const double a = fabs(dot(nR, colv(RI, j)));
    if (a > best) { best = a; f.fj = j; }
  }
  f.sg = dot(nR, colv(RI, f.fj)) > 0.0 ? -1.0 : 1.0;
  face_frame_finish(f);
  return f;
}
DMX_DEV int face_code(const FaceFrame& f) {
  return (f.face << 10) | (f.ns < 0.0 ? 1 << 15 : 0) | (f.fj << 16) | (f.sg < 0.0 ? 1 << 18 : 0);
}
DMX_DEV FaceFrame face_frame_of(int code) {
  FaceFrame f;
  f.face = rc_axis(code);
  f.refA = f.face < 3;
  f.ax = f.face % 3;
  f.ns = rc_bit(code, 15) ? -1.0 : 1.0;
  f.fj = (code >> 16) & 3;
  f.sg = rc_bit(code, 18) ? -1.0 : 1.0;
  face_frame_finish(f);
  return f;
}

constexpr double kS1[4] = {1.0, -1.0, -1.0, 1.0}, kS2[4] = {1.0, 1.0, -1.0, -1.0};

// The face case's construction, shared by the contacts and their reverse:
// reference box (R, c, h), incident box, the reference normal nR, the
// incident face's centre fc and in-face axes, the reference face's point pf
// and side axes.
struct FaceGeo {
  const double *RR, *RI, *hR, *hI;
  V3 cR, cI, nR, uI1, uI2, uR1, uR2, fc, pf;
};
DMX_DEV FaceGeo face_geo(const FaceFrame& f, const double* ha, const double* hb, V3 cA, const M3& RA, V3 cB,
                         const M3& RB) {
  FaceGeo g;
  g.RR = f.refA ? RA.a : RB.a;
  g.RI = f.refA ? RB.a : RA.a;
  g.hR = f.refA ? ha : hb;
  g.hI = f.refA ? hb : ha;
  g.cR = f.refA ? cA : cB;
  g.cI = f.refA ? cB : cA;
  g.nR = f.ns * colv(g.RR, f.ax);
  g.uI1 = colv(g.RI, f.j1); g.uI2 = colv(g.RI, f.j2);
  g.uR1 = colv(g.RR, f.k1); g.uR2 = colv(g.RR, f.k2);
  g.fc = g.cI + (f.sg * g.hI[f.fj]) * colv(g.RI, f.fj);
  g.pf = g.cR + g.hR[f.ax] * g.nR;
  return g;
}
DMX_DEV V3 face_corner(const FaceFrame& f, const FaceGeo& g, int c) {
  return g.fc + (kS1[c] * g.hI[f.j1]) * g.uI1 + (kS2[c] * g.hI[f.j2]) * g.uI2;
}

// Contacts of a box-box pair for a given choice: up to 8 (the clipped
// incident face) or 1 (crossing edges) with r below the margin, and their
// common normal from A toward B (outputs may be null: count only).  The clipped face's vertices are enumerated: (a) incident corners
// inside the reference face's prism |u_k1.(p - cR)| <= h_k1,
// |u_k2.(p - cR)| <= h_k2, (b) crossings of incident edges with the prism's
// side planes inside the other slab, (c) points of the incident face on the
// prism's corner lines strictly inside the face.  Each point P is projected
// halfway to the reference face: r = nR.(P - pf), p = P - (r / 2) nR.
// Crossing edges: the closest points PA, PB of the two supporting edge lines
// give r = n.(PB - PA) at their midpoint.
DMX_DEV int box_box_contacts(const double* ha, const double* hb, V3 cA, const M3& RA, V3 cB, const M3& RB,
                             double margin, const BoxChoice& ch, double* r_out, V3* p_out, V3* n_out, int* code) {
  // (r_out, p_out, n_out are all given or all null)
  if (ch.edge < 0) {
    const FaceFrame f = face_frame(ch.face, cA, RA, cB, RB);
    const FaceGeo g = face_geo(f, ha, hb, cA, RA, cB, RB);
    if (n_out) *n_out = f.refA ? g.nR : (-1.0) * g.nR;
    const int base = face_code(f);
    int cnt = 0;
    auto emit = [&](V3 P, int cc) {
      const double r = dot(g.nR, P - g.pf);
      if (r >= margin || cnt >= kBoxBoxMax) return;
      if (r_out) {
        r_out[cnt] = r;
        p_out[cnt] = P - (0.5 * r) * g.nR;
      }
      if (code) code[cnt] = base | cc;
      ++cnt;
    };
    V3 C[4];
    double g1[4], g2[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      C[c] = face_corner(f, g, c);
      g1[c] = dot(g.uR1, C[c] - g.cR);
      g2[c] = dot(g.uR2, C[c] - g.cR);
    }
    const double hk1 = g.hR[f.k1], hk2 = g.hR[f.k2];
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (fabs(g1[c]) <= hk1 && fabs(g2[c]) <= hk2) emit(C[c], kRcCorner | (c << 3));
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int d = (c + 1) & 3;
#pragma unroll
      for (int pl = 0; pl < 4; ++pl) {
        const bool first = pl < 2;
        const double lim = ((pl & 1) ? -1.0 : 1.0) * (first ? hk1 : hk2);
        const double ga = first ? g1[c] : g2[c], gb = first ? g1[d] : g2[d];
        const double dv = gb - ga;
        if (dv == 0.0) continue;
        const double t = (lim - ga) / dv;
        if (!(t > 0.0 && t < 1.0)) continue;
        const double go = first ? g2[c] + (g2[d] - g2[c]) * t : g1[c] + (g1[d] - g1[c]) * t;
        if (fabs(go) <= (first ? hk2 : hk1)) emit(C[c] + t * (C[d] - C[c]), kRcCross | (c << 3) | (pl << 6));
      }
    }
    const double m11 = dot(g.uR1, g.uI1), m12 = dot(g.uR1, g.uI2), m21 = dot(g.uR2, g.uI1), m22 = dot(g.uR2, g.uI2);
    const double o1 = dot(g.uR1, g.fc - g.cR), o2 = dot(g.uR2, g.fc - g.cR);
    const double det = m11 * m22 - m12 * m21;
    if (det != 0.0) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const double b1 = kS1[c] * hk1 - o1, b2 = kS2[c] * hk2 - o2;
        const double a = (b1 * m22 - b2 * m12) / det, b = (m11 * b2 - m21 * b1) / det;
        if (fabs(a) < g.hI[f.j1] && fabs(b) < g.hI[f.j2]) emit(g.fc + a * g.uI1 + b * g.uI2, kRcLine | (c << 3));
      }
    }
    return cnt;
  }
  const int i = ch.edge / 3, j = ch.edge % 3;
  const V3 ui = colv(RA.a, i), uj = colv(RB.a, j);
  V3 n = cross(ui, uj);
  n = (1.0 / sqrt(dot(n, n))) * n;
  const bool flip = dot(n, cB - cA) < 0.0;
  if (flip) n = (-1.0) * n;
  int signs = 0;
  V3 pA = cA, pB = cB;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const bool na = dot(n, colv(RA.a, k)) < 0.0, nb = dot(n, colv(RB.a, k)) >= 0.0;
    signs |= (na ? 1 << k : 0) | (nb ? 1 << (3 + k) : 0);
    if (k != i) pA += ((na ? -1.0 : 1.0) * ha[k]) * colv(RA.a, k);
    if (k != j) pB += ((nb ? -1.0 : 1.0) * hb[k]) * colv(RB.a, k);
  }
  const V3 w = pA - pB;
  const double b = dot(ui, uj), dd = dot(ui, w), e = dot(uj, w);
  const double den = 1.0 - b * b;
  const double sA = (b * e - dd) / den, tB = (e - b * dd) / den;
  const V3 PA = pA + sA * ui, PB = pB + tB * uj;
  const double r = dot(n, PB - PA);
  if (r >= margin) return 0;
  if (r_out) {
    r_out[0] = r;
    p_out[0] = 0.5 * (PA + PB);
    *n_out = n;
  }
  if (code) code[0] = kRcEdges | (i << 3) | (j << 6) | (ch.edge << 10) | (1 << 14) | (flip ? 1 << 15 : 0) | (signs << 16);
  return 1;
}

// Cotangents of the two box poses (c_bar, R_bar of A and B, accumulated) from
// those of one contact (r_bar, p_bar, n_bar), along the construction its code
// names.
DMX_DEV void box_box_vjp(const double* ha, const double* hb, V3 cA, const M3& RA, V3 cB, const M3& RB, int code,
                         double rb, V3 pb, V3 nb, V3* cAb, double* RAb, V3* cBb, double* RBb) {
  if (!rc_bit(code, 14)) {
    const FaceFrame f = face_frame_of(code);
    const FaceGeo g = face_geo(f, ha, hb, cA, RA, cB, RB);
    double* RRb = f.refA ? RAb : RBb;
    double* RIb = f.refA ? RBb : RAb;
    const int kind = rc_kind(code), c = rc_i(code);
    const double hk1 = g.hR[f.k1], hk2 = g.hR[f.k2];
    // the clipped point P
    V3 P;
    double t = 0.0, la = 0.0, lb = 0.0;
    double m11 = 0.0, m12 = 0.0, m21 = 0.0, m22 = 0.0, det = 1.0;
    if (kind == kRcCorner) {
      P = face_corner(f, g, c);
    } else if (kind == kRcCross) {
      const int d = (c + 1) & 3, pl = rc_j(code);
      const bool first = pl < 2;
      const V3 uk = first ? g.uR1 : g.uR2;
      const double lim = ((pl & 1) ? -1.0 : 1.0) * (first ? hk1 : hk2);
      const V3 Cc = face_corner(f, g, c), Cd = face_corner(f, g, d);
      const double gc = dot(uk, Cc - g.cR), gd = dot(uk, Cd - g.cR);
      t = (lim - gc) / (gd - gc);
      P = Cc + t * (Cd - Cc);
    } else {
      m11 = dot(g.uR1, g.uI1); m12 = dot(g.uR1, g.uI2); m21 = dot(g.uR2, g.uI1); m22 = dot(g.uR2, g.uI2);
      const double o1 = dot(g.uR1, g.fc - g.cR), o2 = dot(g.uR2, g.fc - g.cR);
      det = m11 * m22 - m12 * m21;
      const double b1 = kS1[c] * hk1 - o1, b2 = kS2[c] * hk2 - o2;
      la = (b1 * m22 - b2 * m12) / det;
      lb = (m11 * b2 - m21 * b1) / det;
      P = g.fc + la * g.uI1 + lb * g.uI2;
    }
    const double r = dot(g.nR, P - g.pf);
    // p = P - (r/2) nR, r = nR.(P - pf), n = +-nR
    const double rt = rb - 0.5 * dot(g.nR, pb);
    V3 nRb = (-0.5 * r) * pb + (f.refA ? nb : (-1.0) * nb) + rt * (P - g.pf);
    const V3 Pb = pb + rt * g.nR;
    V3 cRb = (-rt) * g.nR;  // pf = cR + h_R[ax] nR
    nRb += (-rt * g.hR[f.ax]) * g.nR;
    V3 cIb = mk3(0.0, 0.0, 0.0), fcb = mk3(0.0, 0.0, 0.0);
    V3 uR1b = mk3(0.0, 0.0, 0.0), uR2b = mk3(0.0, 0.0, 0.0), uI1b = mk3(0.0, 0.0, 0.0), uI2b = mk3(0.0, 0.0, 0.0);
    auto corner_b = [&](int cc, V3 Cb) {
      fcb += Cb;
      uI1b += (kS1[cc] * g.hI[f.j1]) * Cb;
      uI2b += (kS2[cc] * g.hI[f.j2]) * Cb;
    };
    if (kind == kRcCorner) {
      corner_b(c, Pb);
    } else if (kind == kRcCross) {
      // P = Cc + t (Cd - Cc), t = (lim - gc) / (gd - gc), g = u_k.(C - cR)
      const int d = (c + 1) & 3;
      const bool first = rc_j(code) < 2;
      const V3 uk = first ? g.uR1 : g.uR2;
      const V3 Cc = face_corner(f, g, c), Cd = face_corner(f, g, d);
      const double gc = dot(uk, Cc - g.cR), gd = dot(uk, Cd - g.cR);
      const double D = gd - gc;
      const double tb = dot(Pb, Cd - Cc);
      const double gcb = tb * (t - 1.0) / D, gdb = -tb * t / D;
      const V3 ukb = gcb * (Cc - g.cR) + gdb * (Cd - g.cR);
      if (first) uR1b += ukb; else uR2b += ukb;
      corner_b(c, (1.0 - t) * Pb + gcb * uk);
      corner_b(d, t * Pb + gdb * uk);
      cRb -= (gcb + gdb) * uk;
    } else {
      // P = fc + a u_I1 + b u_I2 with M (a, b) = (s1 h_k1 - o1, s2 h_k2 - o2),
      // M_ij = u_Ri.u_Ij, o_i = u_Ri.(fc - cR)
      const double ab = dot(Pb, g.uI1), bb = dot(Pb, g.uI2);
      fcb += Pb;
      uI1b += la * Pb;
      uI2b += lb * Pb;
      const double y1 = (m22 * ab - m21 * bb) / det, y2 = (-m12 * ab + m11 * bb) / det;  // M^-T (ab, bb)
      // rhs_bar = y: o_bar = -y; M_bar = -y (a, b)^T
      uR1b += (-y1) * (g.fc - g.cR);
      uR2b += (-y2) * (g.fc - g.cR);
      fcb -= y1 * g.uR1 + y2 * g.uR2;
      cRb += y1 * g.uR1 + y2 * g.uR2;
      uR1b -= y1 * (la * g.uI1 + lb * g.uI2);
      uR2b -= y2 * (la * g.uI1 + lb * g.uI2);
      uI1b -= la * (y1 * g.uR1 + y2 * g.uR2);
      uI2b -= lb * (y1 * g.uR1 + y2 * g.uR2);
    }
    // fc = cI + sg h_I[fj] u_I[fj]
    cIb += fcb;
    col_add(RIb, f.fj, (f.sg * g.hI[f.fj]) * fcb);
    col_add(RIb, f.j1, uI1b);
    col_add(RIb, f.j2, uI2b);
    col_add(RRb, f.ax, f.ns * nRb);
    col_add(RRb, f.k1, uR1b);
    col_add(RRb, f.k2, uR2b);
    if (f.refA) { *cAb += cRb; *cBb += cIb; } else { *cBb += cRb; *cAb += cIb; }
    return;
  }
  const int i = rc_i(code), j = rc_j(code);
  const V3 ui = colv(RA.a, i), uj = colv(RB.a, j);
  const V3 cr = cross(ui, uj);
  const double cn = sqrt(dot(cr, cr));
  const double sn = rc_bit(code, 15) ? -1.0 : 1.0;
  const V3 n = (sn / cn) * cr;
  double sgA[3], sgB[3];
  V3 pA = cA, pB = cB;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    sgA[k] = rc_bit(code, 16 + k) ? -1.0 : 1.0;
    sgB[k] = rc_bit(code, 19 + k) ? -1.0 : 1.0;
    if (k != i) pA += (sgA[k] * ha[k]) * colv(RA.a, k);
    if (k != j) pB += (sgB[k] * hb[k]) * colv(RB.a, k);
  }
  const V3 w = pA - pB;
  const double b = dot(ui, uj), dd = dot(ui, w), e = dot(uj, w);
  const double den = 1.0 - b * b;
  const double sA = (b * e - dd) / den, tB = (e - b * dd) / den;
  const V3 PA = pA + sA * ui, PB = pB + tB * uj;
  // r = n.(PB - PA), p = (PA + PB)/2
  const V3 PAb = 0.5 * pb - rb * n, PBb = 0.5 * pb + rb * n;
  const V3 nbt = nb + rb * (PB - PA);
  const double sAb = dot(PAb, ui), tBb = dot(PBb, uj);
  V3 uib = sA * PAb, ujb = tB * PBb;
  // sA = (b e - dd) / den, tB = (e - b dd) / den, den = 1 - b^2
  const double bb = (sAb * (e + 2.0 * b * sA) + tBb * (-dd + 2.0 * b * tB)) / den;
  const double eb = (sAb * b + tBb) / den;
  const double ddb = -(sAb + tBb * b) / den;
  uib += bb * uj + ddb * w;
  ujb += bb * ui + eb * w;
  const V3 wb = ddb * ui + eb * uj;
  const V3 pAb = PAb + wb, pBb = PBb - wb;
  *cAb += pAb;
  *cBb += pBb;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (k != i) col_add(RAb, k, (sgA[k] * ha[k]) * pAb);
    if (k != j) col_add(RBb, k, (sgB[k] * hb[k]) * pBb);
  }
  // n = sn c / |c|, c = u_i x u_j
  const V3 cb = (sn / cn) * (nbt - dot(n, nbt) * n);
  uib += cross(uj, cb);
  ujb += cross(cb, ui);
  col_add(RAb, i, uib);
  col_add(RBb, j, ujb);
}

}  // namespace dmx
