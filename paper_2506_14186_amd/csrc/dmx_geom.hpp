// Contact geometry of box worlds, templated on the scalar type: `double` for
// values, `Dual1` (value + one tangent) for directional derivatives of the
// contact set with respect to a body pose, with every discrete choice (the
// separating axis, the faces, the clipping decisions, the top-four vertices)
// taken on values, so a derivative holds the combinatorics fixed.
//
//  - plane-box: the smoothed four-deepest-vertex detection of App. C.1;
//  - box-box: the separating-axis test over the 15 candidate axes with face
//    clipping (Sutherland-Hodgman) or one crossing-edge contact (primitive-
//    vs-primitive detection of Sec. 2.1).
#pragma once
#include "dmx_common.hpp"

namespace dmx {

// ------------------------------------------------------------ dual numbers
struct Dual1 { double v, d; };
DMX_DEV Dual1 mkd(double v, double d = 0.0) { Dual1 r; r.v = v; r.d = d; return r; }
DMX_DEV Dual1 operator+(Dual1 a, Dual1 b) { return mkd(a.v + b.v, a.d + b.d); }
DMX_DEV Dual1 operator-(Dual1 a, Dual1 b) { return mkd(a.v - b.v, a.d - b.d); }
DMX_DEV Dual1 operator-(Dual1 a) { return mkd(-a.v, -a.d); }
DMX_DEV Dual1 operator*(Dual1 a, Dual1 b) { return mkd(a.v * b.v, a.d * b.v + a.v * b.d); }
DMX_DEV Dual1 operator/(Dual1 a, Dual1 b) {
  const double q = a.v / b.v;
  return mkd(q, (a.d - q * b.d) / b.v);
}
DMX_DEV Dual1 operator+(Dual1 a, double b) { return mkd(a.v + b, a.d); }
DMX_DEV Dual1 operator+(double a, Dual1 b) { return mkd(a + b.v, b.d); }
DMX_DEV Dual1 operator-(Dual1 a, double b) { return mkd(a.v - b, a.d); }
DMX_DEV Dual1 operator-(double a, Dual1 b) { return mkd(a - b.v, -b.d); }
DMX_DEV Dual1 operator*(Dual1 a, double b) { return mkd(a.v * b, a.d * b); }
DMX_DEV Dual1 operator*(double a, Dual1 b) { return mkd(a * b.v, a * b.d); }
DMX_DEV Dual1 operator/(Dual1 a, double b) { return mkd(a.v / b, a.d / b); }
DMX_DEV Dual1& operator+=(Dual1& a, Dual1 b) { a = a + b; return a; }
DMX_DEV Dual1& operator-=(Dual1& a, Dual1 b) { a = a - b; return a; }

DMX_DEV double val(double x) { return x; }
DMX_DEV double val(Dual1 x) { return x.v; }
DMX_DEV double gsqrt(double x) { return sqrt(x); }
DMX_DEV Dual1 gsqrt(Dual1 x) { const double s = sqrt(x.v); return mkd(s, 0.5 * x.d / s); }
DMX_DEV double gabs(double x) { return fabs(x); }
DMX_DEV Dual1 gabs(Dual1 x) { return x.v < 0.0 ? -x : x; }
template <class T> DMX_DEV T lift(double x) { return T(x); }
template <> DMX_DEV Dual1 lift<Dual1>(double x) { return mkd(x); }

template <class T> struct TV { T x, y, z; };
template <class T> DMX_DEV TV<T> tv(T a, T b, T c) { TV<T> r; r.x = a; r.y = b; r.z = c; return r; }
template <class T> DMX_DEV TV<T> liftv(const double* p) { return tv<T>(lift<T>(p[0]), lift<T>(p[1]), lift<T>(p[2])); }
template <class T> DMX_DEV TV<T> operator+(TV<T> a, TV<T> b) { return tv<T>(a.x + b.x, a.y + b.y, a.z + b.z); }
template <class T> DMX_DEV TV<T> operator-(TV<T> a, TV<T> b) { return tv<T>(a.x - b.x, a.y - b.y, a.z - b.z); }
template <class T, class S> DMX_DEV TV<T> scl(TV<T> a, S s) { return tv<T>(a.x * s, a.y * s, a.z * s); }
template <class T> DMX_DEV T tdot(TV<T> a, TV<T> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <class T> DMX_DEV TV<T> tcross(TV<T> a, TV<T> b) {
  return tv<T>(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
// row-major 3x3; column j is the body axis j in the world
template <class T> struct TM { T a[9]; };
template <class T> DMX_DEV TV<T> tcol(const TM<T>& m, int j) { return tv<T>(m.a[j], m.a[3 + j], m.a[6 + j]); }
template <class T> DMX_DEV TV<T> tmul(const TM<T>& m, TV<T> v) {
  return tv<T>(m.a[0] * v.x + m.a[1] * v.y + m.a[2] * v.z, m.a[3] * v.x + m.a[4] * v.y + m.a[5] * v.z,
               m.a[6] * v.x + m.a[7] * v.y + m.a[8] * v.z);
}
template <class T> DMX_DEV TV<T> tmulT(const TM<T>& m, TV<T> v) {
  return tv<T>(m.a[0] * v.x + m.a[3] * v.y + m.a[6] * v.z, m.a[1] * v.x + m.a[4] * v.y + m.a[7] * v.z,
               m.a[2] * v.x + m.a[5] * v.y + m.a[8] * v.z);
}
template <class T> DMX_DEV double cval(const TV<T>& v, int i) { return val(i == 0 ? v.x : (i == 1 ? v.y : v.z)); }
template <class T> DMX_DEV T comp(const TV<T>& v, int i) { return i == 0 ? v.x : (i == 1 ? v.y : v.z); }

// Tangent frame of a unit normal: t1 = normalized (a - (a.n) n) with a = e_x
// unless |n_x| >= 0.5 (then e_y), t2 = n x t1.
template <class T>
DMX_DEV void make_frame_t(TV<T> n, TV<T>* t1, TV<T>* t2) {
  const bool ex = fabs(val(n.x)) < 0.5;
  const TV<T> a = ex ? tv<T>(lift<T>(1.0), lift<T>(0.0), lift<T>(0.0)) : tv<T>(lift<T>(0.0), lift<T>(1.0), lift<T>(0.0));
  const TV<T> t = a - scl(n, tdot(a, n));
  *t1 = scl(t, lift<T>(1.0) / gsqrt(tdot(t, t)));
  *t2 = tcross(n, *t1);
}

// ------------------------------------------------------------ plane-box
// Smoothed four-deepest-vertex detection (App. C.1).  Vertex k of the box
// (centre c, rotation R, half sizes h; coordinate signs from the bits of k:
// x bit 0, y bit 1, z bit 2) is x_k = c + R s_k and penetrates the plane
// (point p0, normal n) by e_k = -n.(x_k - p0).  With the skin 1 mm and
// tau = max(0, e_max - skin), the weight w_k = smoothstep((e_k - (tau - skin))
// / skin) (C^1 smoothstep t^2 (3 - 2t) on [0, 1]), the weighted depth
// z_k = w_k e_k, and the four largest z_k (ties to the lower vertex index)
// are the candidates, with r = -z_k at x_k + (z_k / 2) n.  Candidates with
// r >= margin are dropped (they make no rows).  Returns the count.
template <class T>
DMX_DEV T smoothstep_t(T u) {
  if (val(u) <= 0.0) return lift<T>(0.0);
  if (val(u) >= 1.0) return lift<T>(1.0);
  return u * u * (3.0 - 2.0 * u);
}

template <class T>
DMX_DEV int box_plane_t(const double* h, const double* p0, const double* pn, TV<T> c, const TM<T>& R, double margin,
                        T* r_out, TV<T>* p_out) {
  const double skin = 1e-3;
  const TV<T> n = liftv<T>(pn), q0 = liftv<T>(p0);
  TV<T> x[8];
  T e[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const TV<T> s = tv<T>(lift<T>((k & 1) ? h[0] : -h[0]), lift<T>((k & 2) ? h[1] : -h[1]),
                          lift<T>((k & 4) ? h[2] : -h[2]));
    x[k] = c + tmul(R, s);
    e[k] = lift<T>(0.0) - tdot(n, x[k] - q0);
  }
  int kmax = 0;
#pragma unroll
  for (int k = 1; k < 8; ++k) kmax = val(e[k]) > val(e[kmax]) ? k : kmax;
  T emax = e[0];
#pragma unroll
  for (int k = 1; k < 8; ++k) if (k == kmax) emax = e[k];
  const T tau = val(emax) > skin ? emax - skin : lift<T>(0.0);
  T z[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) z[k] = smoothstep_t<T>((e[k] - (tau - skin)) / skin) * e[k];
  int cnt = 0;
#pragma unroll
  for (int rank = 0; rank < 4; ++rank) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      int rk = 0;
#pragma unroll
      for (int j = 0; j < 8; ++j) rk += (val(z[j]) > val(z[k])) || (j < k && val(z[j]) == val(z[k]));
      if (rk == rank) {
        const T r = lift<T>(0.0) - z[k];
        if (val(r) < margin) {
          r_out[cnt] = r;
          p_out[cnt] = x[k] + scl(n, z[k] * 0.5);
          ++cnt;
        }
      }
    }
  }
  return cnt;
}

// ------------------------------------------------------------ box-box
// The discrete choices of a box-box pair, taken on values and reused by
// derivative passes.
struct BoxChoice {
  int edge;  // -1: face axis `face` (0-2 of box A, 3-5 of box B); else edge axis 3 i + j
  int face;
};

constexpr int kBoxBoxMax = 8;

// Separating-axis test over the 15 axes: the overlap of the projections on a
// unit axis L is o(L) = sum a_i |L.u_i| + sum b_j |L.w_j| - |L.(cB - cA)|
// (u, w the box axes, a, b the half sizes); the contact axis is the face axis
// of least overlap unless the least edge overlap (cross products shorter
// than 1e-6 skipped) is smaller by more than 5% of its magnitude plus 1e-6.
// Returns false if the boxes are apart by at least `margin` along some axis.
DMX_DEV bool box_box_choose(const double* ha, const double* hb, const TV<double>& cA, const TM<double>& RA,
                            const TV<double>& cB, const TM<double>& RB, double margin, BoxChoice* ch) {
  TV<double> uA[3], uB[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) { uA[i] = tcol(RA, i); uB[i] = tcol(RB, i); }
  const TV<double> d = cB - cA;
  auto overlap = [&](const TV<double>& L) {
    double pa = 0.0, pb = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) { pa += fabs(tdot(L, uA[i])) * ha[i]; pb += fabs(tdot(L, uB[i])) * hb[i]; }
    return pa + pb - fabs(tdot(L, d));
  };
  int face = 0, edge = -1;
  double of = 1e300, oe = 1e300;
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const double o = overlap(i < 3 ? uA[i] : uB[i - 3]);
    if (o < of) { of = o; face = i; }
  }
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const TV<double> c = tcross(uA[i], uB[j]);
      const double cn = sqrt(tdot(c, c));
      if (cn < 1e-6) continue;
      const double o = overlap(scl(c, 1.0 / cn));
      if (o < oe) { oe = o; edge = 3 * i + j; }
    }
  const bool use_edge = edge >= 0 && oe < of - (0.05 * fabs(of) + 1e-6);
  ch->edge = use_edge ? edge : -1;
  ch->face = face;
  return fmin(of, oe) > -margin;
}

// Contacts of a box-box pair for a given choice: up to 8 (face clipping) or 1
// (crossing edges) with r below the margin; normal from A toward B.
template <class T>
DMX_DEV int box_box_contacts(const double* ha, const double* hb, TV<T> cA, const TM<T>& RA, TV<T> cB,
                             const TM<T>& RB, double margin, const BoxChoice& ch, T* r_out, TV<T>* p_out,
                             TV<T>* n_out) {
  TV<T> uA[3], uB[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) { uA[i] = tcol(RA, i); uB[i] = tcol(RB, i); }
  const TV<T> d = cB - cA;
  if (ch.edge < 0) {
    const bool refA = ch.face < 3;
    const int ax = ch.face % 3;
    const TV<T>* uR = refA ? uA : uB;
    const TV<T>* uI = refA ? uB : uA;
    const double* hR = refA ? ha : hb;
    const double* hI = refA ? hb : ha;
    const TV<T> cR = refA ? cA : cB, cI = refA ? cB : cA;
    TV<T> nR = uR[ax];
    if (val(tdot(nR, cI - cR)) < 0.0) nR = scl(nR, -1.0);
    int fj = 0;
    double best = -1.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const double a = fabs(val(tdot(nR, uI[j])));
      if (a > best) { best = a; fj = j; }
    }
    const double sg = val(tdot(nR, uI[fj])) > 0.0 ? -1.0 : 1.0;
    const TV<T> fc = cI + scl(uI[fj], sg * hI[fj]);
    const int j1 = (fj + 1) % 3, j2 = (fj + 2) % 3;
    TV<T> poly[2][kBoxBoxMax + 1];
    int np = 4, cur = 0;
    {
      const double s1[4] = {1.0, -1.0, -1.0, 1.0}, s2[4] = {1.0, 1.0, -1.0, -1.0};
#pragma unroll
      for (int c = 0; c < 4; ++c) poly[0][c] = fc + scl(uI[j1], s1[c] * hI[j1]) + scl(uI[j2], s2[c] * hI[j2]);
    }
#pragma unroll
    for (int kk = 1; kk <= 2; ++kk) {
      const int k2 = (ax + kk) % 3;
#pragma unroll
      for (int sgn = 1; sgn >= -1; sgn -= 2) {
        int nn = 0;
        for (int i = 0; i < np; ++i) {
          const TV<T> P = poly[cur][i];
          const TV<T> Q = poly[cur][i + 1 < np ? i + 1 : 0];
          const T fP = tdot(uR[k2], P - cR) * (double)sgn - hR[k2];
          const T fQ = tdot(uR[k2], Q - cR) * (double)sgn - hR[k2];
          const bool inP = val(fP) <= 0.0, inQ = val(fQ) <= 0.0;
          if (inP && nn <= kBoxBoxMax) poly[1 - cur][nn++] = P;
          if (inP != inQ && nn <= kBoxBoxMax) poly[1 - cur][nn++] = P + scl(Q - P, fP / (fP - fQ));
        }
        np = nn;
        cur = 1 - cur;
      }
    }
    const TV<T> pf = cR + scl(nR, hR[ax]);
    int cnt = 0;
    for (int i = 0; i < np; ++i) {
      const TV<T> P = poly[cur][i];
      const T r = tdot(nR, P - pf);
      if (val(r) >= margin || cnt >= kBoxBoxMax) continue;
      r_out[cnt] = r;
      p_out[cnt] = P - scl(nR, r * 0.5);
      n_out[cnt] = refA ? nR : scl(nR, -1.0);
      ++cnt;
    }
    return cnt;
  }
  const int i = ch.edge / 3, j = ch.edge % 3;
  TV<T> n = tcross(uA[i], uB[j]);
  n = scl(n, lift<T>(1.0) / gsqrt(tdot(n, n)));
  if (val(tdot(n, d)) < 0.0) n = scl(n, -1.0);
  TV<T> pA = cA, pB = cB;
#pragma unroll
  for (int k2 = 0; k2 < 3; ++k2) {
    if (k2 != i) pA = pA + scl(uA[k2], (val(tdot(n, uA[k2])) >= 0.0 ? 1.0 : -1.0) * ha[k2]);
    if (k2 != j) pB = pB + scl(uB[k2], (val(tdot(n, uB[k2])) >= 0.0 ? -1.0 : 1.0) * hb[k2]);
  }
  const TV<T> w = pA - pB;
  const T b = tdot(uA[i], uB[j]), dd = tdot(uA[i], w), e = tdot(uB[j], w);
  const T den = lift<T>(1.0) - b * b;
  const T sA = (b * e - dd) / den, tB = (e - b * dd) / den;
  const TV<T> PA = pA + scl(uA[i], sA), PB = pB + scl(uB[j], tB);
  const T r = tdot(n, PB - PA);
  if (val(r) >= margin) return 0;
  r_out[0] = r;
  p_out[0] = scl(PA + PB, 0.5);
  n_out[0] = n;
  return 1;
}

}  // namespace dmx
