// Oracle math: a forward-mode dual number and small vector/matrix helpers.
//
// TEST INFRASTRUCTURE ONLY.  The oracle is a plain, slow FP64 CPU simulator
// used to check the HIP path; nothing in the product links or calls it.
//
// Every simulation routine of the oracle is a template over the scalar type
// S.  With S = double it computes values; with S = Dual<N> it additionally
// carries N tangent directions, so the derivative of the discretized rollout
// (discretize-then-optimize, App. C.2) is obtained by differentiating exactly
// the same arithmetic in forward mode.
#pragma once
#include <cmath>
#include <cstring>

namespace orc {

template <int N>
struct Dual {
  double v;
  double d[N];
  Dual() : v(0.0) { for (int i = 0; i < N; ++i) d[i] = 0.0; }
  Dual(double x) : v(x) { for (int i = 0; i < N; ++i) d[i] = 0.0; }  // NOLINT: implicit constant lift
};

inline double val(double x) { return x; }
template <int N> inline double val(const Dual<N>& x) { return x.v; }

template <int N> inline Dual<N> operator+(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v + b.v; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i]; return r; }
template <int N> inline Dual<N> operator-(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v - b.v; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i]; return r; }
template <int N> inline Dual<N> operator-(const Dual<N>& a) {
  Dual<N> r; r.v = -a.v; for (int i = 0; i < N; ++i) r.d[i] = -a.d[i]; return r; }
template <int N> inline Dual<N> operator*(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v * b.v; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i]; return r; }
template <int N> inline Dual<N> operator/(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v / b.v;
  for (int i = 0; i < N; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) / b.v;
  return r; }
template <int N> inline Dual<N> operator+(const Dual<N>& a, double b) { Dual<N> r = a; r.v += b; return r; }
template <int N> inline Dual<N> operator+(double a, const Dual<N>& b) { Dual<N> r = b; r.v += a; return r; }
template <int N> inline Dual<N> operator-(const Dual<N>& a, double b) { Dual<N> r = a; r.v -= b; return r; }
template <int N> inline Dual<N> operator-(double a, const Dual<N>& b) { return Dual<N>(a) - b; }
template <int N> inline Dual<N> operator*(const Dual<N>& a, double b) {
  Dual<N> r; r.v = a.v * b; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b; return r; }
template <int N> inline Dual<N> operator*(double a, const Dual<N>& b) { return b * a; }
template <int N> inline Dual<N> operator/(const Dual<N>& a, double b) {
  Dual<N> r; r.v = a.v / b; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] / b; return r; }
template <int N> inline Dual<N> operator/(double a, const Dual<N>& b) { return Dual<N>(a) / b; }
template <int N> inline Dual<N>& operator+=(Dual<N>& a, const Dual<N>& b) { a = a + b; return a; }
template <int N> inline Dual<N>& operator-=(Dual<N>& a, const Dual<N>& b) { a = a - b; return a; }
template <int N> inline Dual<N>& operator*=(Dual<N>& a, const Dual<N>& b) { a = a * b; return a; }
template <int N> inline Dual<N>& operator/=(Dual<N>& a, const Dual<N>& b) { a = a / b; return a; }
template <int N> inline Dual<N>& operator+=(Dual<N>& a, double b) { a.v += b; return a; }
template <int N> inline Dual<N>& operator-=(Dual<N>& a, double b) { a.v -= b; return a; }
template <int N> inline Dual<N>& operator*=(Dual<N>& a, double b) { a = a * b; return a; }

// chain rule helper: f(a) with f'(a) = fp
template <int N> inline Dual<N> chain(const Dual<N>& a, double f, double fp) {
  Dual<N> r; r.v = f; for (int i = 0; i < N; ++i) r.d[i] = fp * a.d[i]; return r; }

inline double sqrt_(double x) { return std::sqrt(x); }
inline double sin_(double x) { return std::sin(x); }
inline double cos_(double x) { return std::cos(x); }
inline double exp_(double x) { return std::exp(x); }
inline double log1p_(double x) { return std::log1p(x); }
inline double pow_(double x, double p) { return std::pow(x, p); }
template <int N> inline Dual<N> sqrt_(const Dual<N>& a) { double s = std::sqrt(a.v); return chain(a, s, 0.5 / s); }
template <int N> inline Dual<N> sin_(const Dual<N>& a) { return chain(a, std::sin(a.v), std::cos(a.v)); }
template <int N> inline Dual<N> cos_(const Dual<N>& a) { return chain(a, std::cos(a.v), -std::sin(a.v)); }
template <int N> inline Dual<N> exp_(const Dual<N>& a) { double e = std::exp(a.v); return chain(a, e, e); }
template <int N> inline Dual<N> log1p_(const Dual<N>& a) { return chain(a, std::log1p(a.v), 1.0 / (1.0 + a.v)); }
// x^p for a constant exponent p >= 1 (x >= 0)
template <int N> inline Dual<N> pow_(const Dual<N>& a, double p) {
  double f = std::pow(a.v, p);
  double fp = (a.v == 0.0) ? (p == 1.0 ? 1.0 : 0.0) : p * std::pow(a.v, p - 1.0);
  return chain(a, f, fp); }

// ---------------------------------------------------------------- operation counter
// Flop: a double that tallies the floating-point operations made on it, by
// phase of the method, for the algorithmic operation counts of a rollout (a
// fused multiply-add counts as a multiply and an add; a division, a square
// root or an elementary function as one).  Operations with a structurally
// trivial operand are not counted: adding a structural zero, multiplying by a
// structural zero or by a constant +-1, dividing by a constant +-1.  A
// structural zero is a literal zero of the code (an accumulator's start, the
// zero blocks of J, M and H that the oracle's dense loops visit, a zero
// coefficient of the tableau) or a result computed only from such zeros;
// values that come from the inputs (Flop::data) are never trivial, whatever
// their value.  The dense loops then count what the same steps cost when they
// skip the zero blocks (the body-block structure a batched implementation
// exploits).  Comparisons and absolute values are not counted.
enum { kPhStep = 0, kPhRhs = 1, kPhNewton = 2, kPhLineSearch = 3, kPhOther = 4, kPhases = 5 };
struct FlopTally { long long n[kPhases]; };
inline FlopTally& flop_tally() { static thread_local FlopTally t{}; return t; }
inline int& flop_phase() { static thread_local int p = kPhOther; return p; }
inline void flop_count() { flop_tally().n[flop_phase()] += 1; }
// sets the phase for the lifetime of the object, then restores the previous one
struct FlopPhase {
  int prev;
  explicit FlopPhase(int p) : prev(flop_phase()) { flop_phase() = p; }
  ~FlopPhase() { flop_phase() = prev; }
};

struct Flop {
  double v;
  bool zero;  // structural zero
  bool unit;  // constant +-1
  Flop() : v(0.0), zero(true), unit(false) {}
  Flop(double x) : v(x), zero(x == 0.0), unit(x == 1.0 || x == -1.0) {}  // NOLINT: a constant of the code
  static Flop data(double x) { Flop f(x); f.zero = false; f.unit = false; return f; }
  static Flop result(double x, bool z) { Flop f(x); f.zero = z; f.unit = false; return f; }
};
inline double val(const Flop& x) { return x.v; }
inline Flop operator+(const Flop& a, const Flop& b) {
  if (a.zero) return b;
  if (b.zero) return a;
  flop_count();
  return Flop::result(a.v + b.v, false);
}
inline Flop operator-(const Flop& a) { Flop r = a; r.v = -a.v; return r; }
inline Flop operator-(const Flop& a, const Flop& b) {
  if (b.zero) return a;
  if (a.zero) return -b;
  flop_count();
  return Flop::result(a.v - b.v, false);
}
inline Flop operator*(const Flop& a, const Flop& b) {
  if (a.zero || b.zero) return Flop::result(a.v * b.v, true);
  if (a.unit) return a.v > 0.0 ? b : -b;
  if (b.unit) return b.v > 0.0 ? a : -a;
  flop_count();
  return Flop::result(a.v * b.v, false);
}
inline Flop operator/(const Flop& a, const Flop& b) {
  if (a.zero) return Flop::result(a.v / b.v, true);
  if (b.unit) return b.v > 0.0 ? a : -a;
  flop_count();
  return Flop::result(a.v / b.v, false);
}
inline Flop operator+(const Flop& a, double b) { return a + Flop(b); }
inline Flop operator+(double a, const Flop& b) { return Flop(a) + b; }
inline Flop operator-(const Flop& a, double b) { return a - Flop(b); }
inline Flop operator-(double a, const Flop& b) { return Flop(a) - b; }
inline Flop operator*(const Flop& a, double b) { return a * Flop(b); }
inline Flop operator*(double a, const Flop& b) { return Flop(a) * b; }
inline Flop operator/(const Flop& a, double b) { return a / Flop(b); }
inline Flop operator/(double a, const Flop& b) { return Flop(a) / b; }
inline Flop& operator+=(Flop& a, const Flop& b) { a = a + b; return a; }
inline Flop& operator-=(Flop& a, const Flop& b) { a = a - b; return a; }
inline Flop& operator*=(Flop& a, const Flop& b) { a = a * b; return a; }
inline Flop& operator/=(Flop& a, const Flop& b) { a = a / b; return a; }
inline Flop flop_fn(const Flop& a, double r) { if (a.zero) return Flop::result(r, r == 0.0); flop_count(); return Flop::result(r, false); }
inline Flop sqrt_(const Flop& a) { return flop_fn(a, std::sqrt(a.v)); }
inline Flop sin_(const Flop& a) { return flop_fn(a, std::sin(a.v)); }
inline Flop cos_(const Flop& a) { flop_count(); return Flop::result(std::cos(a.v), false); }
inline Flop exp_(const Flop& a) { flop_count(); return Flop::result(std::exp(a.v), false); }
inline Flop log1p_(const Flop& a) { return flop_fn(a, std::log1p(a.v)); }
inline Flop pow_(const Flop& a, double p) { return flop_fn(a, std::pow(a.v, p)); }

// value of a scalar in the value-only scalar T (double, or Flop keeping the
// counting scalar's structure), and a data value in T
inline double to_value(const double& x, const double*) { return x; }
template <int N> inline double to_value(const Dual<N>& x, const double*) { return x.v; }
inline Flop to_value(const Flop& x, const Flop*) { return x; }
inline Flop to_value(const double& x, const Flop*) { return Flop::data(x); }
template <class T, class S> inline T value_as(const S& x) { return to_value(x, (const T*)nullptr); }

// ---------------------------------------------------------------- 3-vectors
template <class S> struct V3 { S x[3]; };
template <class S> struct M3 { S a[3][3]; };  // a[row][col]
template <class S> struct Q4 { S w, x, y, z; };

template <class S> inline V3<S> v3(S a, S b, S c) { V3<S> r; r.x[0] = a; r.x[1] = b; r.x[2] = c; return r; }
template <class S> inline V3<S> vzero() { return v3<S>(S(0.0), S(0.0), S(0.0)); }
template <class S> inline V3<S> add(const V3<S>& a, const V3<S>& b) {
  return v3<S>(a.x[0] + b.x[0], a.x[1] + b.x[1], a.x[2] + b.x[2]); }
template <class S> inline V3<S> sub(const V3<S>& a, const V3<S>& b) {
  return v3<S>(a.x[0] - b.x[0], a.x[1] - b.x[1], a.x[2] - b.x[2]); }
template <class S, class T> inline V3<S> scale(const V3<S>& a, T s) {
  return v3<S>(a.x[0] * s, a.x[1] * s, a.x[2] * s); }
template <class S> inline S dot(const V3<S>& a, const V3<S>& b) {
  return a.x[0] * b.x[0] + a.x[1] * b.x[1] + a.x[2] * b.x[2]; }
template <class S> inline V3<S> cross(const V3<S>& a, const V3<S>& b) {
  return v3<S>(a.x[1] * b.x[2] - a.x[2] * b.x[1], a.x[2] * b.x[0] - a.x[0] * b.x[2],
               a.x[0] * b.x[1] - a.x[1] * b.x[0]); }
template <class S> inline V3<S> matvec(const M3<S>& m, const V3<S>& v) {
  V3<S> r;
  for (int i = 0; i < 3; ++i) r.x[i] = m.a[i][0] * v.x[0] + m.a[i][1] * v.x[1] + m.a[i][2] * v.x[2];
  return r; }
template <class S> inline V3<S> matTvec(const M3<S>& m, const V3<S>& v) {
  V3<S> r;
  for (int i = 0; i < 3; ++i) r.x[i] = m.a[0][i] * v.x[0] + m.a[1][i] * v.x[1] + m.a[2][i] * v.x[2];
  return r; }
template <class S> inline M3<S> matmul(const M3<S>& a, const M3<S>& b) {
  M3<S> r;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) r.a[i][j] = a.a[i][0] * b.a[0][j] + a.a[i][1] * b.a[1][j] + a.a[i][2] * b.a[2][j];
  return r; }
template <class S> inline M3<S> transpose(const M3<S>& a) {
  M3<S> r;
  for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) r.a[i][j] = a.a[j][i];
  return r; }
template <class S> inline M3<S> eye3() {
  M3<S> r;
  for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) r.a[i][j] = S(i == j ? 1.0 : 0.0);
  return r; }
template <class S> inline V3<S> col(const M3<S>& m, int j) { return v3<S>(m.a[0][j], m.a[1][j], m.a[2][j]); }

// Hamilton product, (w, x, y, z)
template <class S> inline Q4<S> qmul(const Q4<S>& a, const Q4<S>& b) {
  Q4<S> r;
  r.w = a.w * b.w - a.x * b.x - a.y * b.y - a.z * b.z;
  r.x = a.w * b.x + a.x * b.w + a.y * b.z - a.z * b.y;
  r.y = a.w * b.y - a.x * b.z + a.y * b.w + a.z * b.x;
  r.z = a.w * b.z + a.x * b.y - a.y * b.x + a.z * b.w;
  return r; }
template <class S> inline Q4<S> qnormalize(const Q4<S>& q) {
  S n = sqrt_(q.w * q.w + q.x * q.x + q.y * q.y + q.z * q.z);
  Q4<S> r; r.w = q.w / n; r.x = q.x / n; r.y = q.y / n; r.z = q.z / n; return r; }
// rotation matrix (body -> world) of a unit quaternion
template <class S> inline M3<S> qmat(const Q4<S>& q) {
  M3<S> m;
  S ww = q.w * q.w, xx = q.x * q.x, yy = q.y * q.y, zz = q.z * q.z;
  S wx = q.w * q.x, wy = q.w * q.y, wz = q.w * q.z, xy = q.x * q.y, xz = q.x * q.z, yz = q.y * q.z;
  m.a[0][0] = ww + xx - yy - zz; m.a[0][1] = 2.0 * (xy - wz); m.a[0][2] = 2.0 * (xz + wy);
  m.a[1][0] = 2.0 * (xy + wz); m.a[1][1] = ww - xx + yy - zz; m.a[1][2] = 2.0 * (yz - wx);
  m.a[2][0] = 2.0 * (xz - wy); m.a[2][1] = 2.0 * (yz + wx); m.a[2][2] = ww - xx - yy + zz;
  return m; }
// exp of a pure quaternion: the rotation by the rotation vector th (|th| = angle)
template <class S> inline Q4<S> qexp_rotvec(const V3<S>& th) {
  S t2 = dot(th, th);
  Q4<S> r;
  S c, s;  // cos(phi/2), sin(phi/2)/phi
  if (val(t2) < 1e-8) {  // |th| < 1e-4: Taylor series in phi^2 (keeps derivatives finite at 0)
    c = 1.0 - t2 / 8.0 + t2 * t2 / 384.0;
    s = 0.5 - t2 / 48.0 + t2 * t2 / 3840.0;
  } else {
    S phi = sqrt_(t2);
    c = cos_(phi * 0.5);
    s = sin_(phi * 0.5) / phi;
  }
  r.w = c; r.x = th.x[0] * s; r.y = th.x[1] * s; r.z = th.x[2] * s;
  return r; }
// rotation about a unit axis by angle th (axis constant)
template <class S> inline M3<S> axis_rot(const V3<double>& ax, const S& th) {
  S c = cos_(th), s = sin_(th);
  S t = 1.0 - c;
  double x = ax.x[0], y = ax.x[1], z = ax.x[2];
  M3<S> m;
  m.a[0][0] = t * (x * x) + c;     m.a[0][1] = t * (x * y) - s * z; m.a[0][2] = t * (x * z) + s * y;
  m.a[1][0] = t * (x * y) + s * z; m.a[1][1] = t * (y * y) + c;     m.a[1][2] = t * (y * z) - s * x;
  m.a[2][0] = t * (x * z) - s * y; m.a[2][1] = t * (y * z) + s * x; m.a[2][2] = t * (z * z) + c;
  return m; }

template <class S, class T> inline V3<S> lift(const V3<T>& a) { return v3<S>(S(a.x[0]), S(a.x[1]), S(a.x[2])); }
template <class S, class T> inline M3<S> liftm(const M3<T>& a) {
  M3<S> r; for (int i = 0; i < 3; ++i) for (int j = 0; j < 3; ++j) r.a[i][j] = S(a.a[i][j]); return r; }

}  // namespace orc
