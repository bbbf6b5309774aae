// Device helpers: 3-vectors, quaternions, team (lanes-of-one-world) reductions.
//
// A "team" is L consecutive lanes of a 64-wide wavefront that cooperate on one
// world (L divides 64).  Replicated per-world values must stay bitwise equal
// across the team, so every team reduction is a butterfly of pairwise sums
// a + b / b + a (commutative, hence identical on both lanes of a pair).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define DMX_DEV __device__ __forceinline__

namespace dmx {

// model parameters whose cotangents the free-body reverse sweeps accumulate:
// the box geom's half sizes (3), then the friction coefficient, the solref
// time constant and the damping ratio shared by the contact pairs, the body's
// mass, then the five solimp parameters shared by the pairs
constexpr int kParams = 12;

struct V3 { double x, y, z; };
DMX_DEV V3 mk3(double a, double b, double c) { V3 r; r.x = a; r.y = b; r.z = c; return r; }
DMX_DEV V3 operator+(V3 a, V3 b) { return mk3(a.x + b.x, a.y + b.y, a.z + b.z); }
DMX_DEV V3 operator-(V3 a, V3 b) { return mk3(a.x - b.x, a.y - b.y, a.z - b.z); }
DMX_DEV V3 operator*(double s, V3 a) { return mk3(s * a.x, s * a.y, s * a.z); }
DMX_DEV V3& operator+=(V3& a, V3 b) { a.x += b.x; a.y += b.y; a.z += b.z; return a; }
DMX_DEV V3& operator-=(V3& a, V3 b) { a.x -= b.x; a.y -= b.y; a.z -= b.z; return a; }
DMX_DEV double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
DMX_DEV V3 cross(V3 a, V3 b) { return mk3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x); }
DMX_DEV V3 ld3(const double* p) { return mk3(p[0], p[1], p[2]); }

// row-major 3x3
struct M3 { double a[9]; };
DMX_DEV V3 mul(const M3& m, V3 v) {
  return mk3(m.a[0] * v.x + m.a[1] * v.y + m.a[2] * v.z, m.a[3] * v.x + m.a[4] * v.y + m.a[5] * v.z,
             m.a[6] * v.x + m.a[7] * v.y + m.a[8] * v.z);
}
DMX_DEV V3 mulT(const M3& m, V3 v) {
  return mk3(m.a[0] * v.x + m.a[3] * v.y + m.a[6] * v.z, m.a[1] * v.x + m.a[4] * v.y + m.a[7] * v.z,
             m.a[2] * v.x + m.a[5] * v.y + m.a[8] * v.z);
}
DMX_DEV void outer_add(M3& m, V3 a, V3 b) {  // m += a b^T
  m.a[0] += a.x * b.x; m.a[1] += a.x * b.y; m.a[2] += a.x * b.z;
  m.a[3] += a.y * b.x; m.a[4] += a.y * b.y; m.a[5] += a.y * b.z;
  m.a[6] += a.z * b.x; m.a[7] += a.z * b.y; m.a[8] += a.z * b.z;
}

struct Q4 { double w, x, y, z; };
DMX_DEV Q4 mkq(double w, double x, double y, double z) { Q4 q; q.w = w; q.x = x; q.y = y; q.z = z; return q; }
DMX_DEV Q4 qmul(Q4 a, Q4 b) {
  return mkq(a.w * b.w - a.x * b.x - a.y * b.y - a.z * b.z, a.w * b.x + a.x * b.w + a.y * b.z - a.z * b.y,
             a.w * b.y - a.x * b.z + a.y * b.w + a.z * b.x, a.w * b.z + a.x * b.y - a.y * b.x + a.z * b.w);
}
DMX_DEV Q4 qconj(Q4 a) { return mkq(a.w, -a.x, -a.y, -a.z); }
DMX_DEV double qdot(Q4 a, Q4 b) { return a.w * b.w + a.x * b.x + a.y * b.y + a.z * b.z; }
DMX_DEV Q4 qscale(double s, Q4 a) { return mkq(s * a.w, s * a.x, s * a.y, s * a.z); }
DMX_DEV Q4 qadd(Q4 a, Q4 b) { return mkq(a.w + b.w, a.x + b.x, a.y + b.y, a.z + b.z); }

// Rotation matrix (body -> world) of a unit quaternion.
DMX_DEV M3 quat2mat(Q4 q) {
  M3 m;
  double ww = q.w * q.w, xx = q.x * q.x, yy = q.y * q.y, zz = q.z * q.z;
  double wx = q.w * q.x, wy = q.w * q.y, wz = q.w * q.z, xy = q.x * q.y, xz = q.x * q.z, yz = q.y * q.z;
  m.a[0] = ww + xx - yy - zz; m.a[1] = 2.0 * (xy - wz); m.a[2] = 2.0 * (xz + wy);
  m.a[3] = 2.0 * (xy + wz); m.a[4] = ww - xx + yy - zz; m.a[5] = 2.0 * (yz - wx);
  m.a[6] = 2.0 * (xz - wy); m.a[7] = 2.0 * (yz + wx); m.a[8] = ww - xx - yy + zz;
  return m;
}
// Cotangent of the quaternion given the cotangent Rb of quat2mat(q).
DMX_DEV Q4 quat2mat_vjp(Q4 q, const M3& Rb) {
  const double* b = Rb.a;
  Q4 g;
  g.w = 2.0 * (q.w * (b[0] + b[4] + b[8]) + q.x * (b[7] - b[5]) + q.y * (b[2] - b[6]) + q.z * (b[3] - b[1]));
  g.x = 2.0 * (q.x * (b[0] - b[4] - b[8]) + q.w * (b[7] - b[5]) + q.y * (b[1] + b[3]) + q.z * (b[2] + b[6]));
  g.y = 2.0 * (q.y * (-b[0] + b[4] - b[8]) + q.w * (b[2] - b[6]) + q.x * (b[1] + b[3]) + q.z * (b[5] + b[7]));
  g.z = 2.0 * (q.z * (-b[0] - b[4] + b[8]) + q.w * (b[3] - b[1]) + q.x * (b[2] + b[6]) + q.y * (b[5] + b[7]));
  return g;
}
// 1/sqrt(x), x > 0: the hardware estimate refined by two Newton steps
// y <- y (3 - x y^2) / 2 (a few ulp; no square root and division sequence)
DMX_DEV double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * (1.5 - 0.5 * x * y * y);
  return y * (1.5 - 0.5 * x * y * y);
}

// 1/x, x != 0 finite: the hardware estimate refined by two Newton steps
// y <- y (2 - x y) (a few ulp)
DMX_DEV double rcp_nr(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = y * (2.0 - x * y);
  return y * (2.0 - x * y);
}

// y = x / |x| and its cotangent map
DMX_DEV Q4 qnormalize(Q4 x, double* inv_norm) {
  double s = rsqrt_nr(qdot(x, x));
  if (inv_norm) *inv_norm = s;
  return qscale(s, x);
}
DMX_DEV Q4 qnormalize_vjp(Q4 y, double inv_norm, Q4 yb) { return qscale(inv_norm, qadd(yb, qscale(-qdot(y, yb), y))); }

// exp of half a rotation vector th: (cos(|th|/2), sin(|th|/2)/|th| th).  For
// |th| < 1 (every step of the workloads here) both factors are power series
// in u = |th|^2/4, cos(phi/2) = sum (-u)^k/(2k)!, sin(phi/2)/phi = 1/2 sum
// (-u)^k/(2k+1)!, summed to k = 9 (the next term is below 1e-21): no square
// root, trigonometric call or division, and finite derivatives at zero.
DMX_DEV Q4 qexp_half(V3 th, double* cs, double* sn, double* dcs, double* dsn) {
  double t2 = dot(th, th);
  double c, s, dc, ds;  // c(t2), s(t2) and their derivatives with respect to t2
  if (t2 < 1.0) {
    // 1/(2k)! and 1/(2k+1)! for k = 0..9
    constexpr double ce[10] = {1.0, 1.0 / 2, 1.0 / 24, 1.0 / 720, 1.0 / 40320, 1.0 / 3628800, 1.0 / 479001600,
                               1.0 / 87178291200.0, 1.0 / 20922789888000.0, 1.0 / 6402373705728000.0};
    constexpr double se[10] = {1.0, 1.0 / 6, 1.0 / 120, 1.0 / 5040, 1.0 / 362880, 1.0 / 39916800,
                               1.0 / 6227020800.0, 1.0 / 1307674368000.0, 1.0 / 355687428096000.0,
                               1.0 / 121645100408832000.0};
    const double u = 0.25 * t2;
    double pc = ce[9], ps = se[9], qc = 9.0 * ce[9], qs = 9.0 * se[9];
#pragma unroll
    for (int k = 8; k >= 0; --k) {  // Horner; the alternating signs come from "- u *"
      pc = ce[k] - u * pc;
      ps = se[k] - u * ps;
      if (k >= 1) { qc = k * ce[k] - u * qc; qs = k * se[k] - u * qs; }
    }
    c = pc;
    s = 0.5 * ps;
    dc = -0.25 * qc;
    ds = -0.125 * qs;
  } else {
    double phi = sqrt(t2);
    double ch = cos(0.5 * phi), sh = sin(0.5 * phi);
    c = ch;
    s = sh / phi;
    // d/dt2 = (1 / (2 phi)) d/dphi
    dc = -0.5 * sh * 0.5 / phi;
    ds = (0.5 * ch / phi - sh / (phi * phi)) * 0.5 / phi;
  }
  if (cs) { *cs = c; *sn = s; *dcs = dc; *dsn = ds; }
  return mkq(c, s * th.x, s * th.y, s * th.z);
}

// ----------------------------------------------------------------- team ops
// Lane permutation within rows of 16 (quad_perm, row_half_mirror,
// row_mirror): every lane reads a valid lane, so no old value is needed.
template <int CTRL>
DMX_DEV double dpp_f64(double v) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  lo = __builtin_amdgcn_mov_dpp(lo, CTRL, 0xF, 0xF, true);
  hi = __builtin_amdgcn_mov_dpp(hi, CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}

// One butterfly level of N independent team sums: each value adds its
// partner lane's (levels: quad_perm [1,0,3,2] = lane ^ 1, quad_perm [2,3,0,1]
// = lane ^ 2, row_half_mirror = the other quad of 8, row_mirror = the other
// half of 16).  Sums are commutative pairwise, so every lane of the team ends
// with the bitwise-same value; running level by level lets the N butterflies
// interleave instead of running one after another.
template <int CTRL, int N>
DMX_DEV void butterfly_level(double* v) {
  double t[N];
#pragma unroll
  for (int i = 0; i < N; ++i) t[i] = dpp_f64<CTRL>(v[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += t[i];
}
// Team sums of N values (N <= 28) staged through LDS, for teams whose
// nonzero terms sit on the first LIVE lanes: those lanes write their N terms,
// lane j then adds value pair (2j, 2j+1) over the LIVE rows in a fixed tree
// order and writes the sum, and every lane reads all N sums back (the same
// words, so the results are bitwise equal across the team).  The lanes of a
// team are one wavefront's lanes and LDS instructions of a wavefront execute
// in order; the wavefront-scope fences keep the compiler from moving the
// accesses across the phases.
constexpr int kLdsSumMax = 28;
template <int L>
DMX_DEV double* lds_sum_area() {
  __shared__ __attribute__((aligned(16))) double s[64 / L][(L + 1) * kLdsSumMax];
  return s[(threadIdx.x & 63) / L];
}
DMX_DEV void wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
template <int L, int LIVE, int N>
DMX_DEV void team_sum_lds(double* v) {
  static_assert(N <= kLdsSumMax && LIVE <= L && (LIVE & (LIVE - 1)) == 0, "team_sum_lds sizes");
  constexpr int NP = (N + 1) / 2;  // value pairs
  double* area = lds_sum_area<L>();
  double* S = area + L * kLdsSumMax;  // sums
  const int tl = threadIdx.x & (L - 1);
  if (tl < LIVE) {
    double2* row = (double2*)(area + tl * kLdsSumMax);
#pragma unroll
    for (int k = 0; k < NP; ++k) row[k] = make_double2(v[2 * k], 2 * k + 1 < N ? v[2 * k + 1] : 0.0);
  }
  wave_fence();
#pragma unroll
  for (int k0 = 0; k0 < NP; k0 += L) {
    const int k = k0 + tl;
    if (k < NP) {
      double2 t[LIVE];
#pragma unroll
      for (int j = 0; j < LIVE; ++j) t[j] = ((const double2*)(area + j * kLdsSumMax))[k];
#pragma unroll
      for (int w = 1; w < LIVE; w *= 2)
#pragma unroll
        for (int j = 0; j < LIVE; j += 2 * w) { t[j].x += t[j + w].x; t[j].y += t[j + w].y; }
      ((double2*)S)[k] = t[0];
    }
  }
  wave_fence();
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    const double2 t = ((const double2*)S)[k];
    v[2 * k] = t.x;
    if (2 * k + 1 < N) v[2 * k + 1] = t.y;
  }
  wave_fence();
}
// Per-team LDS slots for values computed one component per lane and then
// read by the whole team (N doubles per team).
template <int L, int N>
DMX_DEV double* lds_dof_area() {
  __shared__ __attribute__((aligned(16))) double s[64 / L][N];
  return s[(threadIdx.x & 63) / L];
}
// v[d] of a register array at a lane-dependent index d, by selects: each
// element passes through an empty asm so that the chain is not folded back
// into an indexed load (which would move the array to scratch memory).
template <int N>
DMX_DEV double pick(const double* v, int d) {
  double r = v[0];
  asm("" : "+v"(r));
#pragma unroll
  for (int e = 1; e < N; ++e) {
    double ve = v[e];
    asm("" : "+v"(ve));
    r = (d == e) ? ve : r;
  }
  return r;
}

// Lanes of a team that hold contact slots when slot c sits on lane c mod L:
// the slot count rounded up to a power of two, at most the team.
constexpr int live_lanes(int nc, int L) {
  int p = 1;
  while (p < nc) p *= 2;
  return p < L ? p : L;
}

template <int L, int N>
DMX_DEV void team_sum_arr(double* v) {
  if constexpr (L >= 2) butterfly_level<0xB1, N>(v);
  if constexpr (L >= 4) butterfly_level<0x4E, N>(v);
  if constexpr (L >= 8) butterfly_level<0x141, N>(v);
  if constexpr (L >= 16) butterfly_level<0x140, N>(v);
  if constexpr (L >= 32) {
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] += __shfl_xor(v[i], 16, 64);
  }
  if constexpr (L >= 64) {
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] += __shfl_xor(v[i], 32, 64);
  }
}

// Team-wide boolean reductions through the wave ballot.
template <int L>
DMX_DEV uint64_t team_bits(bool p) {
  uint64_t b = __ballot(p);
  if constexpr (L == 64) return b;
  const int base = (threadIdx.x & 63) & ~(L - 1);
  return (b >> base) & ((L == 64) ? ~0ull : ((1ull << L) - 1ull));
}
template <int L> DMX_DEV bool team_any(bool p) { return team_bits<L>(p) != 0ull; }
template <int L> DMX_DEV bool team_all(bool p) {
  if constexpr (L == 64) return __ballot(!p) == 0ull;
  return team_bits<L>(p) == ((1ull << L) - 1ull);
}

// Dense symmetric positive definite Cholesky (lower, row-major N x N) and solve.
// The diagonal holds the reciprocals 1/L_jj (the solve multiplies by them).
template <int N>
DMX_DEV bool chol(double* A) {
  bool ok = true;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    double s = A[j * N + j];
#pragma unroll
    for (int k = 0; k < j; ++k) s -= A[j * N + k] * A[j * N + k];
    ok = ok && (s > 0.0);
    const double inv = rsqrt_nr(s > 0.0 ? s : 1e-300);
    A[j * N + j] = inv;
#pragma unroll
    for (int i = j + 1; i < N; ++i) {
      double t = A[i * N + j];
#pragma unroll
      for (int k = 0; k < j; ++k) t -= A[i * N + k] * A[j * N + k];
      A[i * N + j] = t * inv;
    }
  }
  return ok;
}
template <int N>
DMX_DEV void chol_solve(const double* Lm, double* x) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double s = x[i];
#pragma unroll
    for (int k = 0; k < i; ++k) s -= Lm[i * N + k] * x[k];
    x[i] = s * Lm[i * N + i];
  }
#pragma unroll
  for (int i = N - 1; i >= 0; --i) {
    double s = x[i];
#pragma unroll
    for (int k = i + 1; k < N; ++k) s -= Lm[k * N + i] * x[k];
    x[i] = s * Lm[i * N + i];
  }
}

// packed lower triangle index (i >= j)
DMX_DEV constexpr int tri(int i, int j) { return i * (i + 1) / 2 + j; }

// Cholesky of a symmetric positive definite matrix in packed lower-triangle
// storage P[tri(i, j)]; the diagonal receives the reciprocals 1/L_jj.
template <int N>
DMX_DEV bool chol_packed(double* P) {
  bool ok = true;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    double s = P[tri(j, j)];
#pragma unroll
    for (int k = 0; k < j; ++k) s -= P[tri(j, k)] * P[tri(j, k)];
    ok = ok && (s > 0.0);
    const double inv = rsqrt_nr(s > 0.0 ? s : 1e-300);
    P[tri(j, j)] = inv;
#pragma unroll
    for (int i = j + 1; i < N; ++i) {
      double t = P[tri(i, j)];
#pragma unroll
      for (int k = 0; k < j; ++k) t -= P[tri(i, k)] * P[tri(j, k)];
      P[tri(i, j)] = t * inv;
    }
  }
  return ok;
}
template <int N>
DMX_DEV void chol_solve_packed(const double* P, double* x) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double s = x[i];
#pragma unroll
    for (int k = 0; k < i; ++k) s -= P[tri(i, k)] * x[k];
    x[i] = s * P[tri(i, i)];
  }
#pragma unroll
  for (int i = N - 1; i >= 0; --i) {
    double s = x[i];
#pragma unroll
    for (int k = i + 1; k < N; ++k) s -= P[tri(k, i)] * x[k];
    x[i] = s * P[tri(i, i)];
  }
}

}  // namespace dmx
