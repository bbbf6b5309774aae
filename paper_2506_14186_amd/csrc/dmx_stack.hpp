// Cube-stack worlds: k <= 32 free cubes (box geoms) on a plane, one world per
// 64-lane wavefront.  The forward acceleration (Sec. 2: the equation of
// motion with the soft contact forces of the relaxed-Gauss primal problem,
// Sec. 2.1) and its integrator; the reverse sweep is in dmx_stack_adj.hpp.
//
// Lanes play two roles.  As dof lanes, lane 2b holds body b's position and
// world linear velocity (3 dofs), lane 2b + 1 its unit quaternion and
// body-frame angular velocity (3 dofs); the integrator's stage combinations
// are lane-local.  As pair lanes, lane l < 32 owns the plane pair of body l
// and lane 32 + i the box pair (i, i + 1) of neighbouring cubes: its contacts
// (at most 4 and 8), their rows and their share of the Newton gradient and
// Hessian.  Contacts between cubes that are not neighbours in the model's
// order stop the world (status bit 64): the Newton Hessian
// H = M + sum_e D_e J_e^T J_e is then block tridiagonal over the bodies, and
// its Cholesky factor has the same pattern (no fill).
#pragma once
#include <cstddef>

#include "dmx_free.hpp"
#include "dmx_geom.hpp"
#include "dmx_rk.hpp"

namespace dmx {

constexpr int kStackBodies = 32;
constexpr int kStackContacts = 256;  // contacts making rows, in pair order
// couplings created by odd-even reduction of a block-tridiagonal matrix of
// 32 blocks: sum over strides s = 1, 2, 4, 8, 16 of floor(31 / 2s)
constexpr int kStackCoupled = 26;
enum { kStOverflow = 16, kStGraph = 64 };

// Per-world model: identical cubes, one plane, identical pair parameters.
struct StackModel {
  int k, nu;
  int ctrl[6];  // dof of control i
  double h[3];  // half sizes
  double mass, imass, I[3], Iinv[3];  // principal inertia in the body frame
  double grav[3];
  double p0[3], pn[3];  // plane point and unit normal
  double mu, bcoef, kscale, ahat_plane, ahat_box;
  double si[5], cf[5], ssc[4], iwid[2];
  double rbound;  // bounding-sphere radius |h|
};

struct StackArgs {
  int W, n_int;
  int w0;                    // first world of a one-world-per-block launch without a queue
  double dt;
  const StackModel* models;  // [W]
  const long long* x_off;    // [W] first element of world w in x0 / xout / x0bar
  const long long* u_off;    // [W] first element of world w's controls in u / ubar
  const long long* t_off;    // [W] first double of world w's tape
  const int* cap_w;          // [W] tape records of world w
  const int* n_int_w;        // [W] intervals of world w (null: n_int)
  int stages;                // the tape holds the stage accelerations
  const double* x0;
  const double* u;
  double* xout;
  int* status;
  int* n_acc;
  int* n_rej;
  double* tape;
  const double* forced;
  const int* forced_n;
  int forced_cap;
  double* steplog;
  int* log_n;
  int log_cap;
  long long* counters;       // [W][kFwdCounters]
  const int* order;
  int* queue;
  SolverOpts o;
  // reverse sweep
  const double* xbar;
  double* x0bar;
  double* ubar;
  long long* adj_counters;   // [W][kAdjCounters]
  // uniform batches (every world of one model, dense layout): the tables
  // above are null and world w's offsets are w times these
  int uniform;
  int one_model;  // every world is models[0], offsets from the tables
  long long x_stride, u_stride, t_stride;
  int cap_uniform;
  // model-parameter cotangents [W][kParams] of the reverse sweep, or null
  double* pbar;
};

// per-world layout of a batch (tables, or the uniform strides)
DMX_DEV const StackModel& st_model(const StackArgs& a, int w) {
  return (a.uniform || a.one_model) ? a.models[0] : a.models[w];
}
DMX_DEV long long st_xoff(const StackArgs& a, int w) { return a.uniform ? w * a.x_stride : a.x_off[w]; }
DMX_DEV long long st_uoff(const StackArgs& a, int w) { return a.uniform ? w * a.u_stride : a.u_off[w]; }
DMX_DEV long long st_toff(const StackArgs& a, int w) { return a.uniform ? w * a.t_stride : a.t_off[w]; }
DMX_DEV long long st_cap(const StackArgs& a, int w) {
  return a.uniform ? a.cap_uniform : (a.cap_w ? a.cap_w[w] : 0);
}

struct StackLds {
  double R[kStackBodies][9];      // body rotations (body -> world)
  double P[kStackBodies][3];      // body origins
  double vec[3][kStackBodies][6]; // vectors over the bodies (world twists in the forward)
  double cp[3][kStackContacts], cr[kStackContacts];  // contacts: point, r (the normal is the pair's)
  double Hd[kStackBodies][21];    // diagonal blocks (packed lower), then their Cholesky factors
  double Ho[kStackBodies - 1][36];  // block (i + 1, i) (rows: body i + 1), then a reduction factor
  double Hn[kStackCoupled][36];   // couplings created by the reduction, then its factors
  double gv[kStackBodies][6];     // block right-hand side / solution
  int code[kStackContacts];       // contact codes (reverse sweep only)
};
enum { kVecX = 0, kVecV = 1, kVecD = 2 };

struct StackStat {
  int status, newton_it;
  long long u_att, u_rhs, u_con, u_nit, u_ncon, u_nedge, u_ls;
  long long u_con2, u_ncon2;  // contacts and Newton contacts of box pairs
  long long u_step, u_vjp, u_vcon, u_vedge;
};

struct StackRole {
  int lane, b, half;  // dof role: body b, half 0 (position, linear velocity) or 1 (quaternion, angular)
  bool dof;
  int pair;           // 0 none, 1 plane pair of body pb2, 2 box pair (pb1, pb2)
  int pb1, pb2;
};

DMX_DEV StackRole stack_role(const StackModel& m) {
  StackRole r;
  r.lane = threadIdx.x & 63;
  r.b = r.lane >> 1;
  r.half = r.lane & 1;
  r.dof = r.b < m.k;
  if (r.lane < 32) {
    r.pair = r.lane < m.k ? 1 : 0;
    r.pb1 = -1;
    r.pb2 = r.lane;
  } else {
    const int i = r.lane - 32;
    r.pair = i + 1 < m.k ? 2 : 0;
    r.pb1 = i;
    r.pb2 = i + 1;
  }
  return r;
}

// ------------------------------------------------------------ wave helpers
DMX_DEV int wave_excl_scan(int v, int* total) {
  const int lane = threadIdx.x & 63;
  int x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  *total = __shfl(x, 63, 64);
  return x - v;
}
template <int N>
DMX_DEV void wave_sum(double* v) { team_sum_arr<64, N>(v); }
DMX_DEV double wave_max(double v) {
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) v = fmax(v, __shfl_xor(v, m, 64));
  return v;
}
DMX_DEV bool wave_any(bool p) { return __ballot(p) != 0ull; }
DMX_DEV bool wave_all(bool p) { return __ballot(!p) == 0ull; }

// ------------------------------------------------------------ impedance
DMX_DEV double spow(double x, double e) {
  if (e == 1.0) return x;
  if (e == 2.0) return x * x;
  if (e == 0.0) return 1.0;
  if (e == 3.0) return x * x * x;
  return pow(x, e);
}
DMX_DEV double spline01(double x, double mid, double pw, double s_lo, double s_hi, double* dydx) {
  if (x >= 1.0) { *dydx = 0.0; return 1.0; }
  if (x <= 0.0) { *dydx = 0.0; return 0.0; }
  if (x <= mid) {
    const double xp = spow(x, pw - 1.0) * s_lo;
    *dydx = pw * xp;
    return xp * x;
  }
  const double z = 1.0 - x;
  const double zp = spow(z, pw - 1.0) * s_hi;
  *dydx = pw * zp;
  return 1.0 - zp * z;
}
// d(r) (Sec. 2.1: the solimp spline of the violation, r < 0) and its
// contacts-from-distance continuation for r >= 0 (Sec. 4), with dd/dr.
DMX_DEV double stack_imp(const StackModel& m, double r, double* ddr) {
  double dy;
  if (r < 0.0) {
    const double x = -r * m.iwid[0];
    const double y = spline01(x, m.si[3], m.si[4], m.ssc[0], m.ssc[1], &dy);
    *ddr = -dy * m.iwid[0] * (m.si[1] - m.si[0]);
    return m.si[0] + y * (m.si[1] - m.si[0]);
  }
  const double x = r * m.iwid[1];
  const double y = spline01(x, m.cf[3], m.cf[4], m.ssc[2], m.ssc[3], &dy);
  *ddr = dy * m.iwid[1] * (m.cf[0] - m.cf[1]);
  return m.cf[1] + y * (m.cf[0] - m.cf[1]);
}
// d(r) of the penetration spline (r < 0) in the solimp parameters (d0,
// dwidth, width, midpoint, power); zero for r >= 0 (the contacts-from-distance
// spline has its own parameters): d = d0 + y (dwidth - d0), x = -r / width,
// y = x^p / mid^(p-1) below the midpoint, 1 - (1-x)^p / (1-mid)^(p-1) above
DMX_DEV void stack_imp_solimp_grad(const StackModel& m, double r, double* g) {
#pragma unroll
  for (int i = 0; i < 5; ++i) g[i] = 0.0;
  if (r >= 0.0) return;
  const double x = -r * m.iwid[0], mid = m.si[3], pw = m.si[4], span = m.si[1] - m.si[0];
  double dy;
  const double y = spline01(x, mid, pw, m.ssc[0], m.ssc[1], &dy);
  g[0] = 1.0 - y;
  g[1] = y;
  if (x >= 1.0) return;
  g[2] = -span * dy * x * m.iwid[0];
  if (x <= mid) {
    g[3] = -span * (pw - 1.0) * y / mid;
    g[4] = span * y * log(x / mid);
  } else {
    g[3] = -span * (pw - 1.0) * (1.0 - y) / (1.0 - mid);
    g[4] = -span * (1.0 - y) * log((1.0 - x) / (1.0 - mid));
  }
}
DMX_DEV double stack_softplus(double z, double beta, double* dsp) {
  const double bz = beta * z;
  if (bz > 30.0) {
    const double e = exp(-bz);
    *dsp = 1.0 / (1.0 + e);
    return z + log1p(e) / beta;
  }
  const double e = exp(bz);
  *dsp = e / (1.0 + e);
  return log1p(e) / beta;
}

// ------------------------------------------------------------ contact rows
// A pair lane's contacts: its slots in the pool, their common normal (the
// plane's, or the box pair's contact axis from A toward B), active edges.
struct PairSlots {
  int off, cnt;     // this pair lane's contacts in the pool
  unsigned act;     // 4 bits per contact: active edges
  double ahat;
  V3 n;
};

// Row data of one contact: frame, lever arms from the two bodies' origins,
// impedance D, and the reference-acceleration parts a_n, a_t1, a_t2 with
// aref_e = a_n +- mu a_t (edges +t1, -t1, +t2, -t2).
struct CRow {
  V3 n, t1, t2, r1, r2;
  double r, D, an, at1, at2;
};

DMX_DEV V3 twist_at(const StackLds& S, int vec, int b, V3 rb) {
  const double* t = S.vec[vec][b];
  return mk3(t[0], t[1], t[2]) + cross(mk3(t[3], t[4], t[5]), rb);
}
// relative velocity (body 2 minus body 1) at the contact of a generalized
// vector published as body twists in S.vec[vec]
DMX_DEV V3 rel_vel(const StackLds& S, int vec, int b1, int b2, const CRow& c) {
  V3 u = twist_at(S, vec, b2, c.r2);
  if (b1 >= 0) u -= twist_at(S, vec, b1, c.r1);
  return u;
}

DMX_DEV void contact_row(const StackModel& m, const StackLds& S, const StackRole& ro, const PairSlots& ps, int j,
                         bool cfd, double beta, CRow& w) {
  const int c = ps.off + j, b1 = ro.pb1, b2 = ro.pb2;
  const double ahat = ps.ahat;
  const V3 p = mk3(S.cp[0][c], S.cp[1][c], S.cp[2][c]);
  w.n = ps.n;
  make_frame(w.n, &w.t1, &w.t2);
  w.r2 = p - ld3(S.P[b2]);
  w.r1 = b1 >= 0 ? p - ld3(S.P[b1]) : mk3(0, 0, 0);
  w.r = S.cr[c];
  double ddr;
  const double d = stack_imp(m, w.r, &ddr);
  w.D = d / (ahat * (1.0 - d));
  const double kk = d * m.kscale;
  double pterm;
  if (cfd) { double dsp; pterm = kk * stack_softplus(-w.r, beta, &dsp); }
  else pterm = -kk * w.r;
  const V3 uv = rel_vel(S, kVecV, b1, b2, w);
  w.an = -m.bcoef * dot(w.n, uv) + pterm;
  w.at1 = -m.bcoef * dot(w.t1, uv);
  w.at2 = -m.bcoef * dot(w.t2, uv);
}

// edge slacks s_e = J_e x - aref_e of a contact for the vector in S.vec[vec]
DMX_DEV void edge_slack(const StackLds& S, int vec, int b1, int b2, const CRow& w, double mu, double* s) {
  const V3 u = rel_vel(S, vec, b1, b2, w);
  const double jn = dot(w.n, u) - w.an, j1 = dot(w.t1, u) - w.at1, j2 = dot(w.t2, u) - w.at2;
  s[0] = jn + mu * j1; s[1] = jn - mu * j1; s[2] = jn + mu * j2; s[3] = jn - mu * j2;
}
// edge directions J_e w for a vector w (no aref)
DMX_DEV void edge_dir(const StackLds& S, int vec, int b1, int b2, const CRow& w, double mu, double* t) {
  const V3 u = rel_vel(S, vec, b1, b2, w);
  const double jn = dot(w.n, u), j1 = dot(w.t1, u), j2 = dot(w.t2, u);
  t[0] = jn + mu * j1; t[1] = jn - mu * j1; t[2] = jn + mu * j2; t[3] = jn - mu * j2;
}

DMX_DEV V3 edge_vec(const CRow& w, double mu, int e) {
  const V3 t = e < 2 ? w.t1 : w.t2;
  return (e & 1) ? w.n - mu * t : w.n + mu * t;
}

// Sums over a pair's contacts for the Hessian blocks and the gradient: with
// G = sum over active edges of D d_e d_e^T (world frame), K_b = [r_b]x G,
// Q_bb' = [r_b]x G [r_b']x, the force f = sum D s_e d_e and torques r_b x f.
struct PairSums {
  double G[6], K1[9], K2[9], Q11[6], Q22[6], Q12[9], f[3], m1[3], m2[3];
};
DMX_DEV void pair_sums_zero(PairSums& a) {
  double* p = a.G;
#pragma unroll
  for (int i = 0; i < 6 + 9 + 9 + 6 + 6 + 9 + 3 + 3 + 3; ++i) p[i] = 0.0;
}
// K = [r]x G for symmetric packed G (columns of G crossed with r)
DMX_DEV void cross_mat(V3 r, const double* G, double* K) {
  const V3 c0 = mk3(G[0], G[1], G[3]), c1 = mk3(G[1], G[2], G[4]), c2 = mk3(G[3], G[4], G[5]);
  const V3 k0 = cross(r, c0), k1 = cross(r, c1), k2 = cross(r, c2);
  K[0] = k0.x; K[3] = k0.y; K[6] = k0.z;
  K[1] = k1.x; K[4] = k1.y; K[7] = k1.z;
  K[2] = k2.x; K[5] = k2.y; K[8] = k2.z;
}
// Q = K [r]x : row i of Q is (row i of K) x r
DMX_DEV void mat_cross(const double* K, V3 r, double* Q) {
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const V3 q = cross(mk3(K[3 * i], K[3 * i + 1], K[3 * i + 2]), r);
    Q[3 * i] = q.x; Q[3 * i + 1] = q.y; Q[3 * i + 2] = q.z;
  }
}

DMX_DEV void pair_sums_add(PairSums& a, const CRow& w, double mu, unsigned act, const double* s, bool two) {
  double G[6] = {0, 0, 0, 0, 0, 0};
  V3 f = mk3(0, 0, 0);
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    if (!((act >> e) & 1u)) continue;
    const V3 d = edge_vec(w, mu, e);
    G[0] += w.D * d.x * d.x; G[1] += w.D * d.y * d.x; G[2] += w.D * d.y * d.y;
    G[3] += w.D * d.z * d.x; G[4] += w.D * d.z * d.y; G[5] += w.D * d.z * d.z;
    f += (w.D * s[e]) * d;
  }
#pragma unroll
  for (int i = 0; i < 6; ++i) a.G[i] += G[i];
  a.f[0] += f.x; a.f[1] += f.y; a.f[2] += f.z;
  double K2[9], Q[9];
  cross_mat(w.r2, G, K2);
#pragma unroll
  for (int i = 0; i < 9; ++i) a.K2[i] += K2[i];
  mat_cross(K2, w.r2, Q);
  a.Q22[0] += Q[0]; a.Q22[1] += Q[3]; a.Q22[2] += Q[4]; a.Q22[3] += Q[6]; a.Q22[4] += Q[7]; a.Q22[5] += Q[8];
  const V3 m2 = cross(w.r2, f);
  a.m2[0] += m2.x; a.m2[1] += m2.y; a.m2[2] += m2.z;
  if (two) {
    double K1[9];
    cross_mat(w.r1, G, K1);
#pragma unroll
    for (int i = 0; i < 9; ++i) a.K1[i] += K1[i];
    mat_cross(K1, w.r1, Q);
    a.Q11[0] += Q[0]; a.Q11[1] += Q[3]; a.Q11[2] += Q[4]; a.Q11[3] += Q[6]; a.Q11[4] += Q[7]; a.Q11[5] += Q[8];
    mat_cross(K1, w.r2, Q);
#pragma unroll
    for (int i = 0; i < 9; ++i) a.Q12[i] += Q[i];
    const V3 m1 = cross(w.r1, f);
    a.m1[0] += m1.x; a.m1[1] += m1.y; a.m1[2] += m1.z;
  }
}

// 3x3 helpers on row-major arrays
DMX_DEV void m3_RtA(const double* R, const double* A, double* out) {  // R^T A
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) out[3 * i + j] = R[i] * A[j] + R[3 + i] * A[3 + j] + R[6 + i] * A[6 + j];
}
DMX_DEV void m3_AR(const double* A, const double* R, double* out) {  // A R
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) out[3 * i + j] = A[3 * i] * R[j] + A[3 * i + 1] * R[3 + j] + A[3 * i + 2] * R[6 + j];
}
DMX_DEV void sym_unpack(const double* s, double* A) {
  A[0] = s[0]; A[1] = s[1]; A[2] = s[3];
  A[3] = s[1]; A[4] = s[2]; A[5] = s[4];
  A[6] = s[3]; A[7] = s[4]; A[8] = s[5];
}

// Diagonal block of body b from a pair's sums (sign +1 either way):
// [[G, K^T R], [R^T K, -R^T Q R]], added to the packed lower triangle.
DMX_DEV void add_diag_block(double* Hd, const double* G, const double* K, const double* Qs, const double* R) {
  double A[9], B[9], Q[9], T[9];
  m3_RtA(R, K, A);  // bottom-left R^T K
  sym_unpack(Qs, Q);
  m3_AR(Q, R, T);
  m3_RtA(R, T, B);  // R^T Q R
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) Hd[tri(i, j)] += G[tri(i, j)];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
#pragma unroll
    for (int j = 0; j < 3; ++j) Hd[tri(3 + i, j)] += A[3 * i + j];
#pragma unroll
    for (int j = 0; j <= i; ++j) Hd[tri(3 + i, 3 + j)] -= B[3 * i + j];
  }
}
// Gradient part of body b: sign * [f; R^T m]
DMX_DEV void add_grad(double* g, double sign, const double* f, const double* mo, const double* R) {
  g[0] += sign * f[0]; g[1] += sign * f[1]; g[2] += sign * f[2];
#pragma unroll
  for (int i = 0; i < 3; ++i) g[3 + i] += sign * (R[i] * mo[0] + R[3 + i] * mo[1] + R[6 + i] * mo[2]);
}

// ------------------------------------------------------------ block solve
// v <- L^-1 v and v <- L^-T v for a packed 6x6 Cholesky factor holding
// 1/L_jj on its diagonal
DMX_DEV void ltri_fwd(const double* L, double* v) {
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    double s = v[j];
#pragma unroll
    for (int m = 0; m < j; ++m) s -= L[tri(j, m)] * v[m];
    v[j] = s * L[tri(j, j)];
  }
}
DMX_DEV void ltri_bwd(const double* L, double* v) {
#pragma unroll
  for (int i = 5; i >= 0; --i) {
    double s = v[i];
#pragma unroll
    for (int m = i + 1; m < 6; ++m) s -= L[tri(m, i)] * v[m];
    v[i] = s * L[tri(i, i)];
  }
}

// Solve H x = g in place in S.gv for the block-tridiagonal SPD H (diagonal
// blocks in S.Hd, couplings in S.Ho) by odd-even block cyclic reduction,
// which is the block Cholesky factorization of H in nested-dissection order.
// At stride s = 1, 2, 4, ... the blocks still present are the multiples of
// s, at positions 0, 1, 2, ..; coupling j joins positions j and j + 1 (for
// s = 1 the blocks H(i + 1, i) in S.Ho, rows of block i + 1; for s > 1 the
// ones created at stride s / 2, stored in order in S.Hn).  The blocks at odd
// positions p are eliminated together: with L = chol(D_p),
// W_L = L^-1 H(p, p - 1), W_R = L^-1 H(p, p + 1) and w = L^-1 g_p, the
// neighbours take D_(p-1) -= W_L^T W_L, D_(p+1) -= W_R^T W_R,
// g_(p-1) -= W_L^T w, g_(p+1) -= W_R^T w, and couple through
// H(p + 1, p - 1) = -W_R^T W_L.  Block 0 remains: x_0 = L_0^-T L_0^-1 g_0;
// going back down the strides, x_p = L^-T (w - W_L x_(p-1) - W_R x_(p+1)).
// The depth is log2(k) block steps, each spread over the wavefront; the
// blocks are overwritten by the factors.  Returns false (on every lane) if
// a pivot is not positive.
DMX_DEV int bcr_positions(int k, int ls) { return ((k - 1) >> ls) + 1; }
// first coupling in S.Hn of stride 2^ls (ls >= 1): those created before
DMX_DEV int bcr_first(int k, int ls) {
  int b = 0;
  for (int l = 0; l + 1 < ls; ++l) b += (bcr_positions(k, l) - 1) / 2;
  return b;
}
// d = sum_r X[r sx] Y[r sy]
DMX_DEV double dot6s(const double* X, int sx, const double* Y, int sy) {
  double d = 0.0;
#pragma unroll
  for (int r = 0; r < 6; ++r) d += X[r * sx] * Y[r * sy];
  return d;
}
// entry q of a packed symmetric 6x6 block: row tp, column tc
DMX_DEV void tri_entry(int q, int* tp, int* tc) {
  const int p = q >= 15 ? 5 : q >= 10 ? 4 : q >= 6 ? 3 : q >= 3 ? 2 : q >= 1 ? 1 : 0;
  *tp = p;
  *tc = q - tri(p, 0);
}
DMX_DEV bool block_factor_solve(StackLds& S, int k) {
  const int lane = threadIdx.x & 63;
  // offsets below are in doubles from the start of the LDS block
  double* const base = reinterpret_cast<double*>(&S);
  constexpr int oHd = offsetof(StackLds, Hd) / 8, oHo = offsetof(StackLds, Ho) / 8, oHn = offsetof(StackLds, Hn) / 8,
                oGv = offsetof(StackLds, gv) / 8;
  // fixed lane roles of the triangular solves: eliminated block slot es
  // (4 per round) and column tc of [W_L | W_R | w]
  const int es = lane / 13, col = lane - 13 * es;
  // fixed lane roles of the update pass: entry q of a surviving block's
  // packed D (0..20) or g (21..26), or of a created coupling (27..62)
  const int q = lane;
  int tp, tc;
  tri_entry(q < 21 ? q : 0, &tp, &tc);
  const int pg = q - 21, pc = q - 27, pp = pc / 6, cc = pc - 6 * (pc / 6);
  bool ok = true;
  int ls = 0, made = 0;  // log2 stride; couplings created so far
  for (; (1 << ls) < k; ++ls) {
    const int np = bcr_positions(k, ls), ne = np / 2, nr = (np - 1) / 2;  // nr: eliminated with a right neighbour
    const int oC = ls == 0 ? oHo : oHn + 36 * bcr_first(k, ls);        // coupling j at oC + 36 j
    const int oN = oHn + 36 * made;                                     // created coupling e at oN + 36 e
    bool okl = true;
    if (lane < ne) {
      double* D = S.Hd[(2 * lane + 1) << ls];
      double P[21];
#pragma unroll
      for (int t = 0; t < 21; ++t) P[t] = D[t];
      okl = chol_packed<6>(P);
#pragma unroll
      for (int t = 0; t < 21; ++t) D[t] = P[t];
    }
    ok = wave_all(okl) && ok;
    wave_fence();
    // W_L = L^-1 H(p, p-1) (columns, in place), W_R = L^-1 H(p, p+1)
    // (stored transposed: rows, in place), w = L^-1 g_p
    for (int e0 = 0; e0 < ne; e0 += 4) {
      const int e = e0 + es;
      if (lane < 52 && e < ne && (col < 6 || col == 12 || e < nr)) {
        const int i = (2 * e + 1) << ls;
        const int o = col < 6 ? oC + 72 * e + col : col < 12 ? oC + 72 * e + 36 + 6 * (col - 6) : oGv + 6 * i;
        const int stride = col < 6 ? 6 : 1;
        double* dst = base + o;
        double v[6];
#pragma unroll
        for (int r = 0; r < 6; ++r) v[r] = dst[r * stride];
        ltri_fwd(S.Hd[i], v);
#pragma unroll
        for (int r = 0; r < 6; ++r) dst[r * stride] = v[r];
      }
    }
    wave_fence();
    // surviving positions j = 2e: D_j -= W_L(e)^T W_L(e) + W_R(e-1)^T W_R(e-1),
    // g_j -= W_L(e)^T w(e) + W_R(e-1)^T w(e-1); the coupling created by
    // position 2e + 1: -W_R(e)^T W_L(e)
    const int na = (np + 1) / 2;
    for (int e = 0; e < na; ++e) {
      const int eL = min(e, ne - 1), eR = max(e - 1, 0);
      const bool fL = q < 27 ? e < ne : e < nr, fR = q < 27 && e >= 1;
      const int oWL = oC + 72 * eL, oWR = oC + 72 * eR + 36;
      int x1, sx1, y1, sy1, x2, y2, t;
      if (q < 21) {
        x1 = oWL + tp; sx1 = 6; y1 = oWL + tc; sy1 = 6;
        x2 = oWR + 6 * tp; y2 = oWR + 6 * tc;
        t = oHd + 21 * ((2 * e) << ls) + q;
      } else if (q < 27) {
        x1 = oWL + pg; sx1 = 6; y1 = oGv + 6 * ((2 * eL + 1) << ls); sy1 = 1;
        x2 = oWR + 6 * pg; y2 = oGv + 6 * ((2 * eR + 1) << ls);
        t = oGv + 6 * ((2 * e) << ls) + pg;
      } else {
        x1 = oC + 72 * eL + 36 + 6 * pp; sx1 = 1; y1 = oWL + cc; sy1 = 6;
        x2 = x1; y2 = x1;
        t = oN + 36 * eL + pc;
      }
      if (lane < 63 && (fL || fR)) {
        double d = 0.0;
        if (fL) d = dot6s(base + x1, sx1, base + y1, sy1);
        if (fR) d += dot6s(base + x2, 1, base + y2, 1);
        base[t] = (q < 27 ? base[t] : 0.0) - d;
      }
    }
    wave_fence();
    made += nr;
  }
  bool ok0 = true;
  if (lane == 0) {
    double P[21], v[6];
#pragma unroll
    for (int q = 0; q < 21; ++q) P[q] = S.Hd[0][q];
    ok0 = chol_packed<6>(P);
#pragma unroll
    for (int r = 0; r < 6; ++r) v[r] = S.gv[0][r];
    ltri_fwd(P, v);
    ltri_bwd(P, v);
#pragma unroll
    for (int r = 0; r < 6; ++r) S.gv[0][r] = v[r];
  }
  ok = wave_all(ok0) && ok;
  wave_fence();
  for (--ls; ls >= 0; --ls) {
    const int np = bcr_positions(k, ls), ne = np / 2;
    const double* Cp = ls == 0 ? &S.Ho[0][0] : &S.Hn[bcr_first(k, ls)][0];
    if (lane < ne) {
      const int i = (2 * lane + 1) << ls;
      const double* WL = Cp + 72 * lane;
      const double* xl = S.gv[(2 * lane) << ls];
      double v[6];
#pragma unroll
      for (int r = 0; r < 6; ++r) {
        double d = S.gv[i][r];
#pragma unroll
        for (int c = 0; c < 6; ++c) d -= WL[6 * r + c] * xl[c];
        v[r] = d;
      }
      if (2 * lane + 2 < np) {
        const double* WR = WL + 36;
        const double* xr = S.gv[(2 * lane + 2) << ls];
#pragma unroll
        for (int r = 0; r < 6; ++r) {
          double d = v[r];
#pragma unroll
          for (int c = 0; c < 6; ++c) d -= WR[6 * c + r] * xr[c];
          v[r] = d;
        }
      }
      ltri_bwd(S.Hd[i], v);
#pragma unroll
      for (int r = 0; r < 6; ++r) S.gv[i][r] = v[r];
    }
    wave_fence();
  }
  return ok;
}

// ------------------------------------------------------------ pair lane work

// Publish a dof vector (3 per dof lane) as world twists of the bodies:
// lane 2b writes the linear part, lane 2b+1 R_b times the angular part.
DMX_DEV void publish_twist(StackLds& S, const StackRole& ro, int vec, const double* x) {
  if (ro.dof) {
    double* t = S.vec[vec][ro.b] + 3 * ro.half;
    if (ro.half == 0) {
      t[0] = x[0]; t[1] = x[1]; t[2] = x[2];
    } else {
      const V3 w = mul(*(const M3*)S.R[ro.b], mk3(x[0], x[1], x[2]));
      t[0] = w.x; t[1] = w.y; t[2] = w.z;
    }
  }
  wave_fence();
}

// Activity of every edge of this lane's contacts at the vector in S.vec[vec]
// (1 bit per edge, 4 per contact).
DMX_DEV unsigned pair_activity(const StackModel& m, const StackLds& S, const StackRole& ro, const PairSlots& ps,
                               int vec, bool cfd, double beta) {
  unsigned act = 0u;
  if (ro.pair) {
    for (int j = 0; j < ps.cnt; ++j) {
      CRow w;
      contact_row(m, S, ro, ps, j, cfd, beta, w);
      double s[4];
      edge_slack(S, vec, ro.pb1, ro.pb2, w, m.mu, s);
#pragma unroll
      for (int e = 0; e < 4; ++e) act |= (s[e] < 0.0 ? 1u : 0u) << (4 * j + e);
    }
  }
  return act;
}

// The active set at x (in S.vec[kVecX]; into ps.act) and its Hessian blocks
// and gradient into S.Hd / S.Ho / S.gv, in a fixed order of phases: the
// plane pair of body b (with M_b), then the box pairs' lower bodies, then
// their upper bodies; the dof lanes then add M (x - a0).
DMX_DEV void assemble(const StackModel& m, StackLds& S, const StackRole& ro, PairSlots& ps, bool cfd,
                      double beta, const double* x, const double* a0) {
  PairSums a;
  pair_sums_zero(a);
  ps.act = 0u;
  if (ro.pair) {
    for (int j = 0; j < ps.cnt; ++j) {
      CRow w;
      contact_row(m, S, ro, ps, j, cfd, beta, w);
      double s[4];
      edge_slack(S, kVecX, ro.pb1, ro.pb2, w, m.mu, s);
      unsigned act = 0u;
#pragma unroll
      for (int e = 0; e < 4; ++e) act |= (s[e] < 0.0 ? 1u : 0u) << e;
      ps.act |= act << (4 * j);
      if (act) pair_sums_add(a, w, m.mu, act, s, ro.pair == 2);
    }
  }
  // phase 1: plane pair of body b (lane b) sets its diagonal block M_b + part
  if (ro.pair == 1) {
    const int b = ro.pb2;
    double* Hd = S.Hd[b];
#pragma unroll
    for (int i = 0; i < 21; ++i) Hd[i] = 0.0;
    Hd[tri(0, 0)] = m.mass; Hd[tri(1, 1)] = m.mass; Hd[tri(2, 2)] = m.mass;
    Hd[tri(3, 3)] = m.I[0]; Hd[tri(4, 4)] = m.I[1]; Hd[tri(5, 5)] = m.I[2];
    add_diag_block(Hd, a.G, a.K2, a.Q22, S.R[b]);
    double* g = S.gv[b];
#pragma unroll
    for (int i = 0; i < 6; ++i) g[i] = 0.0;
    add_grad(g, 1.0, a.f, a.m2, S.R[b]);
  }
  wave_fence();
  // phase 2: box pair (i, i+1), the lower body i; and the off-diagonal block
  if (ro.pair == 2) {
    const int i = ro.pb1;
    add_diag_block(S.Hd[i], a.G, a.K1, a.Q11, S.R[i]);
    add_grad(S.gv[i], -1.0, a.f, a.m1, S.R[i]);
    // block (i+1, i) = -[[G, K1^T R1], [R2^T K2, -R2^T Q12^T R1]]
    const double* R1 = S.R[i];
    const double* R2 = S.R[i + 1];
    double* O = S.Ho[i];
    double TR[9], BL[9], Qt[9], T[9], BR[9];
    // K1^T R1
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) TR[3 * r + c] = a.K1[r] * R1[c] + a.K1[3 + r] * R1[3 + c] + a.K1[6 + r] * R1[6 + c];
    m3_RtA(R2, a.K2, BL);
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) Qt[3 * r + c] = a.Q12[3 * c + r];
    m3_AR(Qt, R1, T);
    m3_RtA(R2, T, BR);
    double Gf[9];
    sym_unpack(a.G, Gf);
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        O[6 * r + c] = -Gf[3 * r + c];
        O[6 * r + 3 + c] = -TR[3 * r + c];
        O[6 * (3 + r) + c] = -BL[3 * r + c];
        O[6 * (3 + r) + 3 + c] = BR[3 * r + c];
      }
  }
  wave_fence();
  // phase 3: box pair (i, i+1), the upper body i+1
  if (ro.pair == 2) {
    const int b = ro.pb2;
    add_diag_block(S.Hd[b], a.G, a.K2, a.Q22, S.R[b]);
    add_grad(S.gv[b], 1.0, a.f, a.m2, S.R[b]);
  }
  wave_fence();
  // M (x - a0) on the dof lanes (M = diag(m, m, m, I))
  if (ro.dof) {
    double* g = S.gv[ro.b] + 3 * ro.half;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const double mj = ro.half == 0 ? m.mass : m.I[j];
      g[j] += mj * (x[j] - a0[j]);
    }
  }
  wave_fence();
}

// ------------------------------------------------------------ collision
// This lane's pair contacts (values), with r below the margin, their normal
// and their codes if `code` is given.  Returns the count.
DMX_DEV int pair_collide(const StackModel& m, const StackLds& S, const StackRole& ro, double margin, double* r,
                         V3* p, V3* n, int* code) {
  if (ro.pair == 1) {
    const int b = ro.pb2;
    const V3 c = ld3(S.P[b]);
    const double hgt = dot(ld3(m.pn), c - ld3(m.p0));
    if (!(hgt < m.rbound + margin)) return 0;
    *n = ld3(m.pn);
    return box_plane(m.h, m.p0, m.pn, c, *(const M3*)S.R[b], margin, r, p, code);
  }
  if (ro.pair == 2) {
    const int i = ro.pb1, j = ro.pb2;
    const V3 cA = ld3(S.P[i]), cB = ld3(S.P[j]);
    const V3 dc = cB - cA;
    const double reach = 2.0 * m.rbound + margin;
    if (!(dot(dc, dc) < reach * reach)) return 0;
    const M3& RA = *(const M3*)S.R[i];
    const M3& RB = *(const M3*)S.R[j];
    BoxChoice ch;
    if (!box_box_choose(m.h, m.h, cA, RA, cB, RB, margin, &ch)) return 0;
    return box_box_contacts(m.h, m.h, cA, RA, cB, RB, margin, ch, r, p, n, code);
  }
  return 0;
}

// True if cubes that are not neighbours in the model's order touch.  Pairs
// (i, j), j >= i + 2: row i is split between lanes i (first half) and
// 32 + i (second half); bounding spheres are tested first, and the
// narrow phase runs only if some pair's spheres overlap.
DMX_DEV bool nonneighbour_contact(const StackModel& m, const StackLds& S, double margin) {
  const int lane = threadIdx.x & 63;
  const int k = m.k;
  const double reach = 2.0 * m.rbound + margin;
  const int i = lane & 31;
  const int row = max(0, k - 2 - i), half = (row + 1) / 2;
  const int j0 = i + 2 + (lane < 32 ? 0 : half), j1 = i + 2 + (lane < 32 ? half : row);
  bool near = false;
  if (i < k) {
    const V3 cA = ld3(S.P[i]);
    for (int j = j0; j < j1; ++j) {
      const V3 dc = ld3(S.P[j]) - cA;
      near = near || dot(dc, dc) < reach * reach;
    }
  }
  if (!wave_any(near)) return false;
  bool hit = false;
  if (near) {
    const V3 cA = ld3(S.P[i]);
    const M3& RA = *(const M3*)S.R[i];
    for (int j = j0; j < j1 && !hit; ++j) {
      const V3 cB = ld3(S.P[j]);
      const V3 dc = cB - cA;
      if (!(dot(dc, dc) < reach * reach)) continue;
      const M3& RB = *(const M3*)S.R[j];
      BoxChoice ch;
      if (box_box_choose(m.h, m.h, cA, RA, cB, RB, margin, &ch) &&
          box_box_contacts(m.h, m.h, cA, RA, cB, RB, margin, ch, nullptr, nullptr, nullptr, nullptr) > 0)
        hit = true;
    }
  }
  return wave_any(hit);
}

// Body frames (FK of the free joints: the quaternion normalized) and the
// velocity twists, then the contact pool: every pair lane's contacts, in
// pair order (plane pairs by body, then box pairs by lower body), at most
// kStackContacts (the rest dropped, status bit 16).  Returns the pair lane's
// slots.
DMX_DEV PairSlots stack_setup(const StackModel& m, StackLds& S, const StackRole& ro, const double* yq,
                              const double* yv, bool cfd, StackStat& st, bool codes = false) {
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
  const double margin = cfd ? m.cf[2] : 0.0;
  double r[kBoxBoxMax];
  V3 p[kBoxBoxMax], n = ld3(m.pn);
  int cc[kBoxBoxMax];
  int cnt = pair_collide(m, S, ro, margin, r, p, &n, codes ? cc : nullptr);
  if (nonneighbour_contact(m, S, margin)) st.status |= kStGraph;
  int total;
  const int off = wave_excl_scan(cnt, &total);
  if (total > kStackContacts) st.status |= kStOverflow;
  const int keep = max(0, min(cnt, kStackContacts - off));
#pragma unroll
  for (int j = 0; j < kBoxBoxMax; ++j) {
    if (j < keep) {
      const int c = off + j;
      S.cp[0][c] = p[j].x; S.cp[1][c] = p[j].y; S.cp[2][c] = p[j].z;
      S.cr[c] = r[j];
      if (codes) S.code[c] = cc[j];
    }
  }
  wave_fence();
  PairSlots ps;
  ps.off = off;
  ps.cnt = keep;
  ps.act = 0u;
  ps.ahat = ro.pair == 2 ? m.ahat_box : m.ahat_plane;
  ps.n = n;
  return ps;
}

// unconstrained acceleration a0 = M^-1 (tau - c) of this dof lane, with
// c = (-m g, w x I w)
DMX_DEV void stack_a0(const StackModel& m, const StackRole& ro, const double* yv, const double* tau, double* a0) {
  if (ro.half == 0) {
#pragma unroll
    for (int j = 0; j < 3; ++j) a0[j] = m.grav[j] + m.imass * tau[j];
  } else {
    const V3 w = mk3(yv[0], yv[1], yv[2]);
    const V3 Iw = mk3(m.I[0] * w.x, m.I[1] * w.y, m.I[2] * w.z);
    const V3 g = cross(w, Iw);
    a0[0] = m.Iinv[0] * (tau[0] - g.x);
    a0[1] = m.Iinv[1] * (tau[1] - g.y);
    a0[2] = m.Iinv[2] * (tau[2] - g.z);
  }
}

// Exact Newton on the primal problem (Sec. 2.1) from a0 (or the warm start
// xw), as for single bodies: the Newton direction of the current active set;
// if the unit step changes no edge's activity (or is at rounding level) it
// ends the solve, otherwise the exact minimizer along the direction by a
// bracketed semismooth Newton iteration on the directional derivative.
DMX_DEV void stack_newton(const StackModel& m, StackLds& S, const StackRole& ro, PairSlots& ps, bool cfd,
                          double beta, int maxit, const double* a0, const double* xw, double* x, StackStat& st) {
#pragma unroll
  for (int j = 0; j < 3; ++j) x[j] = a0[j];
  publish_twist(S, ro, kVecX, x);
  ps.act = pair_activity(m, S, ro, ps, kVecX, cfd, beta);
  if (!wave_any(ps.act != 0u)) return;  // no row active at a0: a0 is the minimizer
  if (xw) {
#pragma unroll
    for (int j = 0; j < 3; ++j) x[j] = xw[j];
    publish_twist(S, ro, kVecX, x);
  }
  const double Mj[2][3] = {{m.mass, m.mass, m.mass}, {m.I[0], m.I[1], m.I[2]}};
  for (int it = 0; it < maxit; ++it) {
    st.newton_it++;
    if (ro.lane == 0) st.u_nit++;
    assemble(m, S, ro, ps, cfd, beta, x, a0);
    if (ro.pair) {
      st.u_nedge += __popc(ps.act);
      int nc = 0;
      for (int j = 0; j < ps.cnt; ++j) nc += ((ps.act >> (4 * j)) & 15u) != 0u;
      st.u_ncon += nc;
      if (ro.pair == 2) st.u_ncon2 += nc;
    }
    // right-hand side -g
    if (ro.dof) {
#pragma unroll
      for (int j = 0; j < 3; ++j) S.gv[ro.b][3 * ro.half + j] = -S.gv[ro.b][3 * ro.half + j];
    }
    wave_fence();
    if (!block_factor_solve(S, m.k)) { st.status |= 4; return; }
    double dl[3] = {0, 0, 0};
    if (ro.dof) {
#pragma unroll
      for (int j = 0; j < 3; ++j) dl[j] = S.gv[ro.b][3 * ro.half + j];
    }
    wave_fence();
    double dmax = 0.0, xmax = 1.0;
    if (ro.dof) {
#pragma unroll
      for (int j = 0; j < 3; ++j) { dmax = fmax(dmax, fabs(dl[j])); xmax = fmax(xmax, fmax(fabs(x[j]), fabs(a0[j]))); }
    }
    dmax = wave_max(dmax);
    xmax = wave_max(xmax);
    if (dmax <= 1e-13 * xmax) {
#pragma unroll
      for (int j = 0; j < 3; ++j) x[j] += dl[j];
      return;
    }
    publish_twist(S, ro, kVecD, dl);
    // activity after the unit step
    unsigned act1 = 0u;
    if (ro.pair) {
      for (int j = 0; j < ps.cnt; ++j) {
        CRow w;
        contact_row(m, S, ro, ps, j, cfd, beta, w);
        double s[4], t[4];
        edge_slack(S, kVecX, ro.pb1, ro.pb2, w, m.mu, s);
        edge_dir(S, kVecD, ro.pb1, ro.pb2, w, m.mu, t);
#pragma unroll
        for (int e = 0; e < 4; ++e) act1 |= (s[e] + t[e] < 0.0 ? 1u : 0u) << (4 * j + e);
      }
    }
    if (wave_all(act1 == ps.act)) {
#pragma unroll
      for (int j = 0; j < 3; ++j) x[j] += dl[j];
      return;
    }
    // exact line search: root of phi'(a) = a C2(a) + C1(a)
    double mm[2] = {0.0, 0.0};
    if (ro.dof) {
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const double Md = Mj[ro.half][j] * dl[j];
        mm[0] += dl[j] * Md;
        mm[1] += (x[j] - a0[j]) * Md;
      }
    }
    wave_sum<2>(mm);
    const double dMd = mm[0], xMd = mm[1];
    double lo = 0.0, hi = 1e300, al = 1.0;
    for (int ls = 0; ls < 60; ++ls) {
      double cc[2] = {0.0, 0.0};
      unsigned sa = 0u, sn = 0u;
      double an = al;
      if (ro.pair) {
        for (int j = 0; j < ps.cnt; ++j) {
          CRow w;
          contact_row(m, S, ro, ps, j, cfd, beta, w);
          double s[4], t[4];
          edge_slack(S, kVecX, ro.pb1, ro.pb2, w, m.mu, s);
          edge_dir(S, kVecD, ro.pb1, ro.pb2, w, m.mu, t);
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const bool on = s[e] + al * t[e] < 0.0;
            sa |= (on ? 1u : 0u) << (4 * j + e);
            const double dt = on ? w.D * t[e] : 0.0;
            cc[1] += dt * t[e];
            cc[0] += dt * s[e];
          }
        }
        st.u_ls += ps.cnt;
      }
      wave_sum<2>(cc);
      const double c1 = cc[0] + xMd, c2 = cc[1] + dMd;
      const double dphi = al * c2 + c1;
      if (dphi > 0.0) hi = al; else lo = al;
      an = (c2 > 0.0) ? -c1 / c2 : al;
      if (!isfinite(an)) an = al;
      if (ro.pair) {
        for (int j = 0; j < ps.cnt; ++j) {
          CRow w;
          contact_row(m, S, ro, ps, j, cfd, beta, w);
          double s[4], t[4];
          edge_slack(S, kVecX, ro.pb1, ro.pb2, w, m.mu, s);
          edge_dir(S, kVecD, ro.pb1, ro.pb2, w, m.mu, t);
#pragma unroll
          for (int e = 0; e < 4; ++e) sn |= (s[e] + an * t[e] < 0.0 ? 1u : 0u) << (4 * j + e);
        }
      }
      if (wave_all(sa == sn)) { al = an; break; }
      if (!(an > lo && an < hi)) an = (hi < 1e299) ? 0.5 * (lo + hi) : 2.0 * al;
      al = an;
      if (hi - lo <= 1e-15 * hi) break;
      if (ls == 59) al = lo > 0.0 ? lo : al;
    }
#pragma unroll
    for (int j = 0; j < 3; ++j) x[j] += al * dl[j];
    publish_twist(S, ro, kVecX, x);
  }
  st.status |= 8;
}

// Acceleration of the right-hand side F(x) = (v, qacc) of a stack world at
// this dof lane's stage state (yq: position or quaternion, yv: its 3
// velocity dofs; tau: generalized forces of its dofs); every lane calls it.
DMX_DEV void stack_acc(const StackModel& m, StackLds& S, const StackRole& ro, const double* yq, const double* yv,
                       const double* tau, bool cfd, double beta, int maxit, const double* xw, double* acc,
                       StackStat& st) {
  PairSlots ps = stack_setup(m, S, ro, yq, yv, cfd, st);
  if (ro.lane == 0) st.u_rhs++;
  if (ro.pair) st.u_con += ps.cnt;
  if (ro.pair == 2) st.u_con2 += ps.cnt;
  double a0[3];
  stack_a0(m, ro, yv, tau, a0);
  if (st.status & kStGraph) {
#pragma unroll
    for (int j = 0; j < 3; ++j) acc[j] = a0[j];
    return;
  }
  stack_newton(m, S, ro, ps, cfd, beta, maxit, a0, xw, acc, st);
}

}  // namespace dmx
