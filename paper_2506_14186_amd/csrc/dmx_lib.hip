// Host side of the dmx C ABI: model compilation, kernel dispatch, tapes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <set>

#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/dmx.h"
#include "dmx_tree.hpp"
#include "dmx_launch.hpp"
#include "dmx_server.hpp"
#include "dmx_stack_host.hpp"

using namespace dmx_host;

namespace {

thread_local std::string g_err;

dmx_status fail(dmx_status code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIP_TRY(expr)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess) return fail(DMX_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

constexpr double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------- host math
void quat_to_mat(const double* q, double* R) {
  double n = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  double w = q[0] / n, x = q[1] / n, y = q[2] / n, z = q[3] / n;
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z); R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z); R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y); R[7] = 2 * (y * z + w * x); R[8] = 1 - 2 * (x * x + y * y);
}

// Principal moments (about the centre) and mass of a uniform solid primitive.
bool solid_inertia(int type, const double* s, double mass_in, double* mass, double* I) {
  double vol;
  switch (type) {
    case DMX_GEOM_SPHERE: vol = 4.0 / 3.0 * kPi * s[0] * s[0] * s[0]; break;
    case DMX_GEOM_BOX: vol = 8.0 * s[0] * s[1] * s[2]; break;
    case DMX_GEOM_CAPSULE: vol = kPi * s[0] * s[0] * (2.0 * s[1]) + 4.0 / 3.0 * kPi * s[0] * s[0] * s[0]; break;
    default: return false;
  }
  const double m = mass_in > 0.0 ? mass_in : 1000.0 * vol;
  *mass = m;
  if (type == DMX_GEOM_SPHERE) {
    I[0] = I[1] = I[2] = 2.0 / 5.0 * m * s[0] * s[0];
  } else if (type == DMX_GEOM_BOX) {
    const double a2 = 4.0 * s[0] * s[0], b2 = 4.0 * s[1] * s[1], c2 = 4.0 * s[2] * s[2];  // full edges squared
    I[0] = m * (b2 + c2) / 12.0; I[1] = m * (a2 + c2) / 12.0; I[2] = m * (a2 + b2) / 12.0;
  } else {
    // capsule: cylinder (length len) + two hemispheres, axis along z
    const double r = s[0], len = 2.0 * s[1];
    const double vcyl = kPi * r * r * len, vcap = 4.0 / 3.0 * kPi * r * r * r;
    const double mcyl = m * vcyl / (vcyl + vcap), mcap = m - mcyl;
    const double hemi_offset = 3.0 * r / 8.0;  // hemisphere centroid from its flat face
    const double ihemi_c = 2.0 / 5.0 * r * r - hemi_offset * hemi_offset;  // per unit mass, about centroid
    const double dist = 0.5 * len + hemi_offset;
    I[2] = mcyl * r * r / 2.0 + mcap * 2.0 / 5.0 * r * r;
    I[0] = I[1] = mcyl * (r * r / 4.0 + len * len / 12.0) + mcap * (ihemi_c + dist * dist);
  }
  return true;
}

// 1/mid^(p-1) and 1/(1-mid)^(p-1) of the penetration and CFD impedance splines
void spline_scales(dmx::PairF& pr) {
  pr.ssc[0] = 1.0 / std::pow(pr.si[3], pr.si[4] - 1.0);
  pr.ssc[1] = 1.0 / std::pow(1.0 - pr.si[3], pr.si[4] - 1.0);
  pr.ssc[2] = 1.0 / std::pow(pr.cf[3], pr.cf[4] - 1.0);
  pr.ssc[3] = 1.0 / std::pow(1.0 - pr.cf[3], pr.cf[4] - 1.0);
  pr.iwid[0] = 1.0 / pr.si[2];
  pr.iwid[1] = 1.0 / pr.cf[2];
}

// solref and the impedance splines within their domain: t_c and the damping
// ratio positive; impedances in [0, 1) (dwidth in (0, 1): it divides the
// stiffness); widths positive; midpoints in [0, 1]; powers at least 1 (the
// spline and its slope stay finite at 0)
static bool contact_params_ok(double tc, double dr, const dmx::PairF& pr) {
  auto spline_ok = [](const double* s) {
    return s[0] >= 0.0 && s[0] < 1.0 && s[1] >= 0.0 && s[1] < 1.0 && s[2] > 0.0 && s[3] >= 0.0 && s[3] <= 1.0 &&
           s[4] >= 1.0;
  };
  return tc > 0.0 && dr > 0.0 && pr.si[1] > 0.0 && spline_ok(pr.si) && spline_ok(pr.cf);
}

void make_tangents(const double* n, double* t1, double* t2) {
  double a[3] = {0, 0, 0};
  if (std::fabs(n[0]) < 0.5) a[0] = 1.0; else a[1] = 1.0;
  const double an = a[0] * n[0] + a[1] * n[1] + a[2] * n[2];
  double t[3] = {a[0] - an * n[0], a[1] - an * n[1], a[2] - an * n[2]};
  const double tn = std::sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
  for (int i = 0; i < 3; ++i) t1[i] = t[i] / tn;
  t2[0] = n[1] * t1[2] - n[2] * t1[1];
  t2[1] = n[2] * t1[0] - n[0] * t1[2];
  t2[2] = n[0] * t1[1] - n[1] * t1[0];
}

int bucket(int n) {
  int b = 1;
  while (b < n) b *= 2;
  return b;
}

size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

}  // namespace

// ---------------------------------------------------------------- objects
struct dmx_model {
  int kind = 0;  // 0: single free body, 1: hinge/slide tree; plane contacts; 2: stack of free cubes
  int nq = 0, nv = 0, nu = 0, nc = 0, ncb = 0, nb = 1;
  dmx::FreeModel host{};
  dmx::TreeModel tree{};
  void* dev = nullptr;
  std::atomic<int> tuned_team{0};  // team size chosen by dmx_autotune (0: none)
  bool stack_ok = false;           // the stack kernels cover the model (a stack of k >= 1 cubes)
  int box_geom = -1;               // single free body: the one box geom its contacts use (-2: several)
  dmx::StackModel stk{};
  void* stk_dev = nullptr;
};

struct dmx_tape {
  const dmx_model* model = nullptr;
  int W = 0, n_int = 0, nu = 0, rec = 0, team = 1;
  double dt = 0.0;
  long long cap = 0;
  double* records = nullptr;
  int* n_acc = nullptr;
  int* status = nullptr;
  const double* u = nullptr;
  dmx::SolverOpts o{};
  AdjFn adj = nullptr;
  AdjFn otd = nullptr;  // the optimize-then-discretize adjoint of the same kernel family
  int64_t* adj_counters = nullptr;
  int plain = 0;
  const int32_t* world_intervals = nullptr;  // tape-owned copies of the caller's tables (or null)
  const int32_t* world_order = nullptr;
  int* tables = nullptr;  // [2][W]: per-world intervals and processing order, copied at each rollout
  int* queue = nullptr;   // [2] work counters of the forward and reverse launches
  bool use_queue = false;
  // stack tapes (ragged worlds): per-world tables on the device and the
  // arguments of the forward launch, reused by the reverse sweep
  bool stack = false;
  std::vector<const dmx_model*> models;  // the worlds' models (host)
  std::vector<long long> t_off_h;        // per-world tape offsets (host copy)
  std::vector<int> rec_h;                // per-world record lengths (host copy)
  void* stk_tables = nullptr;            // device: models, x_off, u_off, t_off, cap, order
  size_t stk_tables_bytes = 0;
  dmx::StackArgs sa{};
};

extern "C" {

const char* dmx_last_error(void) { return g_err.c_str(); }

void dmx_default_opts(dmx_solver_opts* o) {
  std::memset(o, 0, sizeof(*o));
  o->rtol = 1e-6; o->atol = 1e-8; o->h0 = 1e-3; o->safety = 0.9; o->facmin = 0.2; o->facmax = 10.0;
  o->kP = 0.2; o->kI = 0.4; o->err_order = 5.0; o->err_floor = 1e-6; o->max_attempts = 1000000;
  o->newton_maxit = 100; o->cfd = 0; o->softplus_beta = 1e4; o->tape_steps = 0; o->lanes_per_world = 0;
  o->h_levels = 0;
  o->tape_stages = -1;
}

static dmx_status create_tree_model(const dmx_model_desc* d, dmx_model** out);

// A stack of k free cubes on a plane, in the layout the stack kernels take:
// k bodies (parent -1), each with one free joint and one box geom at its
// origin; a world plane; the pairs (plane, cube b) for b in order, then
// (cube i, cube j) for i < j in lexicographic order, all with the same
// parameters; equal cubes with principal axes along the body axes.
static bool make_stack_model(const dmx_model_desc* d, dmx::StackModel* st, std::string* why) {
  auto no = [&](const char* w) { *why = w; return false; };
  const int k = d->nbody;
  if (k < 1 || k > dmx::kStackBodies) return no("stacks take 1..32 cubes");
  if (d->njnt != k) return no("one free joint per cube");
  for (int b = 0; b < k; ++b) {
    if (d->body_parent[b] != -1 || d->jnt_body[b] != b || d->jnt_type[b] != DMX_JOINT_FREE) return no("one free joint per cube");
    if (d->body_iner_type[b] != DMX_GEOM_BOX) return no("cube inertia");
    const double* q = &d->body_iner_quat[4 * b];
    if (q[0] != 1.0 || q[1] != 0.0 || q[2] != 0.0 || q[3] != 0.0) return no("inertia axes along the body axes");
    for (int i = 0; i < 3; ++i)
      if (d->body_iner_size[3 * b + i] != d->body_iner_size[i]) return no("equal cubes");
    if (d->body_mass[b] != d->body_mass[0]) return no("equal cubes");
  }
  if (d->ngeom != k + 1) return no("one plane and one box per cube");
  int plane = -1;
  std::vector<int> box_of(k, -1);
  for (int g = 0; g < d->ngeom; ++g) {
    if (d->geom_type[g] == DMX_GEOM_PLANE && d->geom_body[g] == -1) { plane = g; continue; }
    const int b = d->geom_body[g];
    if (d->geom_type[g] != DMX_GEOM_BOX || b < 0 || b >= k || box_of[b] >= 0) return no("one box per cube");
    for (int i = 0; i < 3; ++i)
      if (d->geom_pos[3 * g + i] != 0.0 || d->geom_size[3 * g + i] != d->body_iner_size[i]) return no("box geom at the cube");
    const double* q = &d->geom_quat[4 * g];
    if (q[0] != 1.0 || q[1] != 0.0 || q[2] != 0.0 || q[3] != 0.0) return no("box geom at the cube");
    box_of[b] = g;
  }
  if (plane < 0) return no("a world plane");
  if (d->npair != k + k * (k - 1) / 2) return no("every cube-plane and cube-cube pair");
  int p = 0;
  for (int b = 0; b < k; ++b, ++p)
    if (d->pair_g1[p] != plane || d->pair_g2[p] != box_of[b]) return no("pairs: plane-cube in cube order first");
  for (int i = 0; i < k; ++i)
    for (int j = i + 1; j < k; ++j, ++p)
      if (d->pair_g1[p] != box_of[i] || d->pair_g2[p] != box_of[j]) return no("pairs: then cube pairs (i, j), i < j");
  for (int q = 1; q < d->npair; ++q) {
    if (d->pair_mu[q] != d->pair_mu[0]) return no("equal pair parameters");
    for (int i = 0; i < 2; ++i) if (d->pair_solref[2 * q + i] != d->pair_solref[i]) return no("equal pair parameters");
    for (int i = 0; i < 5; ++i)
      if (d->pair_solimp[5 * q + i] != d->pair_solimp[i] || d->pair_cfd[5 * q + i] != d->pair_cfd[i])
        return no("equal pair parameters");
  }
  if (d->nu < 0 || d->nu > 6) return no("at most 6 controls");
  dmx::StackModel s{};
  s.k = k;
  s.nu = d->nu;
  for (int i = 0; i < d->nu; ++i) {
    if (d->ctrl_dof[i] < 0 || d->ctrl_dof[i] >= 6 * k) return no("bad ctrl dof");
    s.ctrl[i] = d->ctrl_dof[i];
  }
  double mass, Ip[3];
  if (!solid_inertia(DMX_GEOM_BOX, d->body_iner_size, d->body_mass[0], &mass, Ip)) return no("inertia");
  s.mass = mass;
  s.imass = 1.0 / mass;
  double hn = 0.0;
  for (int i = 0; i < 3; ++i) {
    s.I[i] = Ip[i];
    s.Iinv[i] = 1.0 / Ip[i];
    s.h[i] = d->body_iner_size[i];
    s.grav[i] = d->gravity[i];
    hn += s.h[i] * s.h[i];
  }
  s.rbound = std::sqrt(hn);
  double Rp[9];
  quat_to_mat(&d->geom_quat[4 * plane], Rp);
  for (int i = 0; i < 3; ++i) { s.p0[i] = d->geom_pos[3 * plane + i]; s.pn[i] = Rp[i * 3 + 2]; }
  dmx::PairF pr{};
  for (int i = 0; i < 5; ++i) { pr.si[i] = d->pair_solimp[i]; pr.cf[i] = d->pair_cfd[i]; }
  spline_scales(pr);
  const double tc = d->pair_solref[0], dr = d->pair_solref[1], dw = pr.si[1];
  if (!contact_params_ok(tc, dr, pr)) return no("solref/solimp/cfd out of range");
  for (int i = 0; i < 5; ++i) { s.si[i] = pr.si[i]; s.cf[i] = pr.cf[i]; }
  for (int i = 0; i < 4; ++i) s.ssc[i] = pr.ssc[i];
  s.iwid[0] = pr.iwid[0];
  s.iwid[1] = pr.iwid[1];
  s.mu = d->pair_mu[0];
  s.bcoef = 2.0 / (dw * tc);
  s.kscale = 1.0 / (dw * dw * tc * tc * dr * dr);
  // A = (1 + mu^2)(w_1 + w_2), w = 1/m for a free body, 0 for the world
  s.ahat_plane = (1.0 + s.mu * s.mu) * s.imass;
  s.ahat_box = (1.0 + s.mu * s.mu) * 2.0 * s.imass;
  *st = s;
  return true;
}

static dmx_status upload_stack(dmx_model* m) {
  hipError_t e = hipMalloc(&m->stk_dev, sizeof(dmx::StackModel));
  if (e == hipSuccess) e = hipMemcpy(m->stk_dev, &m->stk, sizeof(dmx::StackModel), hipMemcpyHostToDevice);
  if (e != hipSuccess) return fail(DMX_ERR_HIP, std::string("stack model upload: ") + hipGetErrorString(e));
  return DMX_OK;
}

dmx_status dmx_model_create(const dmx_model_desc* d, dmx_model** out) {
  if (!d || !out) return fail(DMX_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  bool any_free = false;
  for (int j = 0; j < d->njnt; ++j) any_free = any_free || d->jnt_type[j] == DMX_JOINT_FREE;
  if (!any_free) return create_tree_model(d, out);
  dmx::StackModel stk{};
  std::string why;
  const bool stack_ok = make_stack_model(d, &stk, &why);
  if (d->nbody > 1) {
    if (!stack_ok)
      return fail(DMX_ERR_UNSUPPORTED, "several free bodies are supported as a stack of cubes: " + why);
    dmx_model* m = new dmx_model();
    m->kind = 2;
    m->nb = stk.k;
    m->nq = 7 * stk.k;
    m->nv = 6 * stk.k;
    m->nu = d->nu;
    m->nc = dmx::kStackContacts;
    m->stack_ok = true;
    m->stk = stk;
    const dmx_status r = upload_stack(m);
    if (r != DMX_OK) { delete m; return r; }
    *out = m;
    return DMX_OK;
  }
  if (d->nbody != 1 || d->njnt != 1 || d->jnt_type[0] != DMX_JOINT_FREE || d->body_parent[0] != -1)
    return fail(DMX_ERR_UNSUPPORTED, "free joints are supported as the single joint of a single body");
  if (d->npair > dmx::kMaxPairs) return fail(DMX_ERR_UNSUPPORTED, "too many pairs");
  if (d->nu > 6) return fail(DMX_ERR_INVALID_ARG, "at most 6 controls on a free body");
  dmx_model* m = new dmx_model();
  dmx::FreeModel& f = m->host;
  m->nq = 7; m->nv = 6; m->nu = d->nu;
  double mass, Ip[3];
  if (!solid_inertia(d->body_iner_type[0], d->body_iner_size, d->body_mass[0], &mass, Ip)) {
    delete m;
    return fail(DMX_ERR_INVALID_ARG, "unknown inertial primitive");
  }
  double Ri[9];
  quat_to_mat(d->body_iner_quat, Ri);
  f.mass = mass;
  f.imass = 1.0 / mass;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += Ri[i * 3 + k] * Ip[k] * Ri[j * 3 + k];
      f.I[i * 3 + j] = s;
    }
  // inverse of the 3x3 inertia
  {
    const double* A = f.I;
    double c00 = A[4] * A[8] - A[5] * A[7], c01 = A[5] * A[6] - A[3] * A[8], c02 = A[3] * A[7] - A[4] * A[6];
    double det = A[0] * c00 + A[1] * c01 + A[2] * c02;
    f.Iinv[0] = c00 / det; f.Iinv[3] = c01 / det; f.Iinv[6] = c02 / det;
    f.Iinv[1] = (A[2] * A[7] - A[1] * A[8]) / det; f.Iinv[4] = (A[0] * A[8] - A[2] * A[6]) / det;
    f.Iinv[7] = (A[1] * A[6] - A[0] * A[7]) / det;
    f.Iinv[2] = (A[1] * A[5] - A[2] * A[4]) / det; f.Iinv[5] = (A[2] * A[3] - A[0] * A[5]) / det;
    f.Iinv[8] = (A[0] * A[4] - A[1] * A[3]) / det;
  }
  for (int i = 0; i < 3; ++i) f.grav[i] = d->gravity[i];
  for (int i = 0; i < d->nu; ++i) {
    if (d->ctrl_dof[i] < 0 || d->ctrl_dof[i] >= 6) { delete m; return fail(DMX_ERR_INVALID_ARG, "bad ctrl dof"); }
    f.ctrl[i] = d->ctrl_dof[i];
  }
  f.nu = d->nu;
  f.np = d->npair;
  const double invw = 1.0 / mass;  // translational inverse weight of a free body
  int nc = 0;
  for (int p = 0; p < d->npair; ++p) {
    const int g1 = d->pair_g1[p], g2 = d->pair_g2[p];
    if (g1 < 0 || g1 >= d->ngeom || g2 < 0 || g2 >= d->ngeom) { delete m; return fail(DMX_ERR_INVALID_ARG, "bad pair geom"); }
    if (d->geom_type[g1] != DMX_GEOM_PLANE || d->geom_body[g1] != -1 || d->geom_body[g2] != 0) {
      delete m;
      return fail(DMX_ERR_UNSUPPORTED, "pairs must be (world plane, body geom)");
    }
    const int t2 = d->geom_type[g2];
    if (t2 != DMX_GEOM_SPHERE && t2 != DMX_GEOM_CAPSULE && t2 != DMX_GEOM_BOX) {
      delete m;
      return fail(DMX_ERR_UNSUPPORTED, "contact pairs are a world plane against a sphere, capsule or box geom");
    }
    dmx::PairF& pr = f.pair[p];
    pr.gtype = t2;
    if (t2 == DMX_GEOM_BOX) m->box_geom = (m->box_geom == -1 || m->box_geom == g2) ? g2 : -2;
    pr.ncon = (t2 == DMX_GEOM_CAPSULE) ? 2 : (t2 == DMX_GEOM_BOX) ? 4 : 1;
    double Rg[9], Rp[9];
    quat_to_mat(&d->geom_quat[4 * g2], Rg);
    quat_to_mat(&d->geom_quat[4 * g1], Rp);
    for (int i = 0; i < 9; ++i) pr.gR[i] = Rg[i];
    for (int i = 0; i < 3; ++i) {
      pr.l[i] = d->geom_pos[3 * g2 + i];
      pr.ax[i] = (t2 == DMX_GEOM_BOX) ? d->geom_size[3 * g2 + i] : Rg[i * 3 + 2] * d->geom_size[3 * g2 + 1];
      pr.p0[i] = d->geom_pos[3 * g1 + i];
      pr.n[i] = Rp[i * 3 + 2];
    }
    make_tangents(pr.n, pr.t1, pr.t2);
    pr.rad = (t2 == DMX_GEOM_BOX) ? 0.0 : d->geom_size[3 * g2];
    pr.mu = d->pair_mu[p];
    const double tc = d->pair_solref[2 * p], dr = d->pair_solref[2 * p + 1];
    for (int i = 0; i < 5; ++i) { pr.si[i] = d->pair_solimp[5 * p + i]; pr.cf[i] = d->pair_cfd[5 * p + i]; }
    spline_scales(pr);
    const double dw = pr.si[1];
    if (!contact_params_ok(tc, dr, pr)) {
      delete m;
      return fail(DMX_ERR_INVALID_ARG, "solref/solimp/cfd out of range");
    }
    pr.bcoef = 2.0 / (dw * tc);
    pr.kscale = 1.0 / (dw * dw * tc * tc * dr * dr);
    pr.ahat = (1.0 + pr.mu * pr.mu) * invw;
    pr.solref[0] = tc;
    pr.solref[1] = dr;
    for (int c = 0; c < pr.ncon; ++c) {
      if (nc >= dmx::kMaxSlots) { delete m; return fail(DMX_ERR_UNSUPPORTED, "too many contact slots"); }
      f.cpair[nc] = p;
      f.csub[nc] = c;
      ++nc;
    }
  }
  f.nc = nc;
  m->nc = nc;
  m->ncb = bucket(nc > 0 ? nc : 1);
  hipError_t e = hipMalloc(&m->dev, sizeof(dmx::FreeModel));
  if (e == hipSuccess) e = hipMemcpy(m->dev, &f, sizeof(dmx::FreeModel), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    if (m->dev) (void)hipFree(m->dev);
    delete m;
    return fail(DMX_ERR_HIP, std::string("model upload: ") + hipGetErrorString(e));
  }
  if (stack_ok) {  // a one-cube stack: also runs in batches of stacks
    m->stack_ok = true;
    m->stk = stk;
    const dmx_status r = upload_stack(m);
    if (r != DMX_OK) { dmx_model_destroy(m); return r; }
  }
  *out = m;
  return DMX_OK;
}

// host-side forward kinematics of a tree at q (body origins, rotations, joint axes/anchors)
static void host_tree_fk(const dmx::TreeModel& t, const double* q, double (*P)[3], double (*R)[9], double (*A)[3],
                         double (*O)[3]) {
  auto mm = [](const double* a, const double* b, double* r) {
    double tmp[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) tmp[i * 3 + j] = a[i * 3] * b[j] + a[i * 3 + 1] * b[3 + j] + a[i * 3 + 2] * b[6 + j];
    std::memcpy(r, tmp, sizeof(tmp));
  };
  auto mv = [](const double* a, const double* v, double* r) {
    double tmp[3];
    for (int i = 0; i < 3; ++i) tmp[i] = a[i * 3] * v[0] + a[i * 3 + 1] * v[1] + a[i * 3 + 2] * v[2];
    std::memcpy(r, tmp, sizeof(tmp));
  };
  for (int b = 0; b < t.nb; ++b) {
    double pp[3] = {0, 0, 0}, Rp[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    if (t.bparent[b] >= 0) { std::memcpy(pp, P[t.bparent[b]], sizeof(pp)); std::memcpy(Rp, R[t.bparent[b]], sizeof(Rp)); }
    double p[3], Rb[9], off[3];
    mv(Rp, t.bpos[b], off);
    for (int i = 0; i < 3; ++i) p[i] = pp[i] + off[i];
    mm(Rp, t.bR[b], Rb);
    for (int j = t.bj0[b]; j < t.bj0[b] + t.bjn[b]; ++j) {
      double a[3], o[3];
      mv(Rb, t.jaxis[j], a);
      mv(Rb, t.jpos[j], o);
      for (int i = 0; i < 3; ++i) o[i] += p[i];
      std::memcpy(A[j], a, sizeof(a));
      std::memcpy(O[j], o, sizeof(o));
      if (t.jtype[j] == DMX_JOINT_HINGE) {
        const double* k = t.jaxis[j];
        const double c = std::cos(q[j]), s = std::sin(q[j]), u = 1.0 - c;
        const double Rot[9] = {u * k[0] * k[0] + c, u * k[0] * k[1] - s * k[2], u * k[0] * k[2] + s * k[1],
                               u * k[0] * k[1] + s * k[2], u * k[1] * k[1] + c, u * k[1] * k[2] - s * k[0],
                               u * k[0] * k[2] - s * k[1], u * k[1] * k[2] + s * k[0], u * k[2] * k[2] + c};
        mm(Rb, Rot, Rb);
        double rp[3];
        mv(Rb, t.jpos[j], rp);
        for (int i = 0; i < 3; ++i) p[i] = o[i] - rp[i];
      } else {
        for (int i = 0; i < 3; ++i) p[i] += a[i] * q[j];
      }
    }
    std::memcpy(P[b], p, sizeof(p));
    std::memcpy(R[b], Rb, sizeof(Rb));
  }
}

static dmx_status create_tree_model(const dmx_model_desc* d, dmx_model** out) {
  if (d->nbody < 1 || d->nbody > dmx::kTreeBodies || d->njnt < 1 || d->njnt > dmx::kTreeJoints)
    return fail(DMX_ERR_UNSUPPORTED, "tree models take 1..8 bodies and 1..8 hinge/slide joints");
  if (d->npair > dmx::kMaxPairs || d->nu > 8) return fail(DMX_ERR_UNSUPPORTED, "too many pairs or controls");
  dmx_model* m = new dmx_model();
  m->kind = 1;
  dmx::TreeModel& t = m->tree;
  t.nb = d->nbody; t.nj = d->njnt; t.nu = d->nu;
  m->nb = t.nb; m->nq = m->nv = t.nj; m->nu = d->nu;
  for (int b = 0; b < t.nb; ++b) {
    t.bparent[b] = d->body_parent[b];
    if (t.bparent[b] >= b) { delete m; return fail(DMX_ERR_INVALID_ARG, "bodies must follow their parents"); }
    for (int i = 0; i < 3; ++i) t.bpos[b][i] = d->body_pos[3 * b + i];
    quat_to_mat(&d->body_quat[4 * b], t.bR[b]);
    double mass, Ip[3], Ri[9];
    if (!solid_inertia(d->body_iner_type[b], &d->body_iner_size[3 * b], d->body_mass[b], &mass, Ip)) {
      delete m;
      return fail(DMX_ERR_INVALID_ARG, "unknown inertial primitive");
    }
    quat_to_mat(&d->body_iner_quat[4 * b], Ri);
    t.bmass[b] = mass;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double acc = 0.0;
        for (int k = 0; k < 3; ++k) acc += Ri[i * 3 + k] * Ip[k] * Ri[j * 3 + k];
        t.bI[b][i * 3 + j] = acc;
      }
    t.bj0[b] = 0; t.bjn[b] = 0;
  }
  for (int j = 0; j < t.nj; ++j) {
    const int b = d->jnt_body[j];
    if (d->jnt_type[j] != DMX_JOINT_HINGE && d->jnt_type[j] != DMX_JOINT_SLIDE) {
      delete m;
      return fail(DMX_ERR_UNSUPPORTED, "tree joints must be hinge or slide");
    }
    if (b < 0 || b >= t.nb || (j > 0 && b < d->jnt_body[j - 1])) { delete m; return fail(DMX_ERR_INVALID_ARG, "joints must be grouped by body in body order"); }
    if (t.bjn[b] == 0) t.bj0[b] = j;
    t.bjn[b]++;
    t.jtype[j] = d->jnt_type[j];
    double n = 0.0;
    for (int i = 0; i < 3; ++i) n += d->jnt_axis[3 * j + i] * d->jnt_axis[3 * j + i];
    n = std::sqrt(n);
    for (int i = 0; i < 3; ++i) { t.jaxis[j][i] = d->jnt_axis[3 * j + i] / n; t.jpos[j][i] = d->jnt_pos[3 * j + i]; }
  }
  for (int b = 0; b < t.nb; ++b) {
    unsigned mask = 0u;
    for (int c = b; c >= 0; c = t.bparent[c])
      for (int j = t.bj0[c]; j < t.bj0[c] + t.bjn[c]; ++j) mask |= 1u << j;
    t.banc[b] = mask;
  }
  for (int i = 0; i < 3; ++i) t.grav[i] = d->gravity[i];
  for (int i = 0; i < d->nu; ++i) {
    if (d->ctrl_dof[i] < 0 || d->ctrl_dof[i] >= t.nj) { delete m; return fail(DMX_ERR_INVALID_ARG, "bad ctrl dof"); }
    t.ctrl[i] = d->ctrl_dof[i];
  }
  // translational inverse weights at the reference configuration q = 0:
  // w_b = trace(Jp_b M^-1 Jp_b^T) / 3
  const int nv = t.nj;
  double q0[dmx::kTreeJoints] = {0};
  double P[dmx::kTreeBodies][3], R[dmx::kTreeBodies][9], A[dmx::kTreeJoints][3], O[dmx::kTreeJoints][3];
  host_tree_fk(t, q0, P, R, A, O);
  std::vector<double> M(nv * nv, 0.0), Jall(t.nb * 3 * nv, 0.0);
  for (int b = 0; b < t.nb; ++b) {
    double Jp[3][dmx::kTreeJoints] = {{0}}, Jr[3][dmx::kTreeJoints] = {{0}};
    for (int dd = 0; dd < nv; ++dd) {
      if (!((t.banc[b] >> dd) & 1u)) continue;
      const double* a = A[dd];
      if (t.jtype[dd] == DMX_JOINT_HINGE) {
        const double r[3] = {P[b][0] - O[dd][0], P[b][1] - O[dd][1], P[b][2] - O[dd][2]};
        Jp[0][dd] = a[1] * r[2] - a[2] * r[1]; Jp[1][dd] = a[2] * r[0] - a[0] * r[2]; Jp[2][dd] = a[0] * r[1] - a[1] * r[0];
        for (int i = 0; i < 3; ++i) Jr[i][dd] = a[i];
      } else {
        for (int i = 0; i < 3; ++i) Jp[i][dd] = a[i];
      }
    }
    double Iw[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double acc = 0.0;
        for (int k = 0; k < 3; ++k)
          for (int l = 0; l < 3; ++l) acc += R[b][i * 3 + k] * t.bI[b][k * 3 + l] * R[b][j * 3 + l];
        Iw[i * 3 + j] = acc;
      }
    for (int i = 0; i < nv; ++i)
      for (int j = 0; j < nv; ++j) {
        double acc = 0.0;
        for (int r = 0; r < 3; ++r) acc += t.bmass[b] * Jp[r][i] * Jp[r][j];
        for (int r = 0; r < 3; ++r)
          for (int c = 0; c < 3; ++c) acc += Jr[r][i] * Iw[r * 3 + c] * Jr[c][j];
        M[i * nv + j] += acc;
      }
    for (int r = 0; r < 3; ++r)
      for (int i = 0; i < nv; ++i) Jall[(b * 3 + r) * nv + i] = Jp[r][i];
  }
  // Cholesky of M and the inverse weights
  std::vector<double> Lm = M;
  for (int j = 0; j < nv; ++j) {
    double sj = Lm[j * nv + j];
    for (int k = 0; k < j; ++k) sj -= Lm[j * nv + k] * Lm[j * nv + k];
    if (!(sj > 0.0)) { delete m; return fail(DMX_ERR_INVALID_ARG, "singular joint-space inertia"); }
    Lm[j * nv + j] = std::sqrt(sj);
    for (int i = j + 1; i < nv; ++i) {
      double v = Lm[i * nv + j];
      for (int k = 0; k < j; ++k) v -= Lm[i * nv + k] * Lm[j * nv + k];
      Lm[i * nv + j] = v / Lm[j * nv + j];
    }
  }
  double invw[dmx::kTreeBodies];
  for (int b = 0; b < t.nb; ++b) {
    double tr = 0.0;
    for (int r = 0; r < 3; ++r) {
      std::vector<double> x(Jall.begin() + (b * 3 + r) * nv, Jall.begin() + (b * 3 + r + 1) * nv);
      for (int i = 0; i < nv; ++i) { for (int k = 0; k < i; ++k) x[i] -= Lm[i * nv + k] * x[k]; x[i] /= Lm[i * nv + i]; }
      for (int i = nv - 1; i >= 0; --i) { for (int k = i + 1; k < nv; ++k) x[i] -= Lm[k * nv + i] * x[k]; x[i] /= Lm[i * nv + i]; }
      for (int i = 0; i < nv; ++i) tr += Jall[(b * 3 + r) * nv + i] * x[i];
    }
    invw[b] = tr / 3.0;
  }
  int nc = 0;
  t.np = d->npair;
  for (int p = 0; p < d->npair; ++p) {
    const int g1 = d->pair_g1[p], g2 = d->pair_g2[p];
    if (g1 < 0 || g1 >= d->ngeom || g2 < 0 || g2 >= d->ngeom || d->geom_type[g1] != DMX_GEOM_PLANE ||
        d->geom_body[g1] != -1 || d->geom_body[g2] < 0) {
      delete m;
      return fail(DMX_ERR_UNSUPPORTED, "pairs must be (world plane, body geom)");
    }
    const int t2 = d->geom_type[g2];
    if (t2 != DMX_GEOM_SPHERE && t2 != DMX_GEOM_CAPSULE) { delete m; return fail(DMX_ERR_UNSUPPORTED, "sphere/capsule pairs only"); }
    dmx::PairF& pr = t.pair[p];
    pr.gtype = t2;
    pr.ncon = (t2 == DMX_GEOM_CAPSULE) ? 2 : 1;
    t.pbody[p] = d->geom_body[g2];
    double Rg[9], Rp[9];
    quat_to_mat(&d->geom_quat[4 * g2], Rg);
    quat_to_mat(&d->geom_quat[4 * g1], Rp);
    for (int i = 0; i < 3; ++i) {
      pr.l[i] = d->geom_pos[3 * g2 + i];
      pr.ax[i] = Rg[i * 3 + 2] * d->geom_size[3 * g2 + 1];
      pr.p0[i] = d->geom_pos[3 * g1 + i];
      pr.n[i] = Rp[i * 3 + 2];
    }
    make_tangents(pr.n, pr.t1, pr.t2);
    pr.rad = d->geom_size[3 * g2];
    pr.mu = d->pair_mu[p];
    const double tc = d->pair_solref[2 * p], dr = d->pair_solref[2 * p + 1];
    for (int i = 0; i < 5; ++i) { pr.si[i] = d->pair_solimp[5 * p + i]; pr.cf[i] = d->pair_cfd[5 * p + i]; }
    spline_scales(pr);
    const double dw = pr.si[1];
    if (!contact_params_ok(tc, dr, pr)) {
      delete m;
      return fail(DMX_ERR_INVALID_ARG, "solref/solimp/cfd out of range");
    }
    pr.bcoef = 2.0 / (dw * tc);
    pr.kscale = 1.0 / (dw * dw * tc * tc * dr * dr);
    pr.ahat = (1.0 + pr.mu * pr.mu) * invw[t.pbody[p]];
    pr.solref[0] = tc;
    pr.solref[1] = dr;
    for (int c = 0; c < pr.ncon; ++c) {
      if (nc >= dmx::kMaxSlots) { delete m; return fail(DMX_ERR_UNSUPPORTED, "too many contact slots"); }
      t.cpair[nc] = p;
      t.csub[nc] = c;
      ++nc;
    }
  }
  t.nc = nc;
  m->nc = nc;
  m->ncb = bucket(nc > 0 ? nc : 1);
  hipError_t e = hipMalloc(&m->dev, sizeof(dmx::TreeModel));
  if (e == hipSuccess) e = hipMemcpy(m->dev, &t, sizeof(dmx::TreeModel), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    if (m->dev) (void)hipFree(m->dev);
    delete m;
    return fail(DMX_ERR_HIP, std::string("model upload: ") + hipGetErrorString(e));
  }
  *out = m;
  return DMX_OK;
}

dmx_status dmx_model_info(const dmx_model* m, int32_t* nq, int32_t* nv, int32_t* nu, int32_t* max_contacts) {
  if (!m) return fail(DMX_ERR_INVALID_ARG, "null model");
  if (nq) *nq = m->nq;
  if (nv) *nv = m->nv;
  if (nu) *nu = m->nu;
  if (max_contacts) *max_contacts = m->nc;
  return DMX_OK;
}

void dmx_model_destroy(dmx_model* m) {
  if (!m) return;
  if (m->dev) (void)hipFree(m->dev);
  if (m->stk_dev) (void)hipFree(m->stk_dev);
  delete m;
}

// every compiled kernel, in table order
static std::vector<const KernelEntry*> all_kernels() {
  std::vector<const KernelEntry*> v;
  for (KernelTable t : {free_kernels_small(), free_kernels(), free_kernels_wide(), tree_kernels()})
    for (int i = 0; i < t.n; ++i) v.push_back(&t.entries[i]);
  return v;
}

static const KernelEntry* lookup_kernel(const dmx_model* m, int team) {
  static const std::vector<const KernelEntry*> table = all_kernels();
  for (const KernelEntry* kp : table) {
    const KernelEntry& k = *kp;
    if (k.kind == m->kind && k.nc == m->ncb && k.team == team && (m->kind == 0 || (k.nv == m->nv && k.nb == m->nb)))
      return &k;
  }
  return nullptr;
}

// Kernel for a model and team size (lanes per world).  Default team: tree
// worlds keep their kinematic workspace in LDS and take 8 lanes; free bodies
// take two lanes per contact slot where such a team is compiled (each lane
// one tangent direction: the cube with 16 lanes, the box geom with 8),
// otherwise one slot per lane (up to 16).
static const KernelEntry* find_kernel(const dmx_model* m, int team) {
  if (team > 0) return lookup_kernel(m, team);
  if (const int t = m->tuned_team.load()) return lookup_kernel(m, t);
  if (m->kind == 1) {  // 8 lanes measured fastest on the legged chain (16384 worlds); 4 for small trees
    if (const KernelEntry* k = lookup_kernel(m, 8)) return k;
    return lookup_kernel(m, 4);
  }
  if (2 * m->ncb <= 16)
    if (const KernelEntry* k = lookup_kernel(m, 2 * m->ncb)) return k;
  return lookup_kernel(m, m->ncb >= 16 ? 16 : m->ncb);
}

static dmx::SolverOpts to_solver(const dmx_solver_opts& o) {
  dmx::SolverOpts s;
  s.rtol = o.rtol; s.atol = o.atol; s.h0 = o.h0; s.safety = o.safety; s.facmin = o.facmin; s.facmax = o.facmax;
  s.kP = o.kP; s.kI = o.kI; s.err_order = o.err_order; s.err_floor = o.err_floor; s.beta = o.softplus_beta;
  s.max_attempts = o.max_attempts; s.newton_maxit = o.newton_maxit; s.cfd = o.cfd; s.h_levels = o.h_levels;
  s.tableau = o.tableau;
  return s;
}

// Per-world layout of a batch of stack worlds: state offsets (13 k doubles
// per world), control offsets (n_int nu), tape offsets (cap records of 3 +
// 13 k (+ 36 k with stages) doubles), and the processing order (most cubes
// first, index order among equals: the longest worlds start first).
struct StackLayout {
  std::vector<dmx::StackModel> models;
  std::vector<long long> x_off, u_off, t_off;
  std::vector<int> cap, order, rec;
  long long nx = 0, nu = 0, tape_doubles = 0;
};

static void stack_layout(const std::vector<const dmx_model*>& ms, int n_int, long long cap, int stages, StackLayout* L) {
  const int W = (int)ms.size();
  L->models.resize(W); L->x_off.resize(W); L->u_off.resize(W); L->t_off.resize(W);
  L->cap.assign(W, (int)cap); L->order.resize(W); L->rec.resize(W);
  long long xo = 0, uo = 0, to = 0;
  for (int w = 0; w < W; ++w) {
    const dmx::StackModel& sm = ms[w]->stk;
    L->models[w] = sm;
    L->x_off[w] = xo; L->u_off[w] = uo; L->t_off[w] = to;
    L->rec[w] = 3 + 13 * sm.k + (stages ? 36 * sm.k : 0);
    xo += 13 * sm.k;
    uo += (long long)n_int * sm.nu;
    to += cap * L->rec[w];
    L->order[w] = w;
  }
  std::stable_sort(L->order.begin(), L->order.end(), [&](int a, int b) { return ms[a]->stk.k > ms[b]->stk.k; });
  L->nx = xo; L->nu = uo; L->tape_doubles = to;
}

// device tables of a stack batch: models, x_off, u_off, t_off, cap, order, queue[2]
static size_t stack_tables_bytes(int W) {
  return align256(sizeof(dmx::StackModel) * (size_t)W) + 3 * align256(sizeof(long long) * (size_t)W) +
         2 * align256(sizeof(int) * (size_t)W) + 256;
}
static dmx_status stack_tables_upload(const StackLayout& L, void* dev, hipStream_t s, dmx::StackArgs* a) {
  const int W = (int)L.models.size();
  std::vector<char> host(stack_tables_bytes(W), 0);
  size_t o = 0;
  auto put = [&](const void* src, size_t n) { size_t at = o; std::memcpy(host.data() + o, src, n); o += align256(n); return at; };
  const size_t om = put(L.models.data(), sizeof(dmx::StackModel) * W);
  const size_t ox = put(L.x_off.data(), sizeof(long long) * W);
  const size_t ou = put(L.u_off.data(), sizeof(long long) * W);
  const size_t ot = put(L.t_off.data(), sizeof(long long) * W);
  const size_t oc = put(L.cap.data(), sizeof(int) * W);
  const size_t oo = put(L.order.data(), sizeof(int) * W);
  const size_t oq = o;
  // the host buffer must outlive the copy: copy in stream order, then wait
  HIP_TRY(hipMemcpyAsync(dev, host.data(), host.size(), hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  char* D = (char*)dev;
  a->models = (const dmx::StackModel*)(D + om);
  a->x_off = (const long long*)(D + ox);
  a->u_off = (const long long*)(D + ou);
  a->t_off = (const long long*)(D + ot);
  a->cap_w = (const int*)(D + oc);
  a->order = (const int*)(D + oo);
  a->queue = (int*)(D + oq);
  return DMX_OK;
}

// Stack batches.  A batch of one model (uniform) needs no per-world tables:
// the kernels take the model and strides; otherwise the tables are uploaded
// (owned by the tape, or temporary).  With scratch_queue (no tape, uniform
// batches only) nothing is allocated: the work-queue counter lives there.
static dmx_status stack_rollout(const std::vector<const dmx_model*>& ms, int n_int, double dt,
                                const dmx_solver_opts& o, const double* x0, const double* u, double* x_out,
                                int32_t* world_status, int32_t* n_accepted, int32_t* n_rejected, dmx_tape** tape,
                                hipStream_t s, int* scratch_queue = nullptr, const double* x_out_bar = nullptr,
                                double* x0_bar = nullptr, double* u_bar = nullptr) {
  const int W = (int)ms.size();
  bool uniform = true;
  for (const dmx_model* m : ms) uniform = uniform && m == ms[0];
  if (o.launch_mode != 0 && o.launch_mode != 1) return fail(DMX_ERR_INVALID_ARG, "bad launch_mode");
  if (o.world_intervals) return fail(DMX_ERR_UNSUPPORTED, "ragged horizons are not taken by stack batches");
  if (o.tableau != 0) return fail(DMX_ERR_UNSUPPORTED, "stack batches take the Dormand-Prince pair");
  bool any_ctrl = false;
  for (const dmx_model* m : ms) any_ctrl = any_ctrl || m->nu > 0;
  if (any_ctrl && !u) return fail(DMX_ERR_INVALID_ARG, "controls required");
  dmx_tape* reuse = tape ? *tape : nullptr;
  if (reuse) {
    const long long want = o.tape_steps > 0 ? o.tape_steps : reuse->cap;
    if (!reuse->stack || reuse->models != ms || reuse->cap < want)
      return fail(DMX_ERR_INVALID_ARG, "tape to reuse does not match the batch's models/capacity");
  }
  dmx::StackArgs a{};
  a.W = W; a.n_int = n_int; a.dt = dt; a.x0 = x0; a.u = u; a.xout = x_out;
  a.status = world_status; a.n_acc = n_accepted; a.n_rej = n_rejected;
  a.counters = (long long*)o.fwd_counters;
  a.forced = o.forced; a.forced_n = o.forced_n; a.forced_cap = o.forced_cap;
  a.steplog = o.steplog; a.log_n = o.log_n; a.log_cap = o.log_cap;
  a.o = to_solver(o);
  const bool use_queue = o.launch_mode == 0 && o.work_queue != -1;
  if (tape) {
    dmx_tape* tp = reuse;
    if (!tp) {
      tp = new dmx_tape();
      tp->stack = true;
      tp->models = ms;
      tp->W = W; tp->n_int = n_int; tp->dt = dt; tp->u = u;
      tp->cap = o.tape_steps > 0 ? o.tape_steps : 4096;
      StackLayout L0;
      stack_layout(ms, n_int, tp->cap, 1, &L0);
      bool stages = o.tape_stages != 0;
      if (o.tape_stages < 0) {
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) == hipSuccess)
          stages = (double)L0.tape_doubles * sizeof(double) <= 0.5 * (double)free_b;
      }
      StackLayout L;
      stack_layout(ms, n_int, tp->cap, stages ? 1 : 0, &L);
      tp->rec = L.rec[0];  // record length of world 0 (of every world when the models are equal)
      tp->t_off_h = L.t_off;
      tp->rec_h = L.rec;
      tp->stk_tables_bytes = stack_tables_bytes(W);
      hipError_t e = hipMalloc(&tp->records, sizeof(double) * (size_t)std::max(L.tape_doubles, 1ll));
      if (e == hipSuccess) e = hipMalloc(&tp->n_acc, sizeof(int) * W);
      if (e == hipSuccess) e = hipMalloc(&tp->status, sizeof(int) * W);
      if (e == hipSuccess) e = hipMalloc(&tp->stk_tables, tp->stk_tables_bytes);
      if (e != hipSuccess) {
        dmx_tape_destroy(tp);
        return fail(DMX_ERR_OUT_OF_MEMORY, std::string("tape allocation: ") + hipGetErrorString(e));
      }
      if (uniform) {
        tp->sa.uniform = 1;
        tp->sa.models = (const dmx::StackModel*)ms[0]->stk_dev;
        tp->sa.x_stride = 13 * ms[0]->stk.k;
        tp->sa.u_stride = (long long)n_int * ms[0]->stk.nu;
        tp->sa.t_stride = tp->cap * L.rec[0];
        tp->sa.cap_uniform = (int)tp->cap;
        tp->sa.queue = (int*)((char*)tp->stk_tables + (tp->stk_tables_bytes - 256));
      } else {
        const dmx_status r = stack_tables_upload(L, tp->stk_tables, s, &tp->sa);
        if (r != DMX_OK) { dmx_tape_destroy(tp); return r; }
      }
      tp->sa.stages = stages ? 1 : 0;
      tp->model = ms[0];
    }
    tp->n_int = n_int; tp->dt = dt; tp->u = u;
    tp->plain = o.launch_mode;
    tp->adj_counters = o.adj_counters;
    tp->use_queue = use_queue;
    a.models = tp->sa.models; a.x_off = tp->sa.x_off; a.u_off = tp->sa.u_off; a.t_off = tp->sa.t_off;
    a.cap_w = tp->sa.cap_w; a.order = tp->sa.order; a.stages = tp->sa.stages;
    a.uniform = tp->sa.uniform; a.x_stride = tp->sa.x_stride; a.u_stride = tp->sa.u_stride;
    a.t_stride = tp->sa.t_stride; a.cap_uniform = tp->sa.cap_uniform;
    a.queue = use_queue ? tp->sa.queue : nullptr;
    a.tape = tp->records; a.n_acc = tp->n_acc; a.status = tp->status;
    if (x_out_bar) {  // each world's reverse sweep right after its forward rollout
      a.xbar = x_out_bar; a.x0bar = x0_bar; a.ubar = u_bar;
      a.adj_counters = (long long*)o.adj_counters;
      dmx_host::stack_grad(a, s, o.launch_mode);
      a.xbar = nullptr; a.x0bar = nullptr; a.ubar = nullptr; a.adj_counters = nullptr;
    } else {
      dmx_host::stack_fwd(a, s, o.launch_mode);
    }
    HIP_TRY(hipGetLastError());
    tp->sa = a;
    tp->sa.queue = use_queue ? (int*)((char*)tp->stk_tables + (tp->stk_tables_bytes - 256)) : nullptr;
    HIP_TRY(hipMemcpyAsync(world_status, tp->status, sizeof(int) * W, hipMemcpyDeviceToDevice, s));
    if (n_accepted) HIP_TRY(hipMemcpyAsync(n_accepted, tp->n_acc, sizeof(int) * W, hipMemcpyDeviceToDevice, s));
    *tape = tp;
    return DMX_OK;
  }
  if (uniform) {
    a.uniform = 1;
    a.models = (const dmx::StackModel*)ms[0]->stk_dev;
    a.x_stride = 13 * ms[0]->stk.k;
    a.u_stride = (long long)n_int * ms[0]->stk.nu;
    int* q = scratch_queue;
    if (use_queue && !q) HIP_TRY(hipMallocAsync((void**)&q, sizeof(int), s));
    a.queue = use_queue ? q : nullptr;
    dmx_host::stack_fwd(a, s, o.launch_mode);
    HIP_TRY(hipGetLastError());
    if (use_queue && !scratch_queue) HIP_TRY(hipFreeAsync(q, s));
    return DMX_OK;
  }
  if (scratch_queue) return fail(DMX_ERR_INVALID_ARG, "allocation-free rollouts take one model");
  StackLayout L;
  stack_layout(ms, n_int, 0, 0, &L);
  void* tbl = nullptr;
  HIP_TRY(hipMallocAsync(&tbl, stack_tables_bytes(W), s));
  const dmx_status r = stack_tables_upload(L, tbl, s, &a);
  if (r != DMX_OK) { (void)hipFreeAsync(tbl, s); return r; }
  if (!use_queue) a.queue = nullptr;
  a.cap_w = nullptr;
  dmx_host::stack_fwd(a, s, o.launch_mode);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipFreeAsync(tbl, s));
  return DMX_OK;
}

static dmx_status check_opts(const dmx_solver_opts& o) {
  if (!(o.rtol >= 0.0) || !(o.atol > 0.0) || !(o.h0 > 0.0) || o.newton_maxit <= 0 || o.h_levels < 0)
    return fail(DMX_ERR_INVALID_ARG, "bad solver options");
  if (o.forced && (!o.forced_n || o.forced_cap <= 0)) return fail(DMX_ERR_INVALID_ARG, "forced steps need counts");
  if (o.steplog && (!o.log_n || o.log_cap <= 0)) return fail(DMX_ERR_INVALID_ARG, "step log needs counts");
  if (o.work_queue < -1 || o.work_queue > 1) return fail(DMX_ERR_INVALID_ARG, "bad work_queue");
  if (o.tableau < 0 || o.tableau > 1) return fail(DMX_ERR_INVALID_ARG, "bad tableau");
  return DMX_OK;
}

dmx_status dmx_batch_layout(const dmx_batch* b, int64_t* x_off, int64_t* u_off, int64_t* nx_total,
                            int64_t* nu_total) {
  if (!b || (b->n_worlds > 0 && !b->models)) return fail(DMX_ERR_INVALID_ARG, "null argument");
  int64_t xo = 0, uo = 0;
  for (int w = 0; w < b->n_worlds; ++w) {
    const dmx_model* m = b->models[w];
    if (!m) return fail(DMX_ERR_INVALID_ARG, "null model in batch");
    if (x_off) x_off[w] = xo;
    if (u_off) u_off[w] = uo;
    xo += m->nq + m->nv;
    uo += (int64_t)b->n_intervals * m->nu;
  }
  if (nx_total) *nx_total = xo;
  if (nu_total) *nu_total = uo;
  return DMX_OK;
}

dmx_status dmx_rollout_batch(const dmx_batch* b, const dmx_solver_opts* opts, const double* x0, const double* u,
                             double* x_out, int32_t* world_status, int32_t* n_accepted, int32_t* n_rejected,
                             dmx_tape** tape, void* stream) {
  if (!b || (b->n_worlds > 0 && !b->models)) return fail(DMX_ERR_INVALID_ARG, "null argument");
  if (b->n_worlds < 0 || b->n_intervals <= 0 || !(b->interval_dt > 0.0)) return fail(DMX_ERR_INVALID_ARG, "bad batch sizes");
  dmx_solver_opts o;
  if (opts) o = *opts; else dmx_default_opts(&o);
  const dmx_status oc = check_opts(o);
  if (oc != DMX_OK) return oc;
  if (b->n_worlds == 0) { if (tape && !*tape) *tape = nullptr; return DMX_OK; }
  if (!x0 || !x_out || !world_status) return fail(DMX_ERR_INVALID_ARG, "null argument");
  std::vector<const dmx_model*> ms(b->models, b->models + b->n_worlds);
  for (const dmx_model* m : ms) {
    if (!m) return fail(DMX_ERR_INVALID_ARG, "null model in batch");
    if (!m->stack_ok) return fail(DMX_ERR_UNSUPPORTED, "batches of mixed models take stacks of cubes (k >= 1)");
  }
  return stack_rollout(ms, b->n_intervals, b->interval_dt, o, x0, u, x_out, world_status, n_accepted, n_rejected,
                       tape, (hipStream_t)stream);
}

dmx_status dmx_rollout_batch_grad(const dmx_batch* b, const dmx_solver_opts* opts, const double* x0,
                                  const double* u, const double* x_out_bar, double* x_out, int32_t* world_status,
                                  int32_t* n_accepted, int32_t* n_rejected, double* x0_bar, double* u_bar,
                                  dmx_tape** tape, void* stream) {
  if (!b || (b->n_worlds > 0 && !b->models) || !tape) return fail(DMX_ERR_INVALID_ARG, "null argument");
  if (b->n_worlds < 0 || b->n_intervals <= 0 || !(b->interval_dt > 0.0)) return fail(DMX_ERR_INVALID_ARG, "bad batch sizes");
  dmx_solver_opts o;
  if (opts) o = *opts; else dmx_default_opts(&o);
  const dmx_status oc = check_opts(o);
  if (oc != DMX_OK) return oc;
  if (b->n_worlds == 0) { if (!*tape) *tape = nullptr; return DMX_OK; }
  if (!x0 || !x_out || !world_status || !x_out_bar || !x0_bar) return fail(DMX_ERR_INVALID_ARG, "null argument");
  std::vector<const dmx_model*> ms(b->models, b->models + b->n_worlds);
  bool any_ctrl = false;
  for (const dmx_model* m : ms) {
    if (!m) return fail(DMX_ERR_INVALID_ARG, "null model in batch");
    if (!m->stack_ok) return fail(DMX_ERR_UNSUPPORTED, "batches of mixed models take stacks of cubes (k >= 1)");
    any_ctrl = any_ctrl || m->nu > 0;
  }
  if (any_ctrl && !u_bar) return fail(DMX_ERR_INVALID_ARG, "u_bar required");
  return stack_rollout(ms, b->n_intervals, b->interval_dt, o, x0, u, x_out, world_status, n_accepted, n_rejected,
                       tape, (hipStream_t)stream, nullptr, x_out_bar, x0_bar, u_bar);
}

dmx_status dmx_tape_layout(const dmx_tape* tp, int64_t* t_off, int32_t* rec) {
  if (!tp) return fail(DMX_ERR_INVALID_ARG, "null tape");
  for (int w = 0; w < tp->W; ++w) {
    if (tp->stack) {
      if (t_off) t_off[w] = tp->t_off_h[w];
      if (rec) rec[w] = tp->rec_h[w];
    } else {
      if (t_off) t_off[w] = (int64_t)w * tp->cap * tp->rec;
      if (rec) rec[w] = tp->rec;
    }
  }
  return DMX_OK;
}

static dmx_status rollout_impl(const dmx_model* m, int32_t W, int32_t n_int, double dt,
                               const dmx_solver_opts* opts, const double* x0, const double* u, double* x_out,
                               int32_t* world_status, int32_t* n_accepted, int32_t* n_rejected, dmx_tape** tape,
                               void* stream, int* scratch_queue);

dmx_status dmx_rollout(const dmx_model* m, int32_t W, int32_t n_int, double dt, const dmx_solver_opts* opts,
                       const double* x0, const double* u, double* x_out, int32_t* world_status,
                       int32_t* n_accepted, int32_t* n_rejected, dmx_tape** tape, void* stream) {
  return rollout_impl(m, W, n_int, dt, opts, x0, u, x_out, world_status, n_accepted, n_rejected, tape, stream,
                      nullptr);
}

}  // extern "C"

// Scratch memory of the allocation-free entry point: the work-queue counter
// of a persistent launch.  A file-scope device array, one per GPU for the
// life of the process; host code uses its device address from
// hipGetSymbolAddress (taken once per device), never the array's name.
constexpr size_t kScratchBytes = 256;
static __device__ __align__(256) int scratch[kScratchBytes / sizeof(int)];

static dmx_status scratch_address(int** out) {
  static std::mutex mu;
  static std::vector<int*> per_device;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(mu);
  if ((int)per_device.size() <= dev) per_device.resize(dev + 1, nullptr);
  if (!per_device[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return fail(DMX_ERR_HIP, std::string("scratch address: ") + hipGetErrorString(e));
    per_device[dev] = (int*)p;
  }
  *out = per_device[dev];
  return DMX_OK;
}

extern "C" {

dmx_status dmx_rollout_noalloc(const dmx_model* m, int32_t W, int32_t n_int, double dt, const dmx_solver_opts* opts,
                               const double* x0, const double* u, double* x_out, int32_t* world_status,
                               int32_t* n_accepted, int32_t* n_rejected, void* stream) {
  int* q = nullptr;
  const dmx_status r = scratch_address(&q);
  if (r != DMX_OK) return r;
  return rollout_impl(m, W, n_int, dt, opts, x0, u, x_out, world_status, n_accepted, n_rejected, nullptr, stream, q);
}

}  // extern "C"

static dmx_status rollout_impl(const dmx_model* m, int32_t W, int32_t n_int, double dt,
                               const dmx_solver_opts* opts, const double* x0, const double* u, double* x_out,
                               int32_t* world_status, int32_t* n_accepted, int32_t* n_rejected, dmx_tape** tape,
                               void* stream, int* scratch_queue) {
  if (!m) return fail(DMX_ERR_INVALID_ARG, "null model");
  if (m->kind == 2) {
    if (W < 0 || n_int <= 0 || !(dt > 0.0)) return fail(DMX_ERR_INVALID_ARG, "bad batch sizes");
    dmx_solver_opts o;
    if (opts) o = *opts; else dmx_default_opts(&o);
    const dmx_status oc = check_opts(o);
    if (oc != DMX_OK) return oc;
    if (W == 0) { if (tape && !*tape) *tape = nullptr; return DMX_OK; }
    if (!x0 || !x_out || !world_status) return fail(DMX_ERR_INVALID_ARG, "null argument");
    std::vector<const dmx_model*> ms((size_t)W, m);
    return stack_rollout(ms, n_int, dt, o, x0, u, x_out, world_status, n_accepted, n_rejected, tape,
                         (hipStream_t)stream, scratch_queue);
  }
  if (W < 0 || n_int <= 0 || !(dt > 0.0)) return fail(DMX_ERR_INVALID_ARG, "bad batch sizes");
  if (W > 0 && (!x0 || !x_out || !world_status)) return fail(DMX_ERR_INVALID_ARG, "null argument");
  if (W > 0 && m->nu > 0 && !u) return fail(DMX_ERR_INVALID_ARG, "controls required");
  dmx_solver_opts o;
  if (opts) o = *opts; else dmx_default_opts(&o);
  const dmx_status oc = check_opts(o);
  if (oc != DMX_OK) return oc;
  const KernelEntry* k = find_kernel(m, o.lanes_per_world);
  if (!k) return fail(DMX_ERR_UNSUPPORTED, "no kernel for this model and lanes_per_world");
  dmx_tape* reuse = tape ? *tape : nullptr;
  if (reuse) {
    const long long want = o.tape_steps > 0 ? o.tape_steps : reuse->cap;
    if (reuse->model != m || reuse->W != W || reuse->cap < want)
      return fail(DMX_ERR_INVALID_ARG, "tape to reuse does not match model/n_worlds/capacity");
  }
  if (W == 0) { if (tape && !reuse) *tape = nullptr; return DMX_OK; }
  hipStream_t s = (hipStream_t)stream;
  const int NX = m->nq + m->nv;
  dmx::FwdArgs a{};
  if (o.launch_mode != 0 && o.launch_mode != 1) return fail(DMX_ERR_INVALID_ARG, "bad launch_mode");
  if (o.work_queue < -1 || o.work_queue > 1) return fail(DMX_ERR_INVALID_ARG, "bad work_queue");
  if (o.launch_mode == 1 && (o.world_intervals || o.world_order || o.work_queue == 1))
    return fail(DMX_ERR_INVALID_ARG, "the plain launch form takes uniform batches without a work queue");
  const bool use_queue = o.launch_mode == 0 && (o.work_queue == 1 || (o.work_queue == 0 &&
                         (o.world_intervals != nullptr || (long long)W > k->resident())));
  a.W = W; a.n_int = n_int; a.nu = m->nu; a.dt = dt; a.x0 = x0; a.u = u; a.xout = x_out;
  a.counters = (long long*)o.fwd_counters;
  a.fail_state = o.fail_state;
  a.status = world_status; a.n_acc = n_accepted; a.n_rej = n_rejected; a.n_newton = nullptr;
  a.forced = o.forced; a.forced_n = o.forced_n; a.forced_cap = o.forced_cap;
  a.steplog = o.steplog; a.log_n = o.log_n; a.log_cap = o.log_cap;
  a.g.n_int_w = o.world_intervals; a.g.order = o.world_order;
  a.o = to_solver(o);
  dmx_tape* tp = nullptr;
  int* tmp_queue = nullptr;
  if (reuse) {
    tp = reuse;
    tp->n_int = n_int; tp->dt = dt; tp->u = u; tp->o = a.o; tp->adj = k->adj; tp->otd = k->otd; tp->team = k->team;
    tp->adj_counters = o.adj_counters; tp->plain = o.launch_mode;
    a.tape = tp->records; a.cap = tp->cap; a.rec = tp->rec;
    a.n_acc = tp->n_acc; a.status = tp->status;
  } else if (tape) {
    tp = new dmx_tape();
    tp->model = m; tp->W = W; tp->n_int = n_int; tp->nu = m->nu; tp->dt = dt; tp->u = u;
    tp->cap = o.tape_steps > 0 ? o.tape_steps : 4096;
    // stage accelerations on the tape unless asked otherwise or, by default,
    // unless the full tape would take more than half the free device memory
    // (then checkpoints only: the reverse sweep solves the stages again)
    bool stages = o.tape_stages != 0;
    if (o.tape_stages < 0) {
      size_t free_b = 0, total_b = 0;
      if (hipMemGetInfo(&free_b, &total_b) == hipSuccess)
        stages = (double)W * tp->cap * (3 + NX + 6 * m->nv) * sizeof(double) <= 0.5 * (double)free_b;
    }
    tp->rec = 3 + NX + (stages ? 6 * m->nv : 0);
    tp->o = a.o;
    tp->adj = k->adj;
    tp->otd = k->otd;
    tp->team = k->team;
    tp->adj_counters = o.adj_counters;
    tp->plain = o.launch_mode;
    const size_t bytes = (size_t)W * tp->cap * tp->rec * sizeof(double);
    hipError_t e = hipMalloc(&tp->records, bytes);
    if (e == hipSuccess) e = hipMalloc(&tp->n_acc, sizeof(int) * W);
    if (e == hipSuccess) e = hipMalloc(&tp->status, sizeof(int) * W);
    if (e == hipSuccess) e = hipMalloc(&tp->queue, 2 * sizeof(int));
    if (e == hipSuccess) e = hipMalloc(&tp->tables, 2 * sizeof(int) * W);
    if (e != hipSuccess) {
      dmx_tape_destroy(tp);
      return fail(DMX_ERR_OUT_OF_MEMORY, std::string("tape allocation: ") + hipGetErrorString(e));
    }
    a.tape = tp->records; a.cap = tp->cap; a.rec = tp->rec;
    a.n_acc = tp->n_acc; a.status = tp->status;
  }
  if (tp) {
    // the reverse sweep reads the per-world tables later: the tape keeps its
    // own copies, so the caller's arrays need only live until this call's
    // work on the stream is done
    tp->world_intervals = nullptr;
    tp->world_order = nullptr;
    if (o.world_intervals) {
      HIP_TRY(hipMemcpyAsync(tp->tables, o.world_intervals, sizeof(int) * W, hipMemcpyDeviceToDevice, s));
      tp->world_intervals = tp->tables;
    }
    if (o.world_order) {
      HIP_TRY(hipMemcpyAsync(tp->tables + W, o.world_order, sizeof(int) * W, hipMemcpyDeviceToDevice, s));
      tp->world_order = tp->tables + W;
    }
    a.g.n_int_w = tp->world_intervals; a.g.order = tp->world_order;
    tp->use_queue = use_queue;
    if (use_queue) a.g.queue = tp->queue;
  } else if (use_queue) {
    if (scratch_queue) {
      a.g.queue = scratch_queue;
    } else {
      HIP_TRY(hipMallocAsync((void**)&tmp_queue, sizeof(int), s));
      a.g.queue = tmp_queue;
    }
  }
  k->fwd(m->dev, a, s, o.launch_mode);
  HIP_TRY(hipGetLastError());
  if (tmp_queue) HIP_TRY(hipFreeAsync(tmp_queue, s));
  if (tp) {
    HIP_TRY(hipMemcpyAsync(world_status, tp->status, sizeof(int) * W, hipMemcpyDeviceToDevice, s));
    if (n_accepted) HIP_TRY(hipMemcpyAsync(n_accepted, tp->n_acc, sizeof(int) * W, hipMemcpyDeviceToDevice, s));
    *tape = tp;
  }
  return DMX_OK;
}

extern "C" {

dmx_status dmx_accel(const dmx_model* m, int32_t n, const double* x, const double* tau, int32_t cfd, double* acc,
                     int32_t* status, void* stream) {
  if (!m) return fail(DMX_ERR_INVALID_ARG, "null model");
  if (n < 0) return fail(DMX_ERR_INVALID_ARG, "bad count");
  if (n == 0) return DMX_OK;
  if (!x || !acc || !status) return fail(DMX_ERR_INVALID_ARG, "null argument");
  if (m->kind == 2) {
    dmx_solver_opts oo;
    dmx_default_opts(&oo);
    dmx_host::stack_accel((const dmx::StackModel*)m->stk_dev, n, x, tau, cfd, to_solver(oo), acc, status,
                          (hipStream_t)stream);
    HIP_TRY(hipGetLastError());
    return DMX_OK;
  }
  const KernelEntry* k = find_kernel(m, 0);
  if (!k) return fail(DMX_ERR_UNSUPPORTED, "no kernel for this model");
  dmx_solver_opts oo;
  dmx_default_opts(&oo);
  k->acc(m->dev, n, x, tau, cfd, to_solver(oo), acc, status, (hipStream_t)stream);
  HIP_TRY(hipGetLastError());
  return DMX_OK;
}

dmx_status dmx_autotune(dmx_model* m, int32_t W, int32_t n_int, double dt, const double* x0, const double* u,
                        void* stream, int32_t* best_lanes, int32_t* n_tried, int32_t* lanes_tried, double* ms_tried) {
  if (!m || !x0 || !best_lanes) return fail(DMX_ERR_INVALID_ARG, "null argument");
  if (W <= 0 || n_int <= 0 || !(dt > 0.0)) return fail(DMX_ERR_INVALID_ARG, "bad batch sizes");
  if (m->nu > 0 && !u) return fail(DMX_ERR_INVALID_ARG, "controls required");
  hipStream_t s = (hipStream_t)stream;
  const int NX = m->nq + m->nv;
  double* xo = nullptr;
  int* st = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMalloc(&xo, sizeof(double) * (size_t)W * NX);
  if (e == hipSuccess) e = hipMalloc(&st, sizeof(int) * (size_t)W);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  auto cleanup = [&]() {
    if (xo) (void)hipFree(xo);
    if (st) (void)hipFree(st);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  if (e != hipSuccess) { cleanup(); return fail(DMX_ERR_OUT_OF_MEMORY, "autotune buffers"); }
  int best = 0, tried = 0;
  float best_ms = 0.0f;
  for (const KernelEntry* kp : all_kernels()) {
    const KernelEntry& k = *kp;
    if (k.kind != m->kind || k.nc != m->ncb || (m->kind == 1 && (k.nv != m->nv || k.nb != m->nb))) continue;
    dmx_solver_opts o;
    dmx_default_opts(&o);
    o.lanes_per_world = k.team;
    float ms = 0.0f;
    for (int rep = 0; rep < 2; ++rep) {  // the first run loads the code object
      if (hipEventRecord(e0, s) != hipSuccess) { cleanup(); return fail(DMX_ERR_HIP, "event record"); }
      const dmx_status r = dmx_rollout(m, W, n_int, dt, &o, x0, u, xo, st, nullptr, nullptr, nullptr, stream);
      if (r != DMX_OK) { cleanup(); return r; }
      if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        cleanup();
        return fail(DMX_ERR_HIP, "autotune timing");
      }
    }
    if (lanes_tried && tried < 8) lanes_tried[tried] = k.team;
    if (ms_tried && tried < 8) ms_tried[tried] = ms;
    ++tried;
    // a wider team must be at least 2% faster to be chosen (timing noise)
    if (best == 0 || ms < 0.98f * best_ms) { best = k.team; best_ms = ms; }
  }
  cleanup();
  if (!best) return fail(DMX_ERR_UNSUPPORTED, "no kernel for this model");
  m->tuned_team.store(best);
  *best_lanes = best;
  if (n_tried) *n_tried = tried;
  return DMX_OK;
}

// reverse sweep of a stack batch's tape (with the model parameters'
// cotangents into param_bar when given)
static dmx_status stack_vjp(dmx_tape* tp, const double* x_out_bar, double* x0_bar, double* u_bar,
                            double* param_bar, void* stream) {
  bool any_ctrl = false;
  for (const dmx_model* m : tp->models) any_ctrl = any_ctrl || m->nu > 0;
  if (any_ctrl && !u_bar) return fail(DMX_ERR_INVALID_ARG, "u_bar required");
  dmx::StackArgs a = tp->sa;
  a.u = tp->u;
  a.xbar = x_out_bar; a.x0bar = x0_bar; a.ubar = u_bar;
  a.adj_counters = (long long*)tp->adj_counters;
  a.counters = nullptr; a.steplog = nullptr; a.log_n = nullptr; a.forced = nullptr;
  a.queue = tp->use_queue ? tp->sa.queue + 1 : nullptr;
  a.pbar = param_bar;
  if (param_bar) dmx_host::stack_adj_params(a, (hipStream_t)stream, tp->plain);
  else dmx_host::stack_adj(a, (hipStream_t)stream, tp->plain);
  HIP_TRY(hipGetLastError());
  return DMX_OK;
}

dmx_status dmx_rollout_vjp(dmx_tape* tp, const double* x_out_bar, double* x0_bar, double* u_bar, void* stream) {
  if (!tp || !x_out_bar || !x0_bar) return fail(DMX_ERR_INVALID_ARG, "null argument");
  if (tp->stack) return stack_vjp(tp, x_out_bar, x0_bar, u_bar, nullptr, stream);
  if (tp->nu > 0 && !u_bar) return fail(DMX_ERR_INVALID_ARG, "u_bar required");
  dmx::AdjArgs a{};
  a.W = tp->W; a.n_int = tp->n_int; a.nu = tp->nu; a.tape = tp->records; a.cap = tp->cap; a.rec = tp->rec;
  a.n_acc = tp->n_acc; a.status = tp->status; a.u = tp->u; a.xbar = x_out_bar; a.x0bar = x0_bar; a.ubar = u_bar;
  a.o = tp->o;
  a.counters = (long long*)tp->adj_counters;
  a.g.n_int_w = tp->world_intervals; a.g.order = tp->world_order;
  a.g.queue = tp->use_queue ? tp->queue + 1 : nullptr;
  tp->adj(tp->model->dev, a, (hipStream_t)stream, tp->plain);
  HIP_TRY(hipGetLastError());
  return DMX_OK;
}

static dmx_status otd_impl(dmx_tape* tp, const double* x_out_bar, double* x0_bar, double* u_bar,
                           double* param_bar, int npar, void* stream);

dmx_status dmx_rollout_vjp_otd(dmx_tape* tp, const double* x_out_bar, double* x0_bar, double* u_bar, void* stream) {
  return otd_impl(tp, x_out_bar, x0_bar, u_bar, nullptr, 0, stream);
}

dmx_status dmx_rollout_vjp_otd_geom(dmx_tape* tp, const double* x_out_bar, double* x0_bar, double* u_bar,
                                    double* geom_size_bar, void* stream) {
  if (!geom_size_bar) return fail(DMX_ERR_INVALID_ARG, "null argument");
  if (tp && (tp->stack || tp->model->kind != 0 || tp->model->box_geom < 0))
    return fail(DMX_ERR_UNSUPPORTED, "geom size gradients take single free bodies with one box geom");
  return otd_impl(tp, x_out_bar, x0_bar, u_bar, geom_size_bar, 3, stream);
}

dmx_status dmx_rollout_vjp_otd_params(dmx_tape* tp, const double* x_out_bar, double* x0_bar, double* u_bar,
                                      double* param_bar, void* stream) {
  if (!param_bar) return fail(DMX_ERR_INVALID_ARG, "null argument");
  if (tp && tp->stack)
    return fail(DMX_ERR_UNSUPPORTED, "the optimize-then-discretize adjoint takes free-body and tree models");
  return otd_impl(tp, x_out_bar, x0_bar, u_bar, param_bar, dmx::kParams, stream);
}

static dmx_status otd_impl(dmx_tape* tp, const double* x_out_bar, double* x0_bar, double* u_bar,
                           double* param_bar, int npar, void* stream) {
  if (!tp || !x_out_bar || !x0_bar) return fail(DMX_ERR_INVALID_ARG, "null argument");
  if (tp->stack || !tp->otd)
    return fail(DMX_ERR_UNSUPPORTED, "the optimize-then-discretize adjoint takes free-body and tree models");
  if (tp->nu > 0 && !u_bar) return fail(DMX_ERR_INVALID_ARG, "u_bar required");
  if (tp->o.tableau != 0)
    return fail(DMX_ERR_UNSUPPORTED, "the optimize-then-discretize adjoint reads the Dormand-Prince continuous extension");
  const int nx = tp->model->nq + tp->model->nv;
  if (tp->rec < 3 + nx + 6 * tp->model->nv)
    return fail(DMX_ERR_UNSUPPORTED, "the optimize-then-discretize adjoint needs a tape with stage accelerations");
  dmx::AdjArgs a{};
  a.W = tp->W; a.n_int = tp->n_int; a.nu = tp->nu; a.dt = tp->dt; a.tape = tp->records; a.cap = tp->cap;
  a.rec = tp->rec; a.n_acc = tp->n_acc; a.status = tp->status; a.u = tp->u; a.xbar = x_out_bar; a.x0bar = x0_bar;
  a.ubar = u_bar; a.hbar = param_bar; a.npar = npar;
  a.o = tp->o;
  a.counters = (long long*)tp->adj_counters;
  a.g.n_int_w = tp->world_intervals; a.g.order = tp->world_order;
  a.g.queue = tp->use_queue ? tp->queue + 1 : nullptr;
  tp->otd(tp->model->dev, a, (hipStream_t)stream, tp->plain);
  HIP_TRY(hipGetLastError());
  return DMX_OK;
}

static dmx_status params_impl(dmx_tape* tp, const double* x_out_bar, double* x0_bar, double* u_bar,
                              double* param_bar, int npar, void* stream);

dmx_status dmx_rollout_vjp_geom(dmx_tape* tp, const double* x_out_bar, double* x0_bar, double* u_bar,
                                double* geom_size_bar, void* stream) {
  if (!tp || !x_out_bar || !x0_bar || !geom_size_bar) return fail(DMX_ERR_INVALID_ARG, "null argument");
  if (tp->stack || tp->model->kind != 0 || tp->model->box_geom < 0)
    return fail(DMX_ERR_UNSUPPORTED, "geom size gradients take single free bodies with one box geom");
  return params_impl(tp, x_out_bar, x0_bar, u_bar, geom_size_bar, 3, stream);
}

dmx_status dmx_rollout_vjp_params(dmx_tape* tp, const double* x_out_bar, double* x0_bar, double* u_bar,
                                  double* param_bar, void* stream) {
  if (!tp || !x_out_bar || !x0_bar || !param_bar) return fail(DMX_ERR_INVALID_ARG, "null argument");
  if (tp->stack) return stack_vjp(tp, x_out_bar, x0_bar, u_bar, param_bar, stream);
  return params_impl(tp, x_out_bar, x0_bar, u_bar, param_bar, dmx::kParams, stream);
}

static dmx_status params_impl(dmx_tape* tp, const double* x_out_bar, double* x0_bar, double* u_bar,
                              double* param_bar, int npar, void* stream) {
  if (tp->nu > 0 && !u_bar) return fail(DMX_ERR_INVALID_ARG, "u_bar required");
  dmx::AdjArgs a{};
  a.W = tp->W; a.n_int = tp->n_int; a.nu = tp->nu; a.dt = tp->dt; a.tape = tp->records; a.cap = tp->cap;
  a.rec = tp->rec; a.n_acc = tp->n_acc; a.status = tp->status; a.u = tp->u; a.xbar = x_out_bar; a.x0bar = x0_bar;
  a.ubar = u_bar; a.hbar = param_bar; a.npar = npar;
  a.o = tp->o;
  a.counters = (long long*)tp->adj_counters;
  a.g.n_int_w = tp->world_intervals; a.g.order = tp->world_order;
  a.g.queue = tp->use_queue ? tp->queue + 1 : nullptr;
  tp->adj(tp->model->dev, a, (hipStream_t)stream, tp->plain);
  HIP_TRY(hipGetLastError());
  return DMX_OK;
}

dmx_status dmx_tape_info(const dmx_tape* tp, int64_t* steps, int32_t* rec) {
  if (!tp) return fail(DMX_ERR_INVALID_ARG, "null tape");
  if (steps) *steps = tp->cap;
  if (rec) *rec = tp->rec;
  return DMX_OK;
}

dmx_status dmx_tape_data(const dmx_tape* tp, const double** records, const int32_t** n_steps) {
  if (!tp) return fail(DMX_ERR_INVALID_ARG, "null tape");
  if (records) *records = tp->records;
  if (n_steps) *n_steps = tp->n_acc;
  return DMX_OK;
}

void dmx_tape_destroy(dmx_tape* tp) {
  if (!tp) return;
  if (tp->records) (void)hipFree(tp->records);
  if (tp->n_acc) (void)hipFree(tp->n_acc);
  if (tp->status) (void)hipFree(tp->status);
  if (tp->queue) (void)hipFree(tp->queue);
  if (tp->tables) (void)hipFree(tp->tables);
  if (tp->stk_tables) (void)hipFree(tp->stk_tables);
  delete tp;
}

}  // extern "C"

// ---------------------------------------------------------------- graphs
struct dmx_graph {
  dmx_tape* tape = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

extern "C" {

// One forward call (and optionally its reverse sweep) over the batch with the
// given tape: a uniform batch of a free-body or tree model goes through
// dmx_rollout, every other batch through dmx_rollout_batch.
static dmx_status graph_segment(const dmx_batch* b, const dmx_solver_opts* opts, const double* x0, const double* u,
                                double* x_out, int32_t* status, const double* xbar, double* x0bar, double* ubar,
                                dmx_tape** tape, hipStream_t s) {
  const dmx_model* m0 = b->models[0];
  bool uniform = true;
  for (int w = 1; w < b->n_worlds; ++w) uniform = uniform && b->models[w] == m0;
  dmx_status r;
  if (uniform && m0->kind != 2)
    r = rollout_impl(m0, b->n_worlds, b->n_intervals, b->interval_dt, opts, x0, u, x_out, status, nullptr, nullptr,
                     tape, s, nullptr);
  else
    r = dmx_rollout_batch(b, opts, x0, u, x_out, status, nullptr, nullptr, tape, s);
  if (r != DMX_OK || !xbar) return r;
  return dmx_rollout_vjp(*tape, xbar, x0bar, ubar, s);
}

dmx_status dmx_graph_create(const dmx_batch* b, const dmx_solver_opts* opts, const double* x0, const double* u,
                            double* x_out, int32_t* world_status, const double* x_out_bar, double* x0_bar,
                            double* u_bar, void* stream, dmx_graph** out) {
  if (!b || !out || !b->models || b->n_worlds <= 0 || !x0 || !x_out || !world_status)
    return fail(DMX_ERR_INVALID_ARG, "null argument");
  if (x_out_bar && !x0_bar) return fail(DMX_ERR_INVALID_ARG, "x0_bar required with x_out_bar");
  for (int w = 0; w < b->n_worlds; ++w)
    if (!b->models[w]) return fail(DMX_ERR_INVALID_ARG, "null model in batch");
  *out = nullptr;
  hipStream_t s = (hipStream_t)stream;
  dmx_graph* g = new dmx_graph();
  // eager first run: allocates the tape and uploads the per-world tables
  dmx_status r = graph_segment(b, opts, x0, u, x_out, world_status, x_out_bar, x0_bar, u_bar, &g->tape, s);
  if (r == DMX_OK && hipStreamSynchronize(s) != hipSuccess) r = fail(DMX_ERR_HIP, "graph warm-up failed");
  hipStream_t cs = nullptr;
  if (r == DMX_OK && hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess)  // default priority
    r = fail(DMX_ERR_HIP, "capture stream");
  if (r == DMX_OK) {
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      r = fail(DMX_ERR_HIP, "stream capture did not begin");
    } else {
      // with the tape reused, the calls only launch kernels and copy device
      // to device: nothing allocates or synchronizes while capturing
      const dmx_status rc = graph_segment(b, opts, x0, u, x_out, world_status, x_out_bar, x0_bar, u_bar, &g->tape, cs);
      const hipError_t e = hipStreamEndCapture(cs, &g->graph);
      if (rc != DMX_OK) r = rc;
      else if (e != hipSuccess || !g->graph) r = fail(DMX_ERR_HIP, std::string("capture: ") + hipGetErrorString(e));
      else if (hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess)
        r = fail(DMX_ERR_HIP, "graph instantiation failed");
    }
  }
  if (cs) (void)hipStreamDestroy(cs);
  if (r != DMX_OK) {
    dmx_graph_destroy(g);
    return r;
  }
  *out = g;
  return DMX_OK;
}

dmx_status dmx_autotune_batch(const dmx_batch* b, const double* x0, const double* u, void* stream,
                              dmx_tuning* best, int32_t* n_tried, dmx_tuning* tried) {
  if (!b || !b->models || b->n_worlds <= 0 || !x0 || !best) return fail(DMX_ERR_INVALID_ARG, "null argument");
  const int W = b->n_worlds;
  long long nx = 0, nu = 0;
  bool uniform = true;
  for (int w = 0; w < W; ++w) {
    const dmx_model* m = b->models[w];
    if (!m) return fail(DMX_ERR_INVALID_ARG, "null model in batch");
    nx += m->nq + m->nv;
    nu += (long long)b->n_intervals * m->nu;
    uniform = uniform && m == b->models[0];
  }
  if (nu > 0 && !u) return fail(DMX_ERR_INVALID_ARG, "controls required");
  const dmx_model* m0 = b->models[0];
  std::vector<int> teams;
  if (uniform && m0->kind != 2) {
    for (const KernelEntry* kp : all_kernels())
      if (kp->kind == m0->kind && kp->nc == m0->ncb && (m0->kind != 1 || (kp->nv == m0->nv && kp->nb == m0->nb)))
        teams.push_back(kp->team);
    if (teams.empty()) return fail(DMX_ERR_UNSUPPORTED, "no kernel for this model");
  } else {
    teams.push_back(0);
  }
  hipStream_t s = (hipStream_t)stream;
  double *xo = nullptr, *xb = nullptr, *x0b = nullptr, *ub = nullptr;
  int* st = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMalloc(&xo, sizeof(double) * nx);
  if (e == hipSuccess) e = hipMalloc(&xb, sizeof(double) * nx);
  if (e == hipSuccess) e = hipMalloc(&x0b, sizeof(double) * nx);
  if (e == hipSuccess && nu) e = hipMalloc(&ub, sizeof(double) * nu);
  if (e == hipSuccess) e = hipMalloc(&st, sizeof(int) * W);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  auto cleanup = [&]() {
    for (void* p : {(void*)xo, (void*)xb, (void*)x0b, (void*)ub, (void*)st}) if (p) (void)hipFree(p);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  if (e != hipSuccess) { cleanup(); return fail(DMX_ERR_OUT_OF_MEMORY, "autotune buffers"); }
  {
    std::vector<double> ones((size_t)nx, 1.0);
    if (hipMemcpy(xb, ones.data(), sizeof(double) * nx, hipMemcpyHostToDevice) != hipSuccess) {
      cleanup();
      return fail(DMX_ERR_HIP, "autotune cotangent");
    }
  }
  int count = 0;
  bool have = false;
  for (int team : teams)
    for (int stages : {1, 0})
      for (int queue : {1, -1}) {
        dmx_solver_opts o;
        dmx_default_opts(&o);
        o.lanes_per_world = team;
        o.tape_stages = stages;
        o.work_queue = queue;
        dmx_tape* tape = nullptr;
        float ms = 0.0f;
        dmx_status r = graph_segment(b, &o, x0, u, xo, st, xb, x0b, ub, &tape, s);  // allocates the tape
        if (r == DMX_OK && hipEventRecord(e0, s) != hipSuccess) r = fail(DMX_ERR_HIP, "event record");
        if (r == DMX_OK) r = graph_segment(b, &o, x0, u, xo, st, xb, x0b, ub, &tape, s);
        if (r == DMX_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                            hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
          r = fail(DMX_ERR_HIP, "autotune timing");
        if (tape) dmx_tape_destroy(tape);
        if (r != DMX_OK) { cleanup(); return r; }
        const dmx_tuning t{team, stages, queue, (double)ms};
        if (tried && count < 32) tried[count] = t;
        ++count;
        if (!have || t.ms < best->ms) { *best = t; have = true; }
      }
  cleanup();
  if (n_tried) *n_tried = count;
  return DMX_OK;
}

dmx_status dmx_graph_launch(dmx_graph* g, void* stream) {
  if (!g || !g->exec) return fail(DMX_ERR_INVALID_ARG, "null graph");
  HIP_TRY(hipGraphLaunch(g->exec, (hipStream_t)stream));
  return DMX_OK;
}

const dmx_tape* dmx_graph_tape(const dmx_graph* g) { return g ? g->tape : nullptr; }

void dmx_graph_destroy(dmx_graph* g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->tape) dmx_tape_destroy(g->tape);
  delete g;
}

}  // extern "C"

// ---------------------------------------------------------------- serving
namespace {
double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct SrvBatch;

struct SrvReq {
  uint64_t id = 0;
  const dmx_model* model = nullptr;
  int N = 0, H = 0, nu = 0, nx = 0;
  double dt = 0.0, cw = 0.0, target[3] = {0, 0, 0};
  int want_grad = 0;
  std::vector<double> x0, u;
  size_t bytes = 0;     // device bytes this request adds to a batch
  SrvBatch* batch = nullptr;
  int w0 = 0;           // first world in the batch
  long long u0 = 0;     // first control element in the batch
  int state = 0;        // 0 queued, 1 running, 2 done
  double t_submit = 0, t_start = 0, t_done = 0;
};

// Device and pinned layout of a batch.  The inputs (x0 per world, controls,
// per-world tables) are one contiguous region copied host-to-device in one
// transfer; the outputs (cost, u_bar, status) one region copied back.
struct SrvBatch {
  const dmx_model* model = nullptr;
  double dt = 0.0;
  int want_grad = 0, nx = 0, nu = 0, rec = 0, W = 0;
  long long n_u = 0, n_rec = 0;
  std::vector<SrvReq*> reqs;
  size_t off = 0, bytes = 0;
  bool stack = false;  // served by the cube-stack kernels (requests of any cube count merge)
  long long n_x = 0;   // state doubles of all worlds (13 k_w each for stacks)
  long long n_recd = 0;  // tape doubles (records x their lengths)
  size_t o_x0, o_u, o_nint, o_uoff, o_toff, o_xoff, o_cap, o_order, o_target, o_cw, o_models, o_pos, o_nxw, in_end;
  size_t o_cost, o_ubar, o_status, out_end;
  size_t o_xout, o_nacc, o_xbar, o_x0bar, o_queue, o_tape;
  void* pin_in = nullptr;
  void* pin_out = nullptr;
  hipEvent_t ev = nullptr;
  int unpolled = 0;

  void layout() {
    size_t o = 0;
    auto take = [&](size_t n) { size_t at = o; o += align256(n); return at; };
    o_x0 = take(sizeof(double) * (size_t)n_x);
    o_u = take(sizeof(double) * (size_t)(n_u + 1));
    o_nint = take(sizeof(int) * W);
    o_uoff = take(sizeof(long long) * W);
    o_toff = take(sizeof(long long) * W);
    o_xoff = take(sizeof(long long) * W);
    o_cap = take(sizeof(int) * W);
    o_order = take(sizeof(int) * W);
    o_target = take(sizeof(double) * 3 * W);
    o_cw = take(sizeof(double) * W);
    o_models = take(stack ? sizeof(dmx::StackModel) * W : 0);
    o_pos = take(sizeof(int) * W);
    o_nxw = take(sizeof(int) * W);
    in_end = o;
    o_cost = take(sizeof(double) * W);
    o_ubar = take(sizeof(double) * (size_t)(n_u + 1));
    o_status = take(sizeof(int) * W);
    out_end = o;
    o_xout = take(sizeof(double) * (size_t)n_x);
    o_nacc = take(sizeof(int) * W);
    o_xbar = take(sizeof(double) * (size_t)n_x);
    o_x0bar = take(sizeof(double) * (size_t)n_x);
    o_queue = take(2 * sizeof(int));
    o_tape = take(sizeof(double) * (size_t)std::max(n_recd, 1ll));
    bytes = o;
  }
};

// served by the cube-stack kernels (a stack of two or more cubes)
bool served_as_stack(const dmx_model* m) { return !find_kernel(m, 0) && m->stack_ok; }
// tape record of one accepted step: with the stage accelerations, or for
// stacks a checkpoint whose stages the reverse sweep solves again
int served_record(const dmx_model* m) {
  return served_as_stack(m) ? 3 + 13 * m->stk.k : 3 + m->nq + m->nv + 6 * m->nv;
}
int steps_per_interval(const dmx_model* m, const dmx_server_opts& o) {
  return served_as_stack(m) ? o.stack_steps_per_interval : o.steps_per_interval;
}
long long world_records(const SrvReq& r, const dmx_server_opts& o) {
  return (long long)steps_per_interval(r.model, o) * r.H + 64;
}
long long request_records(const SrvReq& r, const dmx_server_opts& o) { return (long long)r.N * world_records(r, o); }

// device bytes a request adds to a batch (its share of every array, with the
// per-array alignment of the batch layout as slack)
size_t request_bytes(const SrvReq& r, const dmx_server_opts& o) {
  const size_t W = r.N, nu_tot = (size_t)r.N * r.H * r.nu, rec = served_record(r.model);
  return sizeof(double) * (W * r.nx * 4 + nu_tot * 2 + W * 5) + sizeof(long long) * 3 * W + sizeof(int) * 7 * W +
         (served_as_stack(r.model) ? sizeof(dmx::StackModel) * W : 0) +
         sizeof(double) * rec * (size_t)request_records(r, o) + 20 * 256;
}
}  // namespace

struct dmx_server {
  dmx_server_opts opts{};
  int device = 0;
  srv::Arena arena;
  srv::PinnedPool pinned;
  std::vector<hipStream_t> streams;
  std::vector<SrvBatch*> stream_batch;  // batch running on each stream (or null)
  std::mutex mu;
  std::condition_variable cv;
  std::deque<SrvReq*> queue;
  std::unordered_map<uint64_t, SrvReq*> all;
  uint64_t next_id = 1;
  int running_reqs = 0;
  std::atomic<bool> stop{false};
  std::thread worker;

  // Oldest waiting request plus every waiting request it can batch with.
  SrvBatch* form_batch() {
    if (queue.empty()) return nullptr;
    SrvReq* head = queue.front();
    SrvBatch* b = new SrvBatch();
    b->model = head->model; b->dt = head->dt; b->want_grad = head->want_grad;
    b->nx = head->nx; b->nu = head->nu; b->rec = served_record(head->model);
    b->stack = served_as_stack(head->model);
    size_t need = 0;
    for (SrvReq* r : queue) {
      // stacks of any cube count share the stack kernels (and the control
      // count of the top cube); other models batch with themselves
      const bool family = b->stack ? served_as_stack(r->model) && r->nu == b->nu : r->model == b->model;
      if (!family || r->dt != b->dt || r->want_grad != b->want_grad) continue;
      if (!b->reqs.empty() && b->W + r->N > opts.max_batch_worlds) break;
      if (need + r->bytes > arena.largest_free()) break;
      need += r->bytes;
      r->w0 = b->W; r->u0 = b->n_u;
      b->W += r->N;
      b->n_u += (long long)r->N * r->H * r->nu;
      b->n_rec += request_records(*r, opts);
      b->n_recd += request_records(*r, opts) * served_record(r->model);
      b->n_x += (long long)r->N * r->nx;
      b->reqs.push_back(r);
    }
    if (b->reqs.empty()) { delete b; return nullptr; }  // the head waits for budget
    b->layout();
    if (!arena.alloc(b->bytes, &b->off)) { delete b; return nullptr; }
    b->pin_in = pinned.get(b->in_end);
    b->pin_out = pinned.get(b->out_end - b->o_cost);
    if (!b->pin_in || !b->pin_out || hipEventCreateWithFlags(&b->ev, hipEventDisableTiming) != hipSuccess) {
      arena.release(b->off, b->bytes);
      if (b->pin_in) pinned.put(b->pin_in, b->in_end);
      if (b->pin_out) pinned.put(b->pin_out, b->out_end - b->o_cost);
      delete b;
      return nullptr;
    }
    for (SrvReq* r : b->reqs) {
      queue.erase(std::find(queue.begin(), queue.end(), r));
      r->batch = b;
      r->state = 1;
      r->t_start = now_s();
    }
    b->unpolled = (int)b->reqs.size();
    running_reqs += (int)b->reqs.size();
    return b;
  }

  bool launch(SrvBatch* b, hipStream_t s) {
    char* pin = (char*)b->pin_in;
    double* x0 = (double*)(pin + b->o_x0);
    double* u = (double*)(pin + b->o_u);
    int* nint = (int*)(pin + b->o_nint);
    long long* uoff = (long long*)(pin + b->o_uoff);
    long long* toff = (long long*)(pin + b->o_toff);
    long long* xoff = (long long*)(pin + b->o_xoff);
    dmx::StackModel* smod = (dmx::StackModel*)(pin + b->o_models);
    int* pos = (int*)(pin + b->o_pos);
    int* nxw = (int*)(pin + b->o_nxw);
    long long x_at = 0;
    int* cap = (int*)(pin + b->o_cap);
    int* order = (int*)(pin + b->o_order);
    double* target = (double*)(pin + b->o_target);
    double* cw = (double*)(pin + b->o_cw);
    long long rec0 = 0;
    for (SrvReq* r : b->reqs) {
      const long long wcap = world_records(*r, opts);
      const int rlen = served_record(r->model);
      for (int i = 0; i < r->N; ++i) {
        const int w = r->w0 + i;
        std::memcpy(x0 + x_at, r->x0.data(), sizeof(double) * r->nx);
        xoff[w] = x_at;
        nxw[w] = r->nx;
        pos[w] = b->stack ? 7 * (r->model->stk.k - 1) : 0;  // the controlled body: the top cube of a stack
        if (b->stack) smod[w] = r->model->stk;
        x_at += r->nx;
        nint[w] = r->H;
        uoff[w] = r->u0 + (long long)i * r->H * r->nu;
        toff[w] = b->stack ? rec0 : rec0 / b->rec;  // stack kernels take offsets in doubles, the others in records
        cap[w] = (int)wcap;
        rec0 += wcap * rlen;
        for (int j = 0; j < 3; ++j) target[3 * w + j] = r->target[j];
        cw[w] = r->cw;
      }
      if (!r->u.empty()) std::memcpy(u + r->u0, r->u.data(), sizeof(double) * r->u.size());
    }
    // longest horizons first
    for (int w = 0; w < b->W; ++w) order[w] = w;
    std::stable_sort(order, order + b->W, [&](int p, int q) { return nint[p] > nint[q]; });

    char* d = arena.base + b->off;
    if (hipMemcpyAsync(d, pin, b->in_end, hipMemcpyHostToDevice, s) != hipSuccess) return false;
    auto D = [&](size_t o) { return (void*)(d + o); };
    dmx_solver_opts oo;
    dmx_default_opts(&oo);
    int max_h = 0;
    for (SrvReq* r : b->reqs) max_h = std::max(max_h, r->H);
    const bool has_u = b->nu > 0;
    if (b->stack) {
      // cube stacks: every world is the batch's model; offsets from the tables
      dmx::StackArgs a{};
      a.W = b->W; a.n_int = max_h; a.dt = b->dt;
      a.models = (const dmx::StackModel*)D(b->o_models);
      a.x_off = (const long long*)D(b->o_xoff); a.u_off = (const long long*)D(b->o_uoff);
      a.t_off = (const long long*)D(b->o_toff); a.cap_w = (const int*)D(b->o_cap);
      a.n_int_w = (const int*)D(b->o_nint); a.order = (const int*)D(b->o_order);
      a.stages = 0;
      a.x0 = (const double*)D(b->o_x0); a.u = has_u ? (const double*)D(b->o_u) : nullptr;
      a.xout = (double*)D(b->o_xout); a.status = (int*)D(b->o_status); a.n_acc = (int*)D(b->o_nacc);
      a.tape = (double*)D(b->o_tape); a.o = to_solver(oo);
      a.queue = (int*)D(b->o_queue);
      dmx_host::stack_fwd(a, s, 0);
      hipLaunchKernelGGL(srv::cost_kernel, dim3((b->W + 63) / 64), dim3(64), 0, s, a.xout, a.status,
                         (const double*)D(b->o_u), b->W, a.x_off, (const int*)D(b->o_nxw), (const int*)D(b->o_pos), 3,
                         b->nu, a.n_int_w, a.u_off, (const double*)D(b->o_target), (const double*)D(b->o_cw), b->dt,
                         (double*)D(b->o_cost), (double*)D(b->o_xbar));
      if (b->want_grad) {
        a.xbar = (const double*)D(b->o_xbar);
        a.x0bar = (double*)D(b->o_x0bar);
        a.ubar = has_u ? (double*)D(b->o_ubar) : nullptr;
        a.queue = (int*)D(b->o_queue) + 1;
        dmx_host::stack_adj(a, s, 0);
        if (has_u)
          hipLaunchKernelGGL(srv::ctrl_grad_kernel, dim3(b->W), dim3(64), 0, s, (double*)D(b->o_ubar),
                             (const double*)D(b->o_u), b->nu, a.n_int_w, a.u_off, (const double*)D(b->o_cw), b->dt);
      }
      if (hipMemcpyAsync(b->pin_out, D(b->o_cost), b->out_end - b->o_cost, hipMemcpyDeviceToHost, s) != hipSuccess)
        return false;
      if (hipEventRecord(b->ev, s) != hipSuccess) return false;
      return hipGetLastError() == hipSuccess;
    }
    const KernelEntry* k = find_kernel(b->model, 0);
    dmx::Ragged g{};
    g.n_int_w = (const int*)D(b->o_nint);
    g.u_off = (const long long*)D(b->o_uoff);
    g.tape_off = (const long long*)D(b->o_toff);
    g.cap_w = (const int*)D(b->o_cap);
    g.order = (const int*)D(b->o_order);
    dmx::FwdArgs a{};
    a.W = b->W; a.n_int = max_h; a.nu = b->nu; a.dt = b->dt; a.x0 = (const double*)D(b->o_x0);
    a.u = has_u ? (const double*)D(b->o_u) : nullptr; a.xout = (double*)D(b->o_xout);
    a.status = (int*)D(b->o_status); a.n_acc = (int*)D(b->o_nacc); a.tape = (double*)D(b->o_tape);
    a.cap = 0; a.rec = b->rec; a.o = to_solver(oo);
    a.g = g; a.g.queue = (int*)D(b->o_queue);
    k->fwd(b->model->dev, a, s, 0);
    hipLaunchKernelGGL(srv::cost_kernel, dim3((b->W + 63) / 64), dim3(64), 0, s, a.xout, a.status,
                       (const double*)D(b->o_u), b->W, (const long long*)D(b->o_xoff), (const int*)D(b->o_nxw),
                       (const int*)D(b->o_pos), std::min(3, b->model->nq), b->nu, g.n_int_w, g.u_off,
                       (const double*)D(b->o_target), (const double*)D(b->o_cw), b->dt, (double*)D(b->o_cost),
                       (double*)D(b->o_xbar));
    if (b->want_grad) {
      dmx::AdjArgs ga{};
      ga.W = b->W; ga.n_int = max_h; ga.nu = b->nu; ga.tape = a.tape; ga.cap = 0; ga.rec = b->rec;
      ga.n_acc = a.n_acc; ga.status = a.status; ga.u = a.u; ga.xbar = (const double*)D(b->o_xbar);
      ga.x0bar = (double*)D(b->o_x0bar); ga.ubar = has_u ? (double*)D(b->o_ubar) : nullptr; ga.o = a.o;
      ga.g = g; ga.g.queue = (int*)D(b->o_queue) + 1;
      k->adj(b->model->dev, ga, s, 0);
      if (has_u)
        hipLaunchKernelGGL(srv::ctrl_grad_kernel, dim3(b->W), dim3(64), 0, s, (double*)D(b->o_ubar),
                           (const double*)D(b->o_u), b->nu, g.n_int_w, g.u_off, (const double*)D(b->o_cw), b->dt);
    }
    if (hipMemcpyAsync(b->pin_out, D(b->o_cost), b->out_end - b->o_cost, hipMemcpyDeviceToHost, s) != hipSuccess)
      return false;
    if (hipEventRecord(b->ev, s) != hipSuccess) return false;
    return hipGetLastError() == hipSuccess;
  }

  void finish(SrvBatch* b, bool ok) {
    const double t = now_s();
    for (SrvReq* r : b->reqs) { r->state = 2; r->t_done = ok ? t : -1.0; }
    running_reqs -= (int)b->reqs.size();
    arena.release(b->off, b->bytes);
    (void)hipEventDestroy(b->ev);
    b->ev = nullptr;
  }

  void loop() {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    int inflight = 0;
    while (!stop.load()) {
      bool progress = false;
      for (size_t i = 0; i < streams.size(); ++i) {
        SrvBatch* b = stream_batch[i];
        if (b && hipEventQuery(b->ev) == hipSuccess) {
          finish(b, true);
          stream_batch[i] = nullptr;
          --inflight;
          progress = true;
        }
      }
      for (size_t i = 0; i < streams.size() && inflight < opts.max_inflight; ++i) {
        if (stream_batch[i]) continue;
        SrvBatch* b = form_batch();
        if (!b) break;
        // the batch's requests left the queue and nothing else writes them
        // while it runs: pack and launch without holding the lock, so that
        // submit and poll are not blocked behind the host-side packing
        lk.unlock();
        const bool ok = launch(b, streams[i]);
        if (!ok) (void)hipStreamSynchronize(streams[i]);
        lk.lock();
        if (!ok) {
          finish(b, false);
        } else {
          stream_batch[i] = b;
          ++inflight;
        }
        progress = true;
      }
      if (progress) cv.notify_all();
      else cv.wait_for(lk, std::chrono::microseconds(50));
    }
  }
};

extern "C" {

void dmx_default_server_opts(dmx_server_opts* o) {
  o->hbm_budget_bytes = 8ll << 30;
  o->max_inflight = 4;
  o->n_streams = 4;
  o->steps_per_interval = 40;
  o->max_batch_worlds = 16384;
  o->stack_steps_per_interval = 128;
}

dmx_status dmx_server_create(const dmx_server_opts* opts, dmx_server** out) {
  if (!out) return fail(DMX_ERR_INVALID_ARG, "null argument");
  dmx_server_opts o;
  if (opts) o = *opts; else dmx_default_server_opts(&o);
  if (o.hbm_budget_bytes <= 0 || o.max_inflight <= 0 || o.n_streams <= 0 || o.steps_per_interval <= 0 ||
      o.max_batch_worlds <= 0 || o.stack_steps_per_interval <= 0)
    return fail(DMX_ERR_INVALID_ARG, "bad server options");
  dmx_server* sv = new dmx_server();
  sv->opts = o;
  HIP_TRY(hipGetDevice(&sv->device));
  hipError_t e = hipMalloc((void**)&sv->arena.base, (size_t)o.hbm_budget_bytes);
  if (e != hipSuccess) { delete sv; return fail(DMX_ERR_OUT_OF_MEMORY, "server arena: " + std::string(hipGetErrorString(e))); }
  sv->arena.size = (size_t)o.hbm_budget_bytes;
  sv->arena.free_[0] = sv->arena.size & ~size_t(255);
  for (int i = 0; i < o.n_streams; ++i) {
    hipStream_t s;
    e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);  // default priority
    if (e != hipSuccess) { dmx_server_destroy(sv); return fail(DMX_ERR_HIP, "stream creation failed"); }
    sv->streams.push_back(s);
    sv->stream_batch.push_back(nullptr);
  }
  sv->worker = std::thread([sv]() { sv->loop(); });
  *out = sv;
  return DMX_OK;
}

dmx_status dmx_submit(dmx_server* sv, const dmx_request* q, uint64_t* ticket) {
  if (!sv || !q || !ticket || !q->model || !q->x0) return fail(DMX_ERR_INVALID_ARG, "null argument");
  if (q->n_worlds <= 0 || q->n_intervals <= 0 || !(q->interval_dt > 0.0)) return fail(DMX_ERR_INVALID_ARG, "bad sizes");
  const dmx_model* m = q->model;
  if (m->nu > 0 && !q->u) return fail(DMX_ERR_INVALID_ARG, "controls required");
  if (!find_kernel(m, 0) && !m->stack_ok) return fail(DMX_ERR_UNSUPPORTED, "no kernel for this model");
  if ((long long)std::max(sv->opts.steps_per_interval, sv->opts.stack_steps_per_interval) * q->n_intervals + 64 >
      INT32_MAX)
    return fail(DMX_ERR_INVALID_ARG, "horizon too long");
  SrvReq* r = new SrvReq();
  r->model = m; r->N = q->n_worlds; r->H = q->n_intervals; r->nu = m->nu; r->nx = m->nq + m->nv;
  r->dt = q->interval_dt; r->cw = q->ctrl_weight; r->want_grad = q->want_grad;
  for (int i = 0; i < 3; ++i) r->target[i] = q->target[i];
  r->x0.assign(q->x0, q->x0 + r->nx);
  if (m->nu > 0) r->u.assign(q->u, q->u + (size_t)r->N * r->H * r->nu);
  r->bytes = request_bytes(*r, sv->opts);
  if (r->bytes > sv->arena.size) { delete r; return fail(DMX_ERR_BUDGET, "request larger than the device budget"); }
  r->t_submit = now_s();
  {
    std::lock_guard<std::mutex> g(sv->mu);
    r->id = sv->next_id++;
    sv->all[r->id] = r;
    sv->queue.push_back(r);
  }
  sv->cv.notify_all();
  *ticket = r->id;
  return DMX_OK;
}

dmx_status dmx_poll(dmx_server* sv, uint64_t ticket, dmx_result* out) {
  if (!sv || !out) return fail(DMX_ERR_INVALID_ARG, "null argument");
  SrvReq* r;
  {
    std::lock_guard<std::mutex> g(sv->mu);
    auto it = sv->all.find(ticket);
    if (it == sv->all.end()) return fail(DMX_ERR_NOT_FOUND, "unknown ticket");
    r = it->second;
    if (r->state != 2) return DMX_PENDING;
    sv->all.erase(it);
  }
  SrvBatch* b = r->batch;
  const size_t nut = (size_t)r->N * r->H * r->nu;
  const char* po = (const char*)b->pin_out;  // region starting at the batch's cost array
  const size_t base = b->o_cost;
  if (out->cost) std::memcpy(out->cost, po + (b->o_cost - base) + sizeof(double) * r->w0, sizeof(double) * r->N);
  if (out->grad_u && r->want_grad && nut)
    std::memcpy(out->grad_u, po + (b->o_ubar - base) + sizeof(double) * r->u0, sizeof(double) * nut);
  if (out->world_status)
    std::memcpy(out->world_status, po + (b->o_status - base) + sizeof(int) * r->w0, sizeof(int) * r->N);
  out->t_submit = r->t_submit; out->t_start = r->t_start; out->t_done = r->t_done;
  const bool ok = r->t_done >= 0.0;
  {
    std::lock_guard<std::mutex> g(sv->mu);
    if (--b->unpolled == 0) {
      sv->pinned.put(b->pin_in, b->in_end);
      sv->pinned.put(b->pin_out, b->out_end - b->o_cost);
      delete b;
    }
  }
  delete r;
  return ok ? DMX_OK : fail(DMX_ERR_HIP, "request launch failed");
}

dmx_status dmx_server_stats(const dmx_server* sv, int32_t* queued, int32_t* inflight, int64_t* bytes) {
  if (!sv) return fail(DMX_ERR_INVALID_ARG, "null server");
  std::lock_guard<std::mutex> g(const_cast<dmx_server*>(sv)->mu);
  if (queued) *queued = (int32_t)sv->queue.size();
  if (inflight) *inflight = (int32_t)sv->running_reqs;
  if (bytes) *bytes = (int64_t)sv->arena.used;
  return DMX_OK;
}

void dmx_server_destroy(dmx_server* sv) {
  if (!sv) return;
  sv->stop.store(true);
  sv->cv.notify_all();
  if (sv->worker.joinable()) sv->worker.join();
  for (hipStream_t s : sv->streams) { (void)hipStreamSynchronize(s); (void)hipStreamDestroy(s); }
  std::set<SrvBatch*> batches;
  for (SrvBatch* b : sv->stream_batch)
    if (b) batches.insert(b);
  for (auto& kv : sv->all) {
    if (kv.second->batch) batches.insert(kv.second->batch);
    delete kv.second;
  }
  for (SrvBatch* b : batches) {
    if (b->ev) (void)hipEventDestroy(b->ev);
    delete b;  // pinned buffers are freed with the pool
  }
  if (sv->arena.base) (void)hipFree(sv->arena.base);
  delete sv;
}

}  // extern "C"
