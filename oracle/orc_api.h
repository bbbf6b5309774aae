/* Oracle C API (TEST INFRASTRUCTURE ONLY).
 *
 * A plain, slow FP64 CPU implementation of the soft-contact rigid-body ODE of
 * the paper (equation of motion, Sec. 2; relaxed-Gauss primal problem and the
 * reference acceleration, Sec. 2.1), integrated by Dormand-Prince 5(4) with a
 * PI step controller (Sec. 3.1, App. C.2), and its derivative by forward-mode
 * differentiation of the discretized solve with step sizes held fixed
 * (discretize-then-optimize, App. C.2), optionally with the contacts-from-
 * distance straight-through rule (Sec. 4).  Only the test-suite, the smoke
 * check and the CPU-baseline leg of the benchmark call it; it shares no code
 * with the HIP library.
 */
#ifndef ORC_API_H
#define ORC_API_H
#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int nb, nj, ng, npair, nu;
  const int* body_parent;        /* nb, parents precede children, -1 = world */
  const double* body_pos;        /* nb*3, frame in parent frame */
  const double* body_quat;       /* nb*4 (w,x,y,z) */
  const int* body_iner_type;     /* nb: 1 sphere, 2 capsule, 3 box */
  const double* body_iner_size;  /* nb*3 */
  const double* body_iner_quat;  /* nb*4, orientation of the primitive in the body frame */
  const double* body_mass;       /* nb, <= 0 means density 1000 kg/m^3 */
  const int* jnt_body;           /* nj, joints grouped by body in body order */
  const int* jnt_type;           /* nj: 0 free, 1 hinge, 2 slide */
  const double* jnt_axis;        /* nj*3 (body frame) */
  const double* jnt_pos;         /* nj*3 (body frame) */
  const int* geom_body;          /* ng, -1 = world */
  const int* geom_type;          /* ng: 0 plane, 1 sphere, 2 capsule, 3 box */
  const double* geom_size;       /* ng*3 */
  const double* geom_pos;        /* ng*3 */
  const double* geom_quat;       /* ng*4 */
  const int* pair_g1;            /* npair; g1 must be the plane for plane pairs */
  const int* pair_g2;
  const double* pair_mu;         /* npair */
  const double* pair_solref;     /* npair*2: time constant, damping ratio */
  const double* pair_solimp;     /* npair*5: d0, dwidth, width, midpoint, power */
  const double* pair_cfd;        /* npair*5: d_c, d_0, w_c, m_c, p_c */
  const int* ctrl_dof;           /* nu */
  double gravity[3];
} orc_model_def;

typedef struct {
  double rtol, atol, h0, safety, facmin, facmax, kP, kI, err_order, err_floor;
  long long max_attempts;
  int newton_maxit;
  int cfd;              /* 1: straight-through contacts-from-distance in the derivative */
  double softplus_beta; /* sharpness of the softplus position term of the CFD force */
  int h_levels;         /* proposed step sizes rounded down to this many mantissa levels per octave (0: off,
                           the default: the continuous controller) */
  int tableau;          /* 0: Dormand-Prince 5(4) (default), 1: Tsitouras 5(4) (Tsit5, the paper's solver,
                           App. E.1); optimize-then-discretize takes 0 only */
} orc_opts;

/* CONTACT_OVERFLOW: more than 256 contacts within reach at some evaluation; the
 * first 256 in pair order were used (not fatal: the world continues). */
enum { ORC_MAX_STEPS = 1, ORC_DT_UNDERFLOW = 2, ORC_NONFINITE = 4, ORC_SOLVER_MAXIT = 8, ORC_CONTACT_OVERFLOW = 16,
       ORC_UNSUPPORTED = 64 };

void* orc_model_new(const orc_model_def* def);
void orc_model_free(void* m);
/* out: nq, nv, nu, max_contacts */
void orc_model_sizes(const void* m, int* out);
/* per body: mass, inertia about the origin in the body frame (3x3), translational inverse weight */
void orc_model_inertia(const void* m, double* mass, double* inertia, double* invweight);

/* kinematics at (q, v): body positions nb*3, rotations nb*9, M nv*nv, bias c nv,
 * body twists nb*6 (world angular velocity, origin linear velocity). */
int orc_kinematics(const void* m, const double* q, const double* v, double* xpos, double* xmat,
                   double* M, double* c, double* twist);
/* all candidate contacts at q: rows of 13 = r, pos[3], n[3], t1[3], t2[3]; returns count */
int orc_contacts(const void* m, const double* q, double* out);
/* the same with cfd = 1: box-box pairs also emit contacts within the CFD width w_c */
int orc_contacts_cfd(const void* m, const double* q, int cfd, double* out);
/* point Jacobian (3*nv) of a point attached to body b */
void orc_point_jac(const void* m, const double* q, int body, const double* point, double* jac);
/* right-hand side F(x) = (v, qacc); info = n_rows, n_active, newton_iterations, status */
int orc_rhs(const void* m, const double* x, const double* u, int cfd, double* xdot, int* info,
            double* forces);
/* the primal problem at x (cfd: the contacts-from-distance rows with softplus sharpness beta):
 * M (nv*nv), a0 (nv), rows J (n*nv), aref (n), D (n); returns n */
int orc_rows(const void* m, const double* x, const double* u, int cfd, double beta, double* M, double* a0, double* J,
             double* aref, double* D);
/* directional derivatives of F: value of F (cfd=0 rule) and, per direction, the
 * tangent of F (or of the CFD field when st=1: straight-through). */
int orc_rhs_jvp(const void* m, const double* x, const double* u, int st, double beta, int n_dir,
                const double* dx, const double* du, double* xdot, double* dxdot);

/* one world.  counters: n_accepted, n_rejected, n_rhs, newton_iterations, status.
 * tape: per accepted step (t_n, h_n, y_n[nx]) up to tape_cap records.
 * steplog: per attempt (t, h, err, accepted) up to log_cap records.
 * forced: if non-NULL, (t_n, h_n) of n_forced steps replayed without control. */
int orc_rollout(const void* m, const double* x0, const double* u, int n_int, double dt_int,
                const orc_opts* o, const double* forced, int n_forced, double* x_out, long long* counters,
                int tape_cap, double* tape, int log_cap, double* steplog);
/* operation count of one world's forward rollout (the rollout of orc_rollout,
 * run in a counting scalar, one thread).  out[16]: floating-point operations
 * by phase (0 the attempt's stage combinations, (+)-maps and error estimate,
 * 1 the right-hand side outside the contact solve: kinematics, mass matrix,
 * collision, contact rows, 2 Newton iterations: gradient, Hessian assembly,
 * factorization, solve, activity tests, 3 line searches, 4 other), then
 * attempts, right-hand sides, Newton iterations, contacts summed over
 * right-hand sides, contacts with an active edge summed over Newton
 * iterations, contacts summed over line-search segments, accepted steps,
 * status, then the three contact sums again for contacts between two bodies
 * only.  Operations with a structurally zero or unit operand are not
 * counted. */
int orc_flop_count(const void* m, const double* x0, const double* u, int n_int, double dt_int,
                   const orc_opts* o, long long* out);  /* out[16] */
/* optimize-then-discretize gradients (App. C.2 eq. adjoint-equations; with
 * cfd, the straight-through adjoint of App. C.4): per world the forward
 * rollout, then the continuous adjoint equations solved backwards with the
 * adaptive Dormand-Prince pair (rtol, atol, controller of o) along the
 * forward's continuous extension.  x0bar [W][nx] (quaternion parts tangent at
 * q0), ubar [W][n_int][nu]; counters [W][4] = adjoint attempts, adjoint
 * accepted steps, forward accepted steps, status. */
int orc_otd_grad_batch(const void* m, int W, const double* x0, const double* u, int n_int, double dt_int,
                       const orc_opts* o, const double* xbar, double* x_out, double* x0bar, double* ubar,
                       long long* counters, int n_threads);
/* weights w[7] of the stage slopes in the Dormand-Prince continuous extension
 * at the fraction theta of a step. */
void orc_dense_weights(double theta, double* w);
/* x(tau) [n_tau][nx] of one world's rollout (forced steps as for orc_rollout)
 * from the continuous extension of its accepted steps. */
int orc_dense_states(const void* m, const double* x0, const double* u, int n_int, double dt_int, const orc_opts* o,
                     const double* forced, int n_forced, int n_tau, const double* tau, double* out);
/* operation count of the oracle's Cholesky factorization and two triangular
 * solves of the n x n row-major matrix A (zero entries structural); -1 if A
 * is not positive definite. */
long long orc_flop_cholesky(const double* A, int n);
/* forward-mode tangents of the rollout with frozen steps (taken from its own
 * adaptive run).  dx0: n_dir*nx, du: n_dir*n_int*nu, tx: n_dir*nx. */
int orc_rollout_jvp(const void* m, const double* x0, const double* u, int n_int, double dt_int,
                    const orc_opts* o, int n_dir, const double* dx0, const double* du, double* x_out,
                    double* tx, long long* counters);
/* the same along a given frozen step sequence forced [n_forced][2] = (t_n, h_n) */
int orc_rollout_jvp_forced(const void* m, const double* x0, const double* u, int n_int, double dt_int,
                           const orc_opts* o, const double* forced, int n_forced, int n_dir, const double* dx0,
                           const double* du, double* x_out, double* tx);
/* batched value rollouts and batched gradients J^T xbar over worlds, on n_threads host threads */
int orc_rollout_batch(const void* m, int n_worlds, const double* x0, const double* u, int n_int,
                      double dt_int, const orc_opts* o, double* x_out, long long* counters, int n_threads);
int orc_grad_batch(const void* m, int n_worlds, const double* x0, const double* u, int n_int, double dt_int,
                   const orc_opts* o, const double* xbar, double* x_out, double* x0bar, double* ubar,
                   long long* counters, int n_threads);
/* the same along given accepted-step sequences forced [n_worlds][forced_cap][2] = (t_n, h_n),
 * forced_n [n_worlds] steps each (controller off) */
int orc_grad_forced_batch(const void* m, int n_worlds, const double* x0, const double* u, int n_int, double dt_int,
                          const orc_opts* o, const double* forced, const int* forced_n, int forced_cap,
                          const double* xbar, double* x_out, double* x0bar, double* ubar, long long* counters,
                          int n_threads);
/* one attempt from y with step h (first stage evaluated at y): 5th-order state and error norm */
int orc_attempt(const void* m, const double* y, const double* u, double h, const orc_opts* o, double* ynew,
                double* err);
/* the controller's next proposed step after an attempt (eprev_out: its memory for the next one) */
double orc_next_step(const orc_opts* o, double err, double eprev, double h, int accepted, double* eprev_out);

#ifdef __cplusplus
}
#endif
#endif
