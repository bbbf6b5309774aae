/* dmx: batched differentiable soft-contact rigid-body rollouts on MI355X.
 *
 * The library integrates the ODE x' = F(t, x) of a penalty/soft-constraint
 * rigid-body simulator (state x = [q, v]; equation of motion of Sec. 2 with the
 * contact forces of the relaxed-Gauss primal problem and the reference
 * acceleration of Sec. 2.1) over piecewise-constant controls with an adaptive
 * Dormand-Prince 5(4) scheme and a PI step controller (Sec. 3.1, App. C.2),
 * for a batch of independent worlds, each with its own step sizes (App. D,
 * "Parallelizing DiffMJX simulations").  dmx_rollout_vjp returns the gradient
 * of the discretized rollout (discretize-then-optimize, App. C.2), optionally
 * with the contacts-from-distance straight-through rule (Sec. 4).
 *
 * Conventions
 *  - All floating point is FP64.  Unless stated otherwise pointers to state,
 *    control and gradient arrays are DEVICE pointers owned by the caller; they
 *    are read/written in order on `stream` and must stay valid until the work
 *    on the stream completes.  The library never frees caller memory.
 *  - State layout: x is world-major [n_worlds][nq + nv]; q holds, per joint in
 *    model order, a free joint's world position and unit quaternion (w,x,y,z)
 *    or a hinge/slide coordinate; v holds a free joint's world linear velocity
 *    of the body origin and body-frame angular velocity, or a hinge/slide rate.
 *  - Controls u are [n_worlds][n_intervals][nu]: generalized forces on the
 *    model's control dofs, constant over each interval of length interval_dt.
 *  - Errors: API-level errors are returned as a negative dmx_status with a
 *    message from dmx_last_error(); nothing is launched then.  Numerical
 *    failures of single worlds do not fail the call: they set bits of that
 *    world's status word and leave its state at the point of termination.
 *  - Thread safety: models are immutable after creation and may be shared;
 *    a tape belongs to one caller at a time.
 */
#ifndef DMX_H
#define DMX_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t dmx_status;
enum {
  DMX_OK = 0,
  DMX_PENDING = 1,
  DMX_ERR_INVALID_ARG = -1,
  DMX_ERR_OUT_OF_MEMORY = -2,
  DMX_ERR_HIP = -3,
  DMX_ERR_BUDGET = -4,
  DMX_ERR_NOT_FOUND = -5,
  DMX_ERR_UNSUPPORTED = -6
};

/* per-world status bits */
enum {
  DMX_W_MAX_STEPS = 1,      /* step-attempt budget exhausted */
  DMX_W_DT_UNDERFLOW = 2,   /* step size fell below 1e-12 max(1, |t|) */
  DMX_W_NONFINITE = 4,      /* non-finite state or singular mass matrix */
  DMX_W_SOLVER_MAXIT = 8,   /* contact Newton solve hit its iteration cap */
  DMX_W_CONTACT_OVERFLOW = 16, /* more than 256 contacts at some evaluation of a stack world; the
                                  first 256 in pair order were used (not fatal: the world goes on
                                  and its gradient is computed) */
  DMX_W_TAPE_OVERFLOW = 32, /* more accepted steps than the tape holds */
  DMX_W_CONTACT_GRAPH = 64  /* stack world: cubes that are not neighbours in the model's body order
                               touched (the solver takes block-tridiagonal Hessians); the world stops */
};

enum { DMX_JOINT_FREE = 0, DMX_JOINT_HINGE = 1, DMX_JOINT_SLIDE = 2 };
enum { DMX_GEOM_PLANE = 0, DMX_GEOM_SPHERE = 1, DMX_GEOM_CAPSULE = 2, DMX_GEOM_BOX = 3 };

/* Host-side model description (all pointers HOST memory, read during the call).
 * Bodies are listed parents first (parent -1 = world).  Each body's mass and
 * inertia are those of a uniform solid primitive (iner_type/iner_size/
 * iner_quat; mass <= 0 means density 1000 kg/m^3) about the body origin.
 * Joints are grouped by body, in body order, applied in order.  Geom sizes:
 * sphere (r), capsule (r, half-length along local z), box (half sizes).
 * Pairs list (g1, g2) with g1 a plane fixed to the world; the contact normal
 * points from g1 to g2.  solref = (time constant t_c, damping ratio);
 * solimp = (d0, dwidth, width, midpoint, power) of the impedance spline;
 * cfd = (d_c, d_0, w_c, m_c, p_c) of the contacts-from-distance spline (Sec. 4).
 * Control i is a generalized force on dof ctrl_dof[i]. */
typedef struct {
  int32_t nbody, njnt, ngeom, npair, nu;
  const int32_t* body_parent;
  const double* body_pos;        /* nbody*3 */
  const double* body_quat;       /* nbody*4 */
  const int32_t* body_iner_type; /* DMX_GEOM_SPHERE/CAPSULE/BOX */
  const double* body_iner_size;  /* nbody*3 */
  const double* body_iner_quat;  /* nbody*4 */
  const double* body_mass;       /* nbody */
  const int32_t* jnt_body;
  const int32_t* jnt_type;
  const double* jnt_axis;        /* njnt*3, body frame */
  const double* jnt_pos;         /* njnt*3, body frame */
  const int32_t* geom_body;
  const int32_t* geom_type;
  const double* geom_size;       /* ngeom*3 */
  const double* geom_pos;        /* ngeom*3 */
  const double* geom_quat;       /* ngeom*4 */
  const int32_t* pair_g1;
  const int32_t* pair_g2;
  const double* pair_mu;
  const double* pair_solref;     /* npair*2 */
  const double* pair_solimp;     /* npair*5 */
  const double* pair_cfd;        /* npair*5 */
  const int32_t* ctrl_dof;       /* nu */
  double gravity[3];
} dmx_model_desc;

typedef struct dmx_model dmx_model;
typedef struct dmx_tape dmx_tape;

/* Integrator options (App. E.1 names the PID controller P = 0.2, I = 0.4,
 * D = 0; the controller is used in PI form with the error exponent K).
 * dmx_default_opts fills: rtol 1e-6, atol 1e-8, h0 1e-3, safety 0.9,
 * facmin 0.2, facmax 10, kP 0.2, kI 0.4, err_order 5, err_floor 1e-6,
 * max_attempts 1e6, newton_maxit 100, cfd 0, softplus_beta 1e4,
 * tape_steps 0 (= chosen by the library), lanes_per_world 0 (= per model),
 * h_levels 0 (the continuous controller), tape_stages -1, work_queue 0. */
typedef struct {
  double rtol, atol, h0, safety, facmin, facmax, kP, kI, err_order, err_floor;
  int64_t max_attempts;
  int32_t newton_maxit;
  int32_t cfd;            /* 1: gradients use the contacts-from-distance field (straight-through) */
  double softplus_beta;   /* sharpness of the CFD position term, 1/m */
  int64_t tape_steps;     /* per-world tape capacity in accepted steps; 0 = library choice */
  int32_t lanes_per_world;/* team size (1,2,4,8,16); 0 = pick per model */
  /* test hooks (device pointers, may be NULL):
   * forced: [n_worlds][forced_cap][2] (t_n, h_n) accepted steps to replay with
   *         the controller off, forced_n[n_worlds] steps per world; a world's
   *         rollout ends after its last listed step;
   * steplog: [n_worlds][log_cap][4] (t, h, err, accepted) per attempt,
   *         log_n[n_worlds] attempts recorded. */
  const double* forced;
  const int32_t* forced_n;
  int32_t forced_cap;
  double* steplog;
  int32_t* log_n;
  int32_t log_cap;
  /* instrumentation (device pointers, may be NULL): per-world work units of
   * the forward, [n_worlds][9] = attempts, rhs evaluations, active contacts
   * over rhs evaluations, Newton iterations, active contacts and active edges
   * over Newton iterations, line-search contact evaluations, then the active
   * contacts over rhs evaluations and over Newton iterations of those
   * contacts that join two bodies (box-box pairs of stacks); and of the
   * reverse sweep, [n_worlds][4] = steps, acceleration vjps, active contacts
   * and active edges over vjps (written by dmx_rollout_vjp on this tape). */
  int64_t* fwd_counters;
  int64_t* adj_counters;
  /* 0: all worlds in one launch (default); 1: one launch per world on the
   * stream, the plain baseline form of the same kernels. */
  int32_t launch_mode;
  /* step-size grid (opt-in reproducibility mode, not part of the paper's
   * controller): the controller's proposed steps are rounded down to h_levels
   * mantissa values per octave, so that step sequences do not depend on
   * rounding-level differences of the error estimate between two
   * implementations; 0 (default): the continuous controller. */
  int32_t h_levels;
  /* failure capture (device, may be NULL): [n_worlds][nq + nv + nv] receives
   * the stage state and generalized force at which a world's contact solve
   * first failed (status bits NONFINITE or SOLVER_MAXIT). */
  double* fail_state;
  /* ragged batches and work distribution (device pointers, may be NULL; a
   * tape keeps its own copies, so they need only stay valid until the
   * rollout's work on the stream is done):
   * world_intervals [n_worlds]: control intervals world w simulates (at most
   * n_intervals; its controls are the first entries of u[w], its x_out is the
   * state at world_intervals[w] * interval_dt, its u_bar beyond them is 0);
   * world_order [n_worlds]: a permutation giving the order in which worlds
   * are taken from the work queue (longest first balances the load). */
  const int32_t* world_intervals;
  const int32_t* world_order;
  /* persistent launch with a device work queue: 0 = library choice (when the
   * batch exceeds the teams the device holds at once, or is ragged), 1 =
   * always, -1 = never (one world per team). */
  int32_t work_queue;
  /* tape contents: 1 = every accepted step with its stage accelerations; 0 =
   * checkpoints only (the step's start state; the reverse sweep solves the
   * step's stages again: about a third of the memory, one more forward's
   * work); -1 (default) = stages unless the tape would take more than half of
   * the free device memory. */
  int32_t tape_stages;
  /* Runge-Kutta pair: 0 = Dormand-Prince 5(4) (default); 1 = Tsitouras 5(4)
   * (Tsit5, the solver of the paper's experiments, App. E.1), for free-body
   * and tree models (stack batches and the optimize-then-discretize adjoint
   * take 0 only: DMX_ERR_UNSUPPORTED). */
  int32_t tableau;
} dmx_solver_opts;

void dmx_default_opts(dmx_solver_opts* opts);

/* Compile a model (inertia, inverse weights, pair tables) and upload it to
 * the current device: the simulator model of Sec. 2.1 (mass matrix, contact
 * pairs with their friction, solref and solimp, the regularizer's A-hat) with
 * the collision pairs of Sec. 2.1 and App. C.1.  The description is read
 * during the call only; the returned model is owned by the caller
 * (dmx_model_destroy).  Returns DMX_ERR_INVALID_ARG for parameters outside
 * their domain and DMX_ERR_UNSUPPORTED for model shapes the compiled kernels
 * do not cover. */
dmx_status dmx_model_create(const dmx_model_desc* desc, dmx_model** out);
/* Sizes of the model: nq, nv of the ODE state x = (q, v) (App. C.2), the
 * control count nu and the most contacts one state can have (host outputs,
 * each may be NULL). */
dmx_status dmx_model_info(const dmx_model* model, int32_t* nq, int32_t* nv, int32_t* nu, int32_t* max_contacts);
void dmx_model_destroy(dmx_model* model);

/* Forward rollout of n_worlds worlds of one model over n_intervals control
 * intervals of interval_dt seconds each.  x0 [W][nx], u [W][n_intervals][nu]
 * (may be NULL when nu == 0), x_out [W][nx], world_status [W].  If tape is
 * non-NULL a tape (device memory owned by the library) is created holding
 * every accepted step and its stage accelerations, for dmx_rollout_vjp; if
 * *tape is already a tape of this model and batch size (and at least
 * opts->tape_steps capacity) it is reused in place, with no allocation.
 * The tape keeps the pointer u: u must stay valid while the tape is used.
 * Per-world step counters: n_accepted, n_rejected ([W] int32, device, may be NULL). */
dmx_status dmx_rollout(const dmx_model* model, int32_t n_worlds, int32_t n_intervals, double interval_dt,
                       const dmx_solver_opts* opts, const double* x0, const double* u, double* x_out,
                       int32_t* world_status, int32_t* n_accepted, int32_t* n_rejected, dmx_tape** tape,
                       void* stream);

/* ------------------------------------------------------------ uneven batches
 * A batch of worlds of different models in one persistent launch (App. D,
 * "Parallelizing DiffMJX simulations": every world takes its own steps, so
 * worlds of different size and step count share a launch; a device work
 * queue hands out worlds, the ones with the most bodies first).  Every model
 * of the batch must be a stack of free cubes (k = 1..32 cubes, as built by a
 * model description with k bodies, one free joint and one box geom each, a
 * world plane, and every plane-cube and cube-cube pair with equal parameters:
 * the primitive-vs-primitive contacts of Sec. 2.1 with the box-box contact
 * reading of the separating-axis test and face clipping).  State, control and
 * gradient arrays are packed world after world: world w's state starts at
 * x_off[w] (13 k_w doubles: q = 7 k_w then v = 6 k_w) and its controls at
 * u_off[w] ([n_intervals][nu_w]); dmx_batch_layout gives the offsets. */
typedef struct {
  int32_t n_worlds;
  const dmx_model* const* models;  /* host array [n_worlds]: the model of each world */
  int32_t n_intervals;             /* control intervals (all worlds) */
  double interval_dt;              /* seconds per interval */
} dmx_batch;

/* Offsets (host arrays [n_worlds], may be NULL) and totals of the packed
 * state and control arrays of a batch. */
dmx_status dmx_batch_layout(const dmx_batch* batch, int64_t* x_off, int64_t* u_off, int64_t* nx_total,
                            int64_t* nu_total);

/* Forward rollout of an uneven batch (the calls and conventions of
 * dmx_rollout, with packed arrays): x0, x_out packed states, u packed
 * controls (NULL if no model has controls), world_status, n_accepted,
 * n_rejected [n_worlds].  With tape != NULL the tape holds every world's
 * accepted steps for dmx_rollout_vjp, whose x_out_bar, x0_bar and u_bar are
 * then packed the same way; a tape is reused in place when *tape is a tape of
 * the same models in the same order.  DMX_ERR_UNSUPPORTED if a model is not a
 * stack of cubes; forced steps, step logs and counters as for dmx_rollout;
 * ragged horizons (world_intervals) are not taken. */
dmx_status dmx_rollout_batch(const dmx_batch* batch, const dmx_solver_opts* opts, const double* x0,
                             const double* u, double* x_out, int32_t* world_status, int32_t* n_accepted,
                             int32_t* n_rejected, dmx_tape** tape, void* stream);

/* Forward rollout and reverse sweep of an uneven batch in one persistent
 * launch, for a final-state cotangent known before the rollout (a loss linear
 * in the final state, as the summed final positions, or a fixed direction):
 * each wavefront runs its world's forward rollout and then, on the tape it
 * has just written, that world's reverse sweep (the discrete adjoint of
 * Sec. 3 with the steps of App. D's batched rollouts), so the launch lasts as
 * long as the slowest world's forward plus reverse instead of the slowest
 * forward plus the slowest reverse.  Arguments as for dmx_rollout_batch
 * followed by dmx_rollout_vjp on its tape: x_out_bar (DEVICE, packed, input),
 * x0_bar and u_bar (DEVICE, packed, overwritten; u_bar required when a model
 * has controls); tape is required (created or reused as for
 * dmx_rollout_batch) and may be passed to dmx_rollout_vjp afterwards for
 * other cotangents.  Results equal those two calls bitwise; worlds whose
 * forward status is nonzero get NaN gradients.  fwd_counters and
 * adj_counters of opts both count. */
dmx_status dmx_rollout_batch_grad(const dmx_batch* batch, const dmx_solver_opts* opts, const double* x0,
                                  const double* u, const double* x_out_bar, double* x_out, int32_t* world_status,
                                  int32_t* n_accepted, int32_t* n_rejected, double* x0_bar, double* u_bar,
                                  dmx_tape** tape, void* stream);

/* The tape is the record of accepted steps that the discretize-then-optimize
 * gradient reverses (App. C.2), owned by the caller (dmx_tape_destroy).
 * Per-world layout of a tape's records (host arrays [n_worlds]): world w's
 * records start at records + t_off[w] and are rec[w] doubles long (t_n, h_n,
 * interval, y_n, then the stage accelerations a_1..a_6 unless the tape holds
 * checkpoints only); dmx_tape_info's steps_per_world is each world's
 * capacity. */
dmx_status dmx_tape_layout(const dmx_tape* tape, int64_t* t_off, int32_t* rec);

/* Autotuner for the batched rollouts of App. D ("Parallelizing DiffMJX
 * simulations"): times the forward rollout of this batch (device x0, u) with
 * every team size (lanes per world) compiled for the model, on the stream,
 * and makes the fastest (a wider team must win by 2%) the model's default
 * (used when lanes_per_world is 0).
 * Pass a representative batch with a short horizon.  best_lanes receives the
 * choice; n_tried, lanes_tried[8] and ms_tried[8] (host, may be NULL) the
 * candidates and their times.  Synchronizes the stream. */
dmx_status dmx_autotune(dmx_model* model, int32_t n_worlds, int32_t n_intervals, double interval_dt,
                        const double* x0, const double* u, void* stream, int32_t* best_lanes, int32_t* n_tried,
                        int32_t* lanes_tried, double* ms_tried);

/* Autotuner over a batch's launch choices (App. D: the batched, persistent
 * form of the rollouts): the tape policy (stage accelerations stored, or
 * checkpoints whose stages the reverse sweep solves again), the work
 * distribution (a device work queue taking the worlds with the most work
 * first, or one world per workgroup) and, for batches of one free-body or
 * tree model, every compiled team size (lanes per world, i.e. worlds packed
 * per wavefront).  Each candidate runs the forward rollout and the reverse
 * sweep (cotangent 1 on every final-state coordinate) of the caller's batch
 * (DEVICE x0, u, packed as for dmx_rollout_batch) twice; the second run, on
 * the tape of the first, is timed with events on the stream.  *best receives
 * the fastest; tried (host, may be NULL) up to 32 candidates, n_tried their
 * count.  Pass a representative batch with a short horizon.  Allocates its
 * own buffers and synchronizes the stream. */
typedef struct {
  int32_t lanes_per_world;  /* team size (0 for stack batches: one wavefront per world) */
  int32_t tape_stages;      /* dmx_solver_opts.tape_stages of the choice (1 or 0) */
  int32_t work_queue;       /* dmx_solver_opts.work_queue of the choice (1 or -1) */
  double ms;                /* forward + reverse milliseconds on the tuning batch */
} dmx_tuning;
dmx_status dmx_autotune_batch(const dmx_batch* batch, const double* x0, const double* u, void* stream,
                              dmx_tuning* best, int32_t* n_tried, dmx_tuning* tried);

/* Gradient of sum(x_out_bar * x_out) with respect to x0 and u through the
 * recorded discretization (step sizes held fixed; rejected attempts play no
 * part).  x0_bar [W][nx] and u_bar [W][n_intervals][nu] are overwritten.
 * Worlds whose forward status is nonzero get NaN gradients.  May be called
 * any number of times on one tape. */
dmx_status dmx_rollout_vjp(dmx_tape* tape, const double* x_out_bar, double* x0_bar, double* u_bar, void* stream);

/* dmx_rollout_vjp plus the gradient of the same loss with respect to the half
 * sizes of the model's box geom (a model parameter: the cube side length that
 * the paper's system identification recovers, Sec. 5.1 and App. E.2), through
 * the same recorded discretization: geom_size_bar [W][3] (DEVICE, overwritten;
 * world w's gradient, NaN for worlds whose forward status is nonzero).
 * Single free bodies whose contacts come from one box geom against planes;
 * DMX_ERR_UNSUPPORTED otherwise. */
dmx_status dmx_rollout_vjp_geom(dmx_tape* tape, const double* x_out_bar, double* x0_bar, double* u_bar,
                                double* geom_size_bar, void* stream);
/* dmx_rollout_vjp plus the gradient of the same loss with respect to the
 * model parameters that App. E.2 identifies: param_bar [W][12] (DEVICE,
 * overwritten; NaN for worlds whose forward status is nonzero) holds, in
 * order, the box geom's three half sizes (0 for models without a box geom),
 * the friction coefficient mu, the solref time constant t_c, the solref
 * damping ratio, the body's mass, and the solimp parameters (d0, dwidth,
 * width, midpoint, power).  The contact parameters (mu, solref, solimp) are
 * each taken as one value that every contact pair shares: the entry is the
 * derivative under the same shift of that parameter in every pair.  mu enters
 * the pyramid edges J_n +- mu J_t and the regularizer R (through (1 + mu^2));
 * t_c and the damping ratio enter a_ref's stiffness and damping; solimp
 * shapes the impedance d(r) in R and a_ref (Sec. 2.1; dwidth also scales
 * a_ref's stiffness and damping); the mass moves the body's inertia with it
 * (a uniform solid).  Free bodies, trees and stack batches (tapes of
 * dmx_rollout_batch, param_bar [n_worlds][12]): for a tree the half sizes are
 * 0 and the mass entry is NaN (a tree has one mass per body); for a stack
 * the half sizes are NaN (not differentiated there) and the mass is the one
 * all its cubes share. */
dmx_status dmx_rollout_vjp_params(dmx_tape* tape, const double* x_out_bar, double* x0_bar, double* u_bar,
                                  double* param_bar, void* stream);

/* Optimize-then-discretize gradient of sum(x_out_bar * x_out) (App. C.2, eq.
 * adjoint-equations; with opts.cfd of the forward, the straight-through
 * adjoint of App. C.4, whose Jacobian is that of the CFD field at the
 * trajectory of F): the continuous adjoint equations solved backwards in time
 * with the forward's Dormand-Prince pair and PI controller (rtol, atol,
 * h_levels of the forward's options) but their own steps, along the
 * continuous extension of the forward's accepted steps; each adjoint stage
 * solves the contact problem at the interpolated state.  Raw coordinates;
 * x0_bar's quaternion components are projected onto the tangent space at the
 * initial quaternion.  Layouts, outputs and NaN rule as for dmx_rollout_vjp.
 * Free-body and tree models whose tape holds stage accelerations
 * (opts.tape_stages != 0 at the rollout); DMX_ERR_UNSUPPORTED otherwise. */
dmx_status dmx_rollout_vjp_otd(dmx_tape* tape, const double* x_out_bar, double* x0_bar, double* u_bar, void* stream);
/* dmx_rollout_vjp_otd plus the box geom half sizes' gradient (the parameter
 * adjoint a_theta of eq. adjoint-equations: the integral of
 * (dF/dtheta)^T a_x over the horizon, by the adjoint's own quadrature):
 * geom_size_bar [W][3] (DEVICE, overwritten), models as for
 * dmx_rollout_vjp_geom. */
dmx_status dmx_rollout_vjp_otd_geom(dmx_tape* tape, const double* x_out_bar, double* x0_bar, double* u_bar,
                                    double* geom_size_bar, void* stream);
/* dmx_rollout_vjp_otd plus the twelve model-parameter gradients of
 * dmx_rollout_vjp_params (same layout and meaning), by the parameter adjoint
 * of eq. adjoint-equations.  Free bodies and trees (as for
 * dmx_rollout_vjp_params); DMX_ERR_UNSUPPORTED for stack batches. */
dmx_status dmx_rollout_vjp_otd_params(dmx_tape* tape, const double* x_out_bar, double* x0_bar, double* u_bar,
                                      double* param_bar, void* stream);

/* Captured rollout segments (HIP graphs), for callers that run the same
 * batch repeatedly with new inputs at the same addresses (receding-horizon
 * control loops, where each planning step is one short segment: App. D's
 * batched rollouts, used as in Sec. 5.2).  dmx_graph_create runs the forward
 * rollout of the batch once (as dmx_rollout_batch, or dmx_rollout when every
 * world has the same free-body or tree model), keeping its tape, then
 * records the same forward launch sequence and, if x_out_bar is given, the
 * reverse sweep (as dmx_rollout_vjp) into a graph over the given DEVICE
 * buffers: x0, u (inputs), x_out, world_status (outputs), x_out_bar (input),
 * x0_bar, u_bar (outputs); layouts as for those calls.  The buffers are the
 * caller's and must stay allocated while the graph lives.  dmx_graph_launch
 * replays the whole sequence on a stream after the caller has written new
 * x0 / u / x_out_bar values into the same buffers; its results are bitwise
 * those of the eager calls.  Nothing is allocated at launch.  Errors:
 * DMX_ERR_INVALID_ARG for null or mismatched arguments, DMX_ERR_HIP if
 * capture or instantiation fails (nothing is left allocated then). */
typedef struct dmx_graph dmx_graph;
dmx_status dmx_graph_create(const dmx_batch* batch, const dmx_solver_opts* opts, const double* x0, const double* u,
                            double* x_out, int32_t* world_status, const double* x_out_bar, double* x0_bar,
                            double* u_bar, void* stream, dmx_graph** out);
dmx_status dmx_graph_launch(dmx_graph* graph, void* stream);
/* The tape the graph writes (valid while the graph lives). */
const dmx_tape* dmx_graph_tape(const dmx_graph* graph);
void dmx_graph_destroy(dmx_graph* graph);

/* Allocation-free forward rollout, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation): the arguments and results of dmx_rollout without a
 * tape (no gradient), every buffer the caller's.  Its one scratch buffer,
 * the work-queue counter of the persistent launch, is a static device array
 * of the library (256 bytes per GPU, held until the process ends), cleared
 * by a kernel at each call; there is no size limit on the batch.  Calls that
 * overlap on one GPU race on that counter: issue them in stream order (one
 * stream, or synchronized streams).  Never calls hipMalloc or hipFree. */
dmx_status dmx_rollout_noalloc(const dmx_model* model, int32_t n_worlds, int32_t n_intervals, double interval_dt,
                               const dmx_solver_opts* opts, const double* x0, const double* u, double* x_out,
                               int32_t* world_status, int32_t* n_accepted, int32_t* n_rejected, void* stream);

/* Sizes of a tape (App. C.2's record of accepted steps): per-world capacity
 * and record length in doubles (host outputs). */
dmx_status dmx_tape_info(const dmx_tape* tape, int64_t* steps_per_world, int32_t* record_doubles);
/* Device pointer to the tape records [W][steps_per_world][record] with records
 * (t_n, h_n, interval, y_n[nx], then a_1..a_6[nv] unless the tape holds
 * checkpoints only) and the per-world accepted-step
 * counts [W] (int32). */
dmx_status dmx_tape_data(const dmx_tape* tape, const double** records, const int32_t** n_steps);
void dmx_tape_destroy(dmx_tape* tape);

/* Acceleration of the right-hand side F(x) = (v, qacc) at n independent states
 * (Sec. 2: the equation of motion with the soft-contact solve of Sec. 2.1).
 * x [n][nq+nv], tau [n][nv] generalized forces (NULL = zero), acc_out
 * [n][nv], status [n] (device pointers).  cfd = 1 evaluates the
 * contacts-from-distance field instead. */
dmx_status dmx_accel(const dmx_model* model, int32_t n, const double* x, const double* tau, int32_t cfd,
                     double* acc_out, int32_t* status, void* stream);

/* ------------------------------------------------------------------ serving
 * A request loop for model-predictive-control style work (the gradient-based
 * MPC of Sec. 5.2 evaluates many candidate control sequences and their
 * gradients per planning step): each request is N candidate control
 * sequences of one model from one initial state over H intervals; the result
 * is each candidate's cost
 *   cost = |p_T - target|^2 + ctrl_weight * sum_k |u_k|^2 * interval_dt
 * (p_T: the position of the controlled body in the final state: the first
 * three position coordinates, or for a stack of cubes the top cube's) and
 * its gradient with respect to the controls.
 *
 * Continuous batching: whenever one of the server's streams is free, the
 * oldest waiting request and every other waiting request of the same model,
 * interval_dt and want_grad (in arrival order, up to max_batch_worlds worlds
 * and the free device budget) are merged into one batch: one persistent
 * forward launch and one reverse launch over all their worlds, with ragged
 * horizons and a device work queue taking the longest worlds first.  Requests
 * arriving while batches run join the next batch.  Every world is computed
 * independently, so results are bitwise the same alone and in any mix.  All
 * request/result pointers are HOST memory; dmx_submit copies the inputs. */
typedef struct dmx_server dmx_server;

typedef struct {
  int64_t hbm_budget_bytes;  /* device arena the server allocates once (default 8 GiB) */
  int32_t max_inflight;      /* batches on the device at once (default 4, at most n_streams) */
  int32_t n_streams;         /* HIP streams, default priority (default 4) */
  int32_t steps_per_interval;/* tape capacity per world = this * n_intervals + 64 (default 40) */
  int32_t max_batch_worlds;  /* worlds merged into one batch (default 16384) */
  int32_t stack_steps_per_interval; /* the same for cube-stack models (default 128); their tapes hold
                                       checkpoints (3 + 13 k doubles per step) and the reverse sweep solves
                                       each step's stages again */
} dmx_server_opts;

typedef struct {
  const dmx_model* model;
  int32_t n_worlds;          /* N candidates */
  int32_t n_intervals;       /* H */
  double interval_dt;
  const double* x0;          /* [nq+nv], shared by the candidates */
  const double* u;           /* [N][H][nu] */
  double target[3];
  double ctrl_weight;
  int32_t want_grad;         /* 0: costs only */
} dmx_request;

typedef struct {
  double* cost;              /* [N] (caller buffers, filled by dmx_poll) */
  double* grad_u;            /* [N][H][nu] or NULL */
  int32_t* world_status;     /* [N] or NULL */
  double t_submit, t_start, t_done;  /* seconds on the server's monotonic clock */
} dmx_result;

void dmx_default_server_opts(dmx_server_opts* opts);
dmx_status dmx_server_create(const dmx_server_opts* opts, dmx_server** out);
/* Queue a request; DMX_ERR_BUDGET if it can never fit the budget. */
dmx_status dmx_submit(dmx_server* server, const dmx_request* req, uint64_t* ticket);
/* DMX_PENDING until the request is done, then DMX_OK with the result copied
 * out (the ticket is then released); DMX_ERR_NOT_FOUND for unknown tickets. */
dmx_status dmx_poll(dmx_server* server, uint64_t ticket, dmx_result* out);
/* Requests waiting and in flight, and bytes of the budget in use. */
dmx_status dmx_server_stats(const dmx_server* server, int32_t* queued, int32_t* inflight, int64_t* bytes_in_use);
/* Waits for in-flight work, then frees everything. */
void dmx_server_destroy(dmx_server* server);

/* Thread-local message of the last failed call. */
const char* dmx_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
