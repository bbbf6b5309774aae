"""Parity of GPU rollouts under the continuous step-size controller.

Two correct implementations of an adaptive integrator agree on every step
only up to rounding, and a chaotic world (a tumbling cube) turns a
rounding-level difference of the error estimate into a different step
sequence.  So a free GPU run is checked in three parts, each against the
oracle:
  1. its accepted-step sequence (t_n, h_n), replayed by the oracle with the
     controller off, gives the GPU's end state (1e-6) and gradient (1e-5,
     normwise and element by element) -- the discretization both sides
     differentiate is then the same one;
  2. every attempt's accept/reject decision equals the one the oracle takes
     from its own error estimate of that attempt (the same start state and
     step size), except where the oracle's own estimate moves across 1 under
     perturbations of the start state by a few ulp (then rounding decides:
     e.g. a body at rest on a stiff contact, where steps sit at the explicit
     stability limit and the estimate is the amplified rounding noise of the
     stiff mode);
  3. every proposed step is the oracle controller's answer to the GPU's
     error estimates (or the landing step on an interval end).
"""
import numpy as np

STATE_TOL, GRAD_TOL = 1e-6, 1e-5
# |eps - 1| below which the accept decision is decided by rounding, at least
DECISION_BAND = 1e-6
# start-state perturbations (relative, in ulp) that probe the estimate's own
# rounding sensitivity, and how many are drawn per attempt
ULP_PROBE, N_PROBES = 4.4e-16, 2


def rel_state(a, b, nq):
    a, b = np.atleast_2d(a), np.atleast_2d(b)
    dq = np.linalg.norm(a[:, :nq] - b[:, :nq], axis=1) / np.maximum(np.linalg.norm(b[:, :nq], axis=1), 1.0)
    dv = np.linalg.norm(a[:, nq:] - b[:, nq:], axis=1) / np.maximum(np.linalg.norm(b[:, nq:], axis=1), 1e-3)
    return np.maximum(dq, dv)


def rel_grad(a, b):
    a, b = np.atleast_2d(a), np.atleast_2d(b)
    return np.linalg.norm(a - b, axis=1) / np.maximum(np.linalg.norm(b, axis=1), 1e-12)


def elementwise_grad(a, b):
    """max_i |a_i - b_i| / max(|b_i|, 1e-3 |b|_inf) per world (element-wise
    relative error with a floor for entries far below the largest one)."""
    a, b = np.atleast_2d(a), np.atleast_2d(b)
    floor = 1e-3 * np.maximum(np.abs(b).max(axis=1, keepdims=True), 1e-300)
    return (np.abs(a - b) / np.maximum(np.abs(b), floor)).max(axis=1)


def tape_steps(tape):
    """(forced [W][cap][2], n [W]) from a GPU tape's accepted records."""
    recs, n = tape.records()
    cap = max(int(n.max()), 1)
    return np.ascontiguousarray(recs[:, :cap, :2]), n.astype(np.int32)


def replay_and_compare(om, nq, x0, u, n_int, dt, x_gpu, forced, n, xbar, gx, gu=None, n_threads=8, **opts):
    """Oracle replay of the GPU's accepted steps: end states and gradients.
    Returns the per-world errors; the caller asserts."""
    ref = om.grad_forced_batch(x0, u, n_int, dt, xbar, forced, n, n_threads=n_threads, **opts)
    assert (ref["status"] == 0).all(), ref["status"]
    out = {"state": rel_state(x_gpu, ref["x"], nq), "grad": rel_grad(gx, ref["x0bar"]),
           "grad_elem": elementwise_grad(gx, ref["x0bar"]), "ref": ref}
    if gu is not None:
        W = x0.shape[0]
        g = np.concatenate([gx, gu.reshape(W, -1)], axis=1)
        r = np.concatenate([ref["x0bar"], ref["ubar"].reshape(W, -1)], axis=1)
        out["grad"] = rel_grad(g, r)
        out["grad_elem"] = elementwise_grad(g, r)
    return out


def _interval(t, dt):
    k = t / dt
    kr = np.round(k)
    return int(kr) if abs(k - kr) < 1e-9 else int(np.floor(k))


def _err_band(om, y, uk, h, err_o, rng, **opts):
    """How far the oracle's error estimate of this attempt moves when the start
    state is perturbed by a few ulp (relative, random signs)."""
    band = DECISION_BAND
    for _ in range(N_PROBES):
        yp = y * (1.0 + ULP_PROBE * rng.choice([-1.0, 1.0], size=y.shape))
        _, e, st = om.attempt(yp, uk, h, **opts)
        if st & 12 or not np.isfinite(e) or not np.isfinite(err_o):
            return np.inf
        band = max(band, abs(e - err_o))
    return band


def check_decisions_and_controller(oracle, om, x0, u, n_int, dt, recs, n, steplog, log_n, worlds=None,
                                   **opts):
    """Parts 2 and 3 above for the listed worlds, each attempt taken from the
    GPU's own start state (its tape records recs [W][cap][3 + nx], n [W]
    accepted steps: a rejected attempt starts where the next accepted step
    does), so the check does not depend on how far a replay has drifted.
    Returns (attempts checked,
    decisions that differ outside the rounding band, decisions that differ
    where rounding decides, max relative difference of the error estimates
    where both are finite and above 1e-3, controller mismatches)."""
    rng = np.random.default_rng(11)
    nu = om.nu
    checked = bad_dec = bad_ctrl = rounding_decided = 0
    max_rel = 0.0
    for w in (range(x0.shape[0]) if worlds is None else worlds):
        uw = u[w] if nu else None
        states = {float(rec[0]): rec[3:3 + om.nx] for rec in recs[w, :n[w]]}
        log = steplog[w, :log_n[w]]
        eprev = 1.0
        h0 = min(opts.get("h0", 1e-3), dt)
        if len(log) and not opts.get("h_levels", 0):
            assert log[0][1] == h0, (w, log[0][1], h0)  # the first step
        for i, (t, h, err, acc) in enumerate(log):
            k = _interval(t, dt)
            y = states.get(float(t))
            assert y is not None, (w, i, t)
            uk = uw[min(k, n_int - 1)] if nu else None
            _, err_o, st = om.attempt(y, uk, h, **opts)
            if st & 12:
                err_o = np.inf
            checked += 1
            dec_g, dec_o = err <= 1.0, err_o <= 1.0
            if dec_g != dec_o and not (abs(err - 1.0) <= DECISION_BAND or abs(err_o - 1.0) <= DECISION_BAND):
                band = _err_band(om, y, uk, h, err_o, rng, **opts)
                if abs(err_o - 1.0) <= band or abs(err - 1.0) <= band:
                    rounding_decided += 1
                else:
                    bad_dec += 1
            if np.isfinite(err) and np.isfinite(err_o) and err_o > 1e-3:
                max_rel = max(max_rel, abs(err - err_o) / err_o)
            # the step the controller proposes after this attempt (GPU's own err)
            hprop, eprev = oracle.next_step(err if np.isfinite(err) else np.inf, eprev, h, bool(acc), **opts)
            if i + 1 < len(log):
                t1, h1 = log[i + 1][0], log[i + 1][1]
                tend = (_interval(t1, dt) + 1) * dt
                landing = t1 + 1.01 * hprop >= tend
                want = (tend - t1) if landing else hprop
                if abs(h1 - want) > 1e-12 * want:
                    bad_ctrl += 1
    return checked, bad_dec, rounding_decided, max_rel, bad_ctrl
