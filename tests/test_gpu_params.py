"""Model-parameter gradients beyond the side length (App. E.2 identifies mass,
solref, solimp and friction alongside it): the gradient of a final-state loss
with respect to the contact pairs' friction coefficient and solref (time
constant, damping ratio), solimp and the body's mass, with the box half sizes, through the recorded
discretization (dmx_rollout_vjp_params) and by the parameter adjoint of the
continuous adjoint equations (dmx_rollout_vjp_otd_params).

Parity: central differences of the oracle's frozen-step map (the GPU's own
accepted steps replayed by the oracle with every pair's parameter shifted by
+-eps, the model rebuilt each time), 1e-4 relative (to the parameter's largest gradient over the worlds) where the
differences have converged (relative steps 1e-6 and 1e-7 agree to 2e-5: no
contact or friction state switches within the perturbation), 2e-3 elsewhere.
Cases: a box and a corner cube (eight sphere-plane pairs) sliding and tipping
on the plane on persistent contact, the corner cube under controls (without
controls the accelerations do not depend on the mass: its gradient is 0).  The
continuous form is checked against the discrete adjoint on the same tape at
rtol 1e-10 (1e-3 relative; solimp d0 excepted) and against central differences
of the oracle's forward at rtol 1e-12 where those have converged."""
import copy

import numpy as np
import pytest

from paper_2506_14186_amd import workloads as W
from replay_check import tape_steps

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def D():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_14186_amd import dmx
    return dmx


def _t(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _shifted(desc, j, delta):
    """desc with parameter column j (3 friction, 4 solref t_c, 5 damping
    ratio, 7-11 solimp: in every contact pair; 6 the body's mass) shifted by
    delta."""
    d = copy.deepcopy(desc)
    if j == 6:  # every body (the cubes of a stack share one mass)
        for b in d["bodies"]:
            b["inertial"]["mass"] += delta
        return d
    for p in d["pairs"]:
        if j == 3:
            p["mu"] += delta
        elif j < 6:
            p["solref"][j - 4] += delta
        else:
            p["solimp"][j - 7] += delta
    return d


def _base_value(desc, j):
    if j == 6:
        return desc["bodies"][0]["inertial"]["mass"]
    p = desc["pairs"][0]
    return p["mu"] if j == 3 else p["solref"][j - 4] if j < 6 else p["solimp"][j - 7]


COLS = (3, 4, 5, 6, 7, 8, 9, 10, 11)


def _step(desc, j, rel):
    """Difference step for column j: relative to the value, absolute (rel)
    for the solimp d0 of the cube-toss setting, which is 0."""
    return rel * max(abs(_base_value(desc, j)), 1.0 if j == 7 else 0.0)


def _sliding_states(n, seed, height):
    rng = np.random.default_rng(seed)
    x0 = np.zeros((n, 13))
    x0[:, 2] = height
    tilt = rng.uniform(0.0, 0.1, n)
    x0[:, 3] = np.cos(tilt / 2)
    x0[:, 4] = np.sin(tilt / 2)
    x0[:, 7] = rng.uniform(-1.0, 1.0, n)
    x0[:, 8] = rng.uniform(-1.0, 1.0, n)
    x0[:, 12] = rng.uniform(-2.0, 2.0, n)
    return x0


# the cube-toss contact setting (solimp (0, 0.95, 0.001, 0.5, 2): resting
# contacts sit inside the impedance spline, on both sides of its midpoint)
CASES = {
    "box": (lambda: W.model_box(tc=0.005, mu=0.5), 0.0995, False),
    "corner_cube": (lambda: W.model_cube_corners(tc=0.005, mu=0.5, ctrl=True), 0.1095, True),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_contact_parameter_gradient_matches_oracle_differences(D, oracle, case):
    make, height, ctrl = CASES[case]
    desc = make()
    x0 = _sliding_states(6, 3, height)
    T, n_int = 0.08, 2
    rng = np.random.default_rng(4)
    model = D.Model(desc)
    u = rng.uniform(-2.0, 2.0, (x0.shape[0], n_int, model.nu)) if ctrl else None
    xb = np.zeros_like(x0)
    xb[:, 0], xb[:, 1], xb[:, 2], xb[:, 5] = 1.0, -0.5, 2.0, 1.0
    r = D.rollout(model, _t(x0), None if u is None else _t(u), n_int, T / n_int,
                  opts=D.default_opts(tape_steps=8192), tape=True)
    assert int(r["status"].abs().sum()) == 0
    gx, gu, gp = D.rollout_vjp_params(r["tape"], _t(xb))
    gp = gp.cpu().numpy()
    gx_plain, gu_plain = D.rollout_vjp(r["tape"], _t(xb))
    np.testing.assert_array_equal(gx.cpu().numpy(), gx_plain.cpu().numpy())
    if ctrl:
        np.testing.assert_array_equal(gu.cpu().numpy(), gu_plain.cpu().numpy())
    else:
        _, _, gh = D.rollout_vjp_geom(r["tape"], _t(xb))
        np.testing.assert_array_equal(gp[:, :3], gh.cpu().numpy())
    if ctrl:
        assert not gp[:, :3].any()  # no box geom
    forced, n = tape_steps(r["tape"])

    def central(rel):
        fd = np.zeros((x0.shape[0], len(COLS)))
        for c, j in enumerate(COLS):
            eps = _step(desc, j, rel)
            vals = []
            for s in (+1, -1):
                om = oracle.Model(_shifted(desc, j, s * eps))
                res = om.grad_forced_batch(x0, u, n_int, T / n_int, xb, forced, n, n_threads=6)
                vals.append(np.sum(xb * res["x"], axis=1))
            fd[:, c] = (vals[0] - vals[1]) / (2 * eps)
        return fd

    fd6, fd7 = central(1e-6), central(1e-7)
    g = gp[:, 3:]
    if not ctrl:  # mass: 0 without applied forces, the differences at rounding level
        assert not g[:, 3].any()
        assert np.abs(fd6[:, 3]).max() <= 1e-8, fd6[:, 3]
        keep = [c for c in range(len(COLS)) if c != 3]
        g, fd6, fd7 = g[:, keep], fd6[:, keep], fd7[:, keep]
    scale = np.maximum(np.abs(fd7).max(axis=0, keepdims=True), 1e-12)  # per parameter: units differ
    smooth = np.abs(fd6 - fd7) / scale <= 2e-5
    err = np.abs(g - fd7) / scale
    print(f"{case}: friction/solref/mass/solimp gradient vs oracle differences: max rel err {err[smooth].max():.2e} over "
          f"{int(smooth.sum())}/{smooth.size} converged entries (all entries {err.max():.2e})\n{g}\n{fd7}")
    assert smooth.mean() >= 0.8
    assert err[smooth].max() <= 1e-4
    assert err.max() <= 2e-3


@pytest.mark.parametrize("case", sorted(CASES))
def test_otd_contact_parameter_gradient_is_the_continuous_derivative(D, oracle, case):
    make, height, ctrl = CASES[case]
    desc = make()
    x0 = _sliding_states(4, 5, height)
    T, n_int = 0.08, 2
    model = D.Model(desc)
    rng = np.random.default_rng(6)
    u = rng.uniform(-2.0, 2.0, (x0.shape[0], n_int, model.nu)) if ctrl else None
    xb = np.zeros_like(x0)
    xb[:, 0], xb[:, 2] = 1.0, 2.0
    opts = D.default_opts(rtol=1e-10, atol=1e-10, tape_steps=65536, tape_stages=1)
    r = D.rollout(model, _t(x0), None if u is None else _t(u), n_int, T / n_int, opts=opts, tape=True)
    assert int(r["status"].abs().sum()) == 0
    _, _, p_otd = D.rollout_vjp_otd_params(r["tape"], _t(xb))
    p_otd = p_otd.cpu().numpy()
    if not ctrl:
        _, _, h_otd = D.rollout_vjp_otd_geom(r["tape"], _t(xb))
        np.testing.assert_array_equal(p_otd[:, :3], h_otd.cpu().numpy())
        assert not p_otd[:, 6].any()  # no applied forces
    cols = COLS if ctrl else tuple(j for j in COLS if j != 6)
    g = p_otd[:, list(cols)]
    # the discrete adjoint on the same tape (its parameter gradient is pinned
    # to the oracle above): at rtol 1e-10 both are the continuous derivative
    _, _, p_dto = D.rollout_vjp_params(r["tape"], _t(xb))
    g_dto = p_dto.cpu().numpy()[:, list(cols)]

    def central(rel):
        fd = np.zeros((x0.shape[0], len(cols)))
        for c, j in enumerate(cols):
            eps = _step(desc, j, rel)
            vals = []
            for s in (+1, -1):
                om = oracle.Model(_shifted(desc, j, s * eps))
                res = om.rollout_batch(x0, u, n_int, T / n_int, n_threads=4, rtol=1e-12, atol=1e-12)
                vals.append(np.sum(xb * res["x"], axis=1))
            fd[:, c] = (vals[0] - vals[1]) / (2 * eps)
        return fd

    fd5, fd6 = central(1e-5), central(1e-6)
    scale = np.maximum(np.abs(g_dto).max(axis=0, keepdims=True), 1e-12)
    # solimp d0 at 0 acts through the force step at each contact activation,
    # which the frozen steps of the discrete map resolve differently (that map's
    # d0 derivative, pinned above, departs from the converged differences of
    # the tight forward by up to 0.7%): d0 is held to the differences only
    not_d0 = [c for c, j in enumerate(cols) if j != 7]
    e_dto = np.abs(g - g_dto)[:, not_d0] / scale[:, not_d0]
    # differences of the adaptive forward converge only where no contact or
    # friction state switches within the perturbation
    smooth = np.abs(fd5 - fd6) / scale <= 1e-3
    e_fd = np.abs(g - fd6) / scale
    print(f"{case}: parameter gradient (continuous adjoint) vs discrete adjoint at rtol 1e-10: {e_dto.max():.2e}; "
          f"vs differences at rtol 1e-12: {e_fd[smooth].max() if smooth.any() else float('nan'):.2e} over "
          f"{int(smooth.sum())}/{smooth.size} converged entries\n{g}\n{g_dto}\n{fd6}")
    assert e_dto.max() <= 1e-3
    # the corner cube under controls: the adaptive forward's differences
    # converge for one world of four (3 of 4 change their contact sequence
    # within a relative shift of 1e-5), so the discrete adjoint is the bar there
    assert smooth.sum() >= len(cols)
    assert e_fd[smooth].max() <= 5e-3


def test_side_length_and_friction_identification(D):
    """Joint identification in the manner of App. E.2 (several parameters at
    once, synthetic tosses standing in for the recorded ones): tosses with
    horizontal velocity generated at half size 0.1 m and friction 0.5; Adam
    with a decaying step on the mean squared final-position error, from
    0.12 m and 0.7, recovers both within 1%."""
    import torch
    rng = np.random.default_rng(12)
    n, T = 64, 0.5
    x0 = np.zeros((n, 13))
    x0[:, 2] = rng.uniform(0.2, 0.4, n)
    x0[:, 3:7] = W.uniform_quat(rng, n)
    x0[:, 7:9] = rng.uniform(-2.0, 2.0, (n, 2))
    x0[:, 10:13] = rng.normal(0.0, 3.0, (n, 3))
    true = np.array([0.1, 0.5])

    def desc_of(p):
        d = W.model_box(tc=0.005, mu=p[1])
        d["geoms"][1]["size"] = [p[0]] * 3
        return d

    x0t = _t(x0)
    obs = D.rollout(D.Model(desc_of(true)), x0t, None, 1, T)["x"][:, :3].clone()
    p = np.array([0.12, 0.7])
    lr0 = np.array([4e-3, 2e-2])
    m_, v_ = np.zeros(2), np.zeros(2)
    b1, b2 = 0.9, 0.999
    hist = []
    for it in range(1, 81):
        r = D.rollout(D.Model(desc_of(p)), x0t, None, 1, T, opts=D.default_opts(tape_steps=8192), tape=True)
        assert int(r["status"].abs().sum()) == 0
        d = r["x"][:, :3] - obs
        loss = float((d * d).sum(dim=1).mean())
        xb = torch.zeros_like(x0t)
        xb[:, :3] = 2.0 * d / n
        _, _, gp = D.rollout_vjp_params(r["tape"], xb)
        gp = gp.sum(dim=0).cpu().numpy()
        g = np.array([gp[0] + gp[1] + gp[2], gp[3]])  # one side length; the friction
        m_ = b1 * m_ + (1 - b1) * g
        v_ = b2 * v_ + (1 - b2) * g * g
        lr = lr0 * 0.95 ** (it - 1)
        p = p - lr * (m_ / (1 - b1 ** it)) / (np.sqrt(v_ / (1 - b2 ** it)) + 1e-12)
        hist.append((it, p.copy(), loss))
    for it, pp, loss in hist[::10] + [hist[-1]]:
        print(f"iteration {it}: half size {pp[0]:.5f} m, friction {pp[1]:.4f}, loss {loss:.3e}")
    err = np.abs(p - true) / true
    assert err.max() < 1e-2, p


def test_contact_parameters_outside_their_domain_are_refused(D):
    """Damping ratio 0, a spline power below 1, a midpoint above 1 or an
    impedance of 1 have no finite impedance, stiffness or parameter
    derivatives: model creation refuses them (the free-body and the stack
    paths alike)."""
    bad = [("solref", 1, 0.0), ("solimp", 4, 0.5), ("solimp", 3, 1.5), ("solimp", 0, 1.0), ("cfd", 2, 0.0)]
    for make in (lambda: W.model_box(), lambda: W.model_stack(2)):
        D.Model(make())  # the unmodified model is accepted
        for key, i, v in bad:
            d = make()
            d["pairs"][0][key][i] = v
            with pytest.raises(D.DmxError):
                D.Model(d)


def test_tree_contact_parameter_gradient_matches_oracle_differences(D, oracle):
    """The legged chain (hinge/slide tree, capsule feet on the plane) under
    hinge torques: friction, solref and solimp gradients against the oracle's
    frozen-step differences, as for single bodies; the half-size entries are
    0 (no box geom) and the mass entry NaN (a tree has one mass per body)."""
    n_int, dt = 30, 0.01
    cfg = W.chain_walk(seed=3, n_worlds=6, n_intervals=n_int, interval_dt=dt)
    desc, x0, u = cfg["model"], cfg["x0"], cfg["u"]
    model = D.Model(desc)
    xb = np.zeros_like(x0)
    xb[:, 0], xb[:, 1], xb[:, 2] = 1.0, 2.0, 0.5
    r = D.rollout(model, _t(x0), _t(u), n_int, dt, opts=D.default_opts(tape_steps=8192), tape=True)
    assert int(r["status"].abs().sum()) == 0
    gx, gu, gp = D.rollout_vjp_params(r["tape"], _t(xb))
    gx_plain, gu_plain = D.rollout_vjp(r["tape"], _t(xb))
    np.testing.assert_array_equal(gx.cpu().numpy(), gx_plain.cpu().numpy())
    np.testing.assert_array_equal(gu.cpu().numpy(), gu_plain.cpu().numpy())
    gp = gp.cpu().numpy()
    assert not gp[:, :3].any() and np.isnan(gp[:, 6]).all()
    cols = (3, 4, 5, 7, 8, 9, 10, 11)
    forced, n = tape_steps(r["tape"])

    def central(rel):
        fd = np.zeros((x0.shape[0], len(cols)))
        for c, j in enumerate(cols):
            eps = _step(desc, j, rel)
            vals = []
            for s in (+1, -1):
                om = oracle.Model(_shifted(desc, j, s * eps))
                res = om.grad_forced_batch(x0, u, n_int, dt, xb, forced, n, n_threads=6)
                vals.append(np.sum(xb * res["x"], axis=1))
            fd[:, c] = (vals[0] - vals[1]) / (2 * eps)
        return fd

    fd6, fd7 = central(1e-6), central(1e-7)
    g = gp[:, list(cols)]
    scale = np.maximum(np.abs(fd7).max(axis=0, keepdims=True), 1e-12)
    assert (np.abs(fd7).max(axis=0) > 0).all()  # every parameter acts on the loss
    smooth = np.abs(fd6 - fd7) / scale <= 2e-5
    err = np.abs(g - fd7) / scale
    print(f"chain: friction/solref/solimp gradient vs oracle differences: max rel err {err[smooth].max():.2e} over "
          f"{int(smooth.sum())}/{smooth.size} converged entries (all entries {err.max():.2e})\n{g}\n{fd7}")
    assert smooth.mean() >= 0.8
    assert err[smooth].max() <= 1e-4
    assert err.max() <= 2e-3


def test_tree_otd_contact_parameter_gradient(D, oracle):
    """The legged chain's contact-parameter gradient by the parameter adjoint
    of the continuous adjoint equations (rtol 1e-10) against central
    differences of the oracle's forward at rtol 1e-12 where those converge
    (5e-3 relative to each parameter's largest gradient, as for single
    bodies), and beside the discrete adjoint on the same tape (whose solimp
    derivatives depart from the continuous ones by up to ~2e-3 at contact
    activations; 5e-3); the mass entry is NaN, the half sizes 0."""
    n_int, dt = 30, 0.01
    cfg = W.chain_walk(seed=5, n_worlds=4, n_intervals=n_int, interval_dt=dt)
    desc, x0, u = cfg["model"], cfg["x0"], cfg["u"]
    model = D.Model(desc)
    xb = np.zeros_like(x0)
    xb[:, 0], xb[:, 1] = 1.0, 2.0
    opts = D.default_opts(rtol=1e-10, atol=1e-10, tape_steps=65536, tape_stages=1)
    r = D.rollout(model, _t(x0), _t(u), n_int, dt, opts=opts, tape=True)
    assert int(r["status"].abs().sum()) == 0
    _, _, p_otd = D.rollout_vjp_otd_params(r["tape"], _t(xb))
    _, _, p_dto = D.rollout_vjp_params(r["tape"], _t(xb))
    p_otd, p_dto = p_otd.cpu().numpy(), p_dto.cpu().numpy()
    assert not p_otd[:, :3].any() and np.isnan(p_otd[:, 6]).all()
    cols = [3, 4, 5, 7, 8, 9, 10, 11]

    def central(rel):
        fd = np.zeros((x0.shape[0], len(cols)))
        for c, j in enumerate(cols):
            eps = _step(desc, j, rel)
            vals = []
            for sg in (+1, -1):
                om = oracle.Model(_shifted(desc, j, sg * eps))
                res = om.rollout_batch(x0, u, n_int, dt, n_threads=4, rtol=1e-12, atol=1e-12)
                vals.append(np.sum(xb * res["x"], axis=1))
            fd[:, c] = (vals[0] - vals[1]) / (2 * eps)
        return fd

    fd5, fd6 = central(1e-5), central(1e-6)
    g = p_otd[:, cols]
    scale = np.maximum(np.abs(p_dto[:, cols]).max(axis=0, keepdims=True), 1e-12)
    smooth = np.abs(fd5 - fd6) / scale <= 1e-3
    e_fd = np.abs(g - fd6) / scale
    not_d0 = [c for c, j in enumerate(cols) if j != 7]
    e_dto = (np.abs(g - p_dto[:, cols]) / scale)[:, not_d0]
    print(f"chain: parameter gradient (continuous adjoint) vs differences at rtol 1e-12: "
          f"{e_fd[smooth].max() if smooth.any() else float('nan'):.2e} over {int(smooth.sum())}/{smooth.size} "
          f"converged entries; vs the discrete adjoint: {e_dto.max():.2e}\n{g}\n{fd6}")
    assert smooth.sum() >= len(cols)
    assert e_fd[smooth].max() <= 5e-3
    assert e_dto.max() <= 5e-3


def test_stack_parameter_gradient_matches_oracle_differences(D, oracle):
    """Stack worlds (an uneven batch of 2- and 3-cube stacks, a control force
    and torque on the top cube): friction, solref, solimp and the cubes'
    common mass through the stack reverse sweep, against the oracle's
    frozen-step differences as for single bodies; the half sizes are NaN (not
    differentiated in stack worlds), the state and control gradients are
    bitwise the plain sweep's."""
    ks = (2, 3)
    rng = np.random.default_rng(9)
    descs = [W.model_stack(k, ctrl=True) for k in ks]
    xs = [W.stack_state(rng.normal(0.0, 0.02, size=(k, 2))) for k in ks]
    us = [rng.uniform(-2.0, 2.0, size=(1, 6)) for _ in ks]
    T = 0.05
    models = [D.Model(d) for d in descs]
    res = D.rollout_batch(models, _t(np.concatenate(xs)), _t(np.concatenate([u.ravel() for u in us])), 1, T,
                          opts=D.default_opts(tape_steps=8192), tape=True)
    assert (res["status"].cpu().numpy() == 0).all()
    xbs = [np.concatenate([np.tile([1.0, 0.5, 2.0, 0, 0, 0, 0], k), np.zeros(6 * k)]) for k in ks]
    xb = _t(np.concatenate(xbs))
    gx, gu, gp = D.rollout_batch_vjp_params(res["tape"], xb)
    gx0, gu0 = D.rollout_batch_vjp(res["tape"], xb)
    np.testing.assert_array_equal(gx.cpu().numpy(), gx0.cpu().numpy())
    np.testing.assert_array_equal(gu.cpu().numpy(), gu0.cpu().numpy())
    gp = gp.cpu().numpy()
    assert np.isnan(gp[:, :3]).all()
    recs, n = res["tape"].world_records()
    cols = (3, 4, 5, 6, 7, 8, 9, 10, 11)

    def central(rel):
        fd = np.zeros((len(ks), len(cols)))
        for w in range(len(ks)):
            forced = np.ascontiguousarray(recs[w][:, :2])[None]
            for c, j in enumerate(cols):
                eps = _step(descs[w], j, rel)
                vals = []
                for sg in (+1, -1):
                    om = oracle.Model(_shifted(descs[w], j, sg * eps))
                    r = om.grad_forced_batch(xs[w][None], us[w][None], 1, T, xbs[w][None], forced,
                                             np.array([n[w]], np.int32), n_threads=1)
                    vals.append(float(np.sum(xbs[w] * r["x"][0])))
                fd[w, c] = (vals[0] - vals[1]) / (2 * eps)
        return fd

    fd6, fd7 = central(1e-6), central(1e-7)
    g = gp[:, list(cols)]
    scale = np.maximum(np.abs(fd7).max(axis=0, keepdims=True), 1e-12)
    smooth = np.abs(fd6 - fd7) / scale <= 2e-5
    err = np.abs(g - fd7) / scale
    print(f"stacks: friction/solref/mass/solimp gradient vs oracle differences: max rel err {err[smooth].max():.2e} "
          f"over {int(smooth.sum())}/{smooth.size} converged entries (all entries {err.max():.2e})\n{g}\n{fd7}")
    assert smooth.mean() >= 0.8
    assert err[smooth].max() <= 1e-4
    assert err.max() <= 2e-3


def test_stack_friction_identification(D):
    """Friction identified from stacks (the parameter-gradient path of stack
    batches in use): 2-cube stacks whose top cube is pushed sideways past the
    friction limit; synthetic final positions generated at mu 0.6; a
    sign-based step (Rprop: the step grows by 1.2 while the gradient keeps its
    sign and halves when it flips) on their mean squared error recovers mu
    within 1% from 0.4."""
    import torch
    rng = np.random.default_rng(21)
    n, T, true_mu = 16, 0.3, 0.6
    xs = [W.stack_state(rng.normal(0.0, 0.005, size=(2, 2))) for _ in range(n)]
    u = np.zeros((n, 6))
    ang = rng.uniform(0.0, 2.0 * np.pi, n)
    mag = rng.uniform(7.0, 10.0, n)  # past mu m g = 5.9 N at the true friction
    u[:, 0], u[:, 1] = mag * np.cos(ang), mag * np.sin(ang)
    x0t, ut = _t(np.concatenate(xs)), _t(u.ravel())
    top = (7, 8, 9)  # the top cube's position in a world's 26 state doubles
    sel = torch.tensor([26 * w + t for w in range(n) for t in top], device="cuda")

    def run(mu, tape=False):
        models = [D.Model(W.model_stack(2, mu=mu, ctrl=True))] * n
        return D.rollout_batch(models, x0t, ut, 1, T, opts=D.default_opts(tape_steps=8192), tape=tape)

    obs = run(true_mu)["x"][sel].clone()
    mu, step, g_prev = 0.4, 0.05, 0.0
    hist = []
    for it in range(1, 41):
        r = run(mu, tape=True)
        assert int(r["status"].abs().sum()) == 0
        d = r["x"][sel] - obs
        loss = float((d * d).sum() / n)
        xb = torch.zeros_like(x0t)
        xb[sel] = 2.0 * d / n
        _, _, gp = D.rollout_batch_vjp_params(r["tape"], xb)
        g = float(gp[:, 3].sum())
        step = step * 0.5 if g * g_prev < 0.0 else step * 1.2
        mu -= np.sign(g) * step
        g_prev = g
        hist.append((it, mu, loss))
    for it, mm, loss in hist[::10] + [hist[-1]]:
        print(f"iteration {it}: friction {mm:.4f}, loss {loss:.3e}")
    assert abs(mu - true_mu) / true_mu < 1e-2, mu
