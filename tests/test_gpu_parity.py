"""Parity of the HIP library (through its C ABI) with the oracle.

Tolerances: an acceleration F(x) at the same state agrees to 1e-10; a GPU step
fed the oracle's step and state agrees to 1e-10 relative; a whole replayed step
sequence to 1e-6 (stiff contact at large steps amplifies rounding differences
along a trajectory); end states to 1e-6; gradients to 1e-5, normwise and
element by element (relative, per world: |dq|/max(|q|,1), |dv|/max(|v|,1e-3),
|dg|/max(|g|,1e-12); entries |dg_i|/max(|g_i|, 1e-3 |g|_inf)).  Free runs use
the paper's continuous PI controller: each GPU run's accepted-step sequence is
replayed by the oracle (end state and gradient), and each attempt's
accept/reject decision and proposed step are checked against the oracle's
error estimate and controller (tests/replay_check.py).  The opt-in step grid
(h_levels) is checked separately.
"""
import numpy as np
import pytest

from paper_2506_14186_amd import workloads as W
from replay_check import (GRAD_TOL, STATE_TOL, check_decisions_and_controller, elementwise_grad, rel_grad, rel_state,
                          replay_and_compare, tape_steps)

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


def _sphere_batch(seeds):
    x0 = np.concatenate([W.sphere_drop(seed=s)["x0"] for s in seeds])
    return W.model_sphere(), x0, 1, 1.0


def _cube_batch(n, horizon=0.5, seed=2):
    cfg = W.cube_toss(seed=seed, n_worlds=n, horizon=horizon)
    return cfg["model"], cfg["x0"], 1, horizon


def _box_batch(n, horizon=0.5, seed=4):
    cfg = W.box_toss(seed=seed, n_worlds=n, horizon=horizon)
    return cfg["model"], cfg["x0"], 1, horizon


CASES = {"sphere": lambda: _sphere_batch([1, 2, 3, 4]), "cube": lambda: _cube_batch(6), "box": lambda: _box_batch(6)}
FREE_CASES = {"sphere": lambda: _sphere_batch([1, 2, 3, 4, 5, 6]), "cube": lambda: _cube_batch(16),
              "box": lambda: _box_batch(16)}
# (case, lanes per world): 0 = the library's default team, which for the cube
# (8 contact slots, 16 lanes) and the box geom (4 slots, 8 lanes) holds each
# contact on two lanes; the cube and the box also with one lane per slot
CASE_LANES = [(c, 0) for c in CASES] + [("cube", 8), ("box", 4)]
FREE_CASE_LANES = [(c, 0) for c in FREE_CASES] + [("cube", 8)]


@pytest.mark.parametrize("case", ["cube", "box"])
def test_accel_parity(D, oracle, case):
    """F(x) at states along oracle trajectories (contacts on and off)."""
    desc, x0, n_int, dt = _cube_batch(6) if case == "cube" else _box_batch(6)
    om, tapes = _oracle_tapes(oracle, desc, x0, n_int, dt)
    ys = np.vstack([r["tape"][:, 2:] for r in tapes])
    model = D.Model(desc)
    acc, st = D.accel(model, _t(ys))
    assert int(st.abs().sum()) == 0
    ref = np.stack([om.rhs(y)[0][6:] for y in ys])
    scale = np.maximum(np.linalg.norm(ref, axis=1), 1e-3)
    err = np.linalg.norm(acc.cpu().numpy() - ref, axis=1) / scale
    nc = sum(om.rhs(y)[1]["n_rows"] > 0 for y in ys)
    # conditioning of F at each state, from the oracle itself: the change of F
    # under relative state perturbations of a few ulp (the top-four vertex
    # choice of the plane-box detection is discontinuous where two vertices
    # tie, and the soft mask is steep): the two sides may differ by that much
    sens = _rhs_sensitivity(om, ys, ref, scale)
    tol = np.maximum(1e-10, 10.0 * sens)
    print(f"{case} accel: {len(ys)} states ({nc} in contact), max rel err {err.max():.3e}; "
          f"{int((sens > 1e-11).sum())} states where F moves by more than 1e-11 under 4-ulp perturbations "
          f"(max {sens.max():.1e}); max err/tol {(err / tol).max():.2f}")
    assert (err <= tol).all()


def _rhs_sensitivity(om, ys, ref, scale, reps=4, seed=3):
    rng = np.random.default_rng(seed)
    sens = np.zeros(len(ys))
    for _ in range(reps):
        for i, y in enumerate(ys):
            yp = y * (1.0 + 4.4e-16 * rng.choice([-1.0, 1.0], size=y.shape))
            sens[i] = max(sens[i], np.linalg.norm(om.rhs(yp)[0][6:] - ref[i]) / scale[i])
    return sens


def _oracle_tapes(oracle, desc, x0, n_int, dt):
    om = oracle.Model(desc)
    out = []
    for w in range(x0.shape[0]):
        r = om.rollout(x0[w], None, n_int, dt, tape_cap=200000)
        assert r["status"] == 0
        out.append(r)
    return om, out


@pytest.mark.parametrize("case,lanes", CASE_LANES)
def test_single_step_parity(D, oracle, case, lanes):
    """Every oracle step replayed as an independent one-step GPU world."""
    desc, x0, n_int, dt = CASES[case]()
    om, tapes = _oracle_tapes(oracle, desc, x0, n_int, dt)
    ys, hs, nxt = [], [], []
    for r in tapes:
        tp = r["tape"]
        y_next = np.vstack([tp[1:, 2:], r["x"][None]])
        ys.append(tp[:, 2:]); hs.append(tp[:, 1]); nxt.append(y_next)
    ys, hs, nxt = np.vstack(ys), np.concatenate(hs), np.vstack(nxt)
    model = D.Model(desc)
    Wn = ys.shape[0]
    forced = np.zeros((Wn, 1, 2))
    forced[:, 0, 1] = hs
    f_t, fn = _t(forced), _t(np.ones(Wn)).int()
    o = D.default_opts(forced=f_t.data_ptr(), forced_n=fn.data_ptr(), forced_cap=1, lanes_per_world=lanes)
    res = D.rollout(model, _t(ys), None, 1, 10.0, opts=o)
    assert int(res["status"].abs().sum()) == 0
    err = rel_state(res["x"].cpu().numpy(), nxt, model.nq)
    # conditioning of the one-step map at each state, from the oracle (see
    # test_accel_parity): steps whose result moves under 4-ulp perturbations
    # of the state may differ by that much
    rng = np.random.default_rng(5)
    sens = np.zeros(Wn)
    if case == "box":
        for _ in range(3):
            for i in range(Wn):
                yp = ys[i] * (1.0 + 4.4e-16 * rng.choice([-1.0, 1.0], size=ys[i].shape))
                r1 = om.rollout(yp, None, 1, 10.0, forced=[[0.0, hs[i]]])
                sens[i] = max(sens[i], rel_state(r1["x"], nxt[i], model.nq)[0])
    tol = np.maximum(1e-10, 10.0 * sens)
    print(f"{case} (lanes {lanes or 'default'}): {Wn} single steps, max rel err {err.max():.3e}; "
          f"{int((sens > 1e-11).sum())} ill-conditioned "
          f"steps (max {sens.max():.1e}); max err/tol {(err / tol).max():.2f}")
    assert (err <= tol).all()


@pytest.mark.parametrize("case", list(CASES))
def test_replayed_sequence_parity(D, oracle, case):
    desc, x0, n_int, dt = CASES[case]()
    om, tapes = _oracle_tapes(oracle, desc, x0, n_int, dt)
    model = D.Model(desc)
    cap = max(r["n_acc"] for r in tapes)
    forced = np.zeros((x0.shape[0], cap, 2))
    fn = np.zeros(x0.shape[0])
    for w, r in enumerate(tapes):
        forced[w, :r["n_acc"]] = r["tape"][:, :2]
        fn[w] = r["n_acc"]
    f_t, fn_t = _t(forced), _t(fn).int()
    o = D.default_opts(forced=f_t.data_ptr(), forced_n=fn_t.data_ptr(), forced_cap=cap, tape_steps=cap + 8)
    res = D.rollout(model, _t(x0), None, n_int, dt, opts=o, tape=True)
    assert int(res["status"].abs().sum()) == 0
    recs, n = res["tape"].records()
    worst = 0.0
    for w, r in enumerate(tapes):
        assert n[w] == r["n_acc"]
        e = rel_state(recs[w, :n[w], 3:3 + model.nx], r["tape"][:, 2:], model.nq)
        worst = max(worst, e.max())
        np.testing.assert_array_equal(recs[w, :n[w], :2], r["tape"][:, :2])
    ef = rel_state(res["x"].cpu().numpy(), np.stack([r["x"] for r in tapes]), model.nq)
    print(f"{case}: replayed {int(fn.sum())} steps, max per-step rel err {worst:.3e}, final {ef.max():.3e}")
    assert worst <= 1e-6 and ef.max() <= 1e-6


def _steplog_opts(D, W, cap, **kw):
    import torch
    log = torch.zeros((W, cap, 4), dtype=torch.float64, device="cuda")
    logn = torch.zeros(W, dtype=torch.int32, device="cuda")
    return D.default_opts(steplog=log.data_ptr(), log_n=logn.data_ptr(), log_cap=cap, **kw), (log, logn)


def _free_run_checked(D, oracle, desc, x0, u, n_int, dt, xbar, lanes=0, levels=0, label="", decisions=None):
    """A free GPU run (the paper's continuous controller unless levels > 0),
    checked against the oracle replay of its own accepted steps and, for the
    worlds in `decisions` (default all), attempt by attempt."""
    om = oracle.Model(desc)
    model = D.Model(desc)
    Wn = x0.shape[0]
    o, (log, logn) = _steplog_opts(D, Wn, 8192, lanes_per_world=lanes, h_levels=levels, tape_steps=8192)
    ut = _t(u) if model.nu else None
    res = D.rollout(model, _t(x0), ut, n_int, dt, opts=o, tape=True, counters=True)
    assert int(res["status"].abs().sum()) == 0
    gx, gu = D.rollout_vjp(res["tape"], _t(xbar))
    forced, n = tape_steps(res["tape"])
    uu = u if model.nu else None
    cmp = replay_and_compare(om, model.nq, x0, uu, n_int, dt, res["x"].cpu().numpy(), forced, n, xbar,
                             gx.cpu().numpy(), None if gu is None else gu.cpu().numpy(), h_levels=levels)
    logs, logn = log.cpu().numpy(), logn.cpu().numpy()
    assert (logn < 8192).all()
    checked, bad_dec, by_rounding, max_rel, bad_ctrl = check_decisions_and_controller(
        oracle, om, x0, uu, n_int, dt, res["tape"].records()[0], n, logs, logn, worlds=decisions, h_levels=levels)
    print(f"{label} (lanes {lanes or 'default'}, levels {levels}): accepted steps {n.tolist() if Wn <= 32 else n.mean()}; "
          f"replay: state {cmp['state'].max():.2e}, grad {cmp['grad'].max():.2e} (element-wise "
          f"{cmp['grad_elem'].max():.2e}); {checked} attempts: {bad_dec} decisions differ outside the rounding band "
          f"({by_rounding} decided by rounding), error estimates agree to {max_rel:.1e}, {bad_ctrl} proposed steps "
          f"differ from the oracle controller")
    assert cmp["state"].max() <= STATE_TOL
    assert cmp["grad"].max() <= GRAD_TOL and cmp["grad_elem"].max() <= GRAD_TOL
    assert bad_dec == 0 and bad_ctrl == 0
    return res, n, cmp


@pytest.mark.parametrize("case,lanes", FREE_CASE_LANES)
def test_free_adaptive_parity_and_gradient(D, oracle, case, lanes):
    """Free runs under the paper's continuous PI controller, every world
    checked: end state and gradient against the oracle replay of the GPU's
    accepted steps, and every attempt's decision and proposed step."""
    desc, x0, n_int, dt = FREE_CASES[case]()
    xbar = np.zeros_like(x0)
    # summed final position (for the sphere the final height alone would be a
    # vanishing cotangent: the ball rests after 1 s and its height no longer
    # depends on the start, both sides return rounding noise of ~1e-20; the
    # rolling distance does depend on it)
    xbar[:, 0:3] = 1.0
    _free_run_checked(D, oracle, desc, x0, np.zeros((x0.shape[0], n_int, 0)), n_int, dt, xbar, lanes=lanes,
                      label=case)


@pytest.mark.parametrize("levels", [0, 16])
def test_free_run_full_horizon(D, oracle, levels):
    """Full 0.5 s free runs of 32 tumbling cubes, every world checked through
    the replay of its GPU step sequence (continuous controller and the opt-in
    step grid).  On the grid the two sides' own free runs also take the same
    steps; how many do is reported for both settings."""
    desc, x0, n_int, dt = _cube_batch(32)
    xbar = np.zeros_like(x0)
    xbar[:, :3] = 1.0
    res, n, cmp = _free_run_checked(D, oracle, desc, x0, np.zeros((32, 1, 0)), n_int, dt, xbar, levels=levels,
                                    label="32 cubes 0.5 s")
    om = oracle.Model(desc)
    ref = om.rollout_batch(x0, None, n_int, dt, n_threads=8, h_levels=levels)
    same = n == ref["n_acc"]
    ex = rel_state(res["x"].cpu().numpy(), ref["x"], 7)
    print(f"levels {levels}: own free runs of both sides: {int(same.sum())}/32 equal accepted-step counts, "
          f"{int((ex <= 1e-6).sum())}/32 end states within 1e-6 (median {np.median(ex):.1e})")
    if levels:
        assert ex[same].max() <= 1e-6


@pytest.mark.parametrize("case,lanes", [("cube", 0), ("box", 0), ("cube", 8)])
def test_replayed_gradient_matches_oracle_tightly(D, oracle, case, lanes):
    """Same step sequence on both sides: the reverse sweep equals the
    forward-mode derivative of the oracle to rounding."""
    desc, x0, n_int, dt = _cube_batch(4, horizon=0.3) if case == "cube" else _box_batch(4, horizon=0.6)
    om, tapes = _oracle_tapes(oracle, desc, x0, n_int, dt)
    model = D.Model(desc)
    cap = max(r["n_acc"] for r in tapes)
    forced = np.zeros((x0.shape[0], cap, 2))
    fn = np.zeros(x0.shape[0])
    for w, r in enumerate(tapes):
        forced[w, :r["n_acc"]] = r["tape"][:, :2]
        fn[w] = r["n_acc"]
    f_t, fn_t = _t(forced), _t(fn).int()
    o = D.default_opts(forced=f_t.data_ptr(), forced_n=fn_t.data_ptr(), forced_cap=cap, tape_steps=cap + 8,
                       lanes_per_world=lanes)
    res = D.rollout(model, _t(x0), None, n_int, dt, opts=o, tape=True)
    rng = np.random.default_rng(7)
    xbar = rng.normal(size=x0.shape)
    g, _ = D.rollout_vjp(res["tape"], _t(xbar))
    ref = om.grad_batch(x0, None, n_int, dt, xbar, n_threads=4)
    eg = rel_grad(g.cpu().numpy(), ref["x0bar"])
    print(f"{case} (lanes {lanes or 'default'}): replayed-sequence gradient rel err {eg.max():.3e}")
    assert eg.max() <= 1e-8


def test_batch_and_team_invariance(D):
    desc, x0, n_int, dt = _cube_batch(37, horizon=0.2)
    model = D.Model(desc)
    xbar = np.zeros_like(x0)
    xbar[:, :3] = 1.0
    full = D.rollout(model, _t(x0), None, n_int, dt, tape=True)
    gfull, _ = D.rollout_vjp(full["tape"], _t(xbar))
    for w in (0, 17, 36):
        one = D.rollout(model, _t(x0[w:w + 1]), None, n_int, dt, tape=True)
        g1, _ = D.rollout_vjp(one["tape"], _t(xbar[w:w + 1]))
        np.testing.assert_array_equal(one["x"].cpu().numpy()[0], full["x"].cpu().numpy()[w])
        np.testing.assert_array_equal(g1.cpu().numpy()[0], gfull.cpu().numpy()[w])
    # other team sizes, replaying the default team size's step sequence
    recs, n = full["tape"].records()
    cap = int(n.max())
    forced = np.ascontiguousarray(recs[:, :cap, :2])
    f_t, fn_t = _t(forced), _t(n.astype(np.float64)).int()
    ref = full["x"].cpu().numpy()
    for L in (1, 2, 4, 8, 16):
        o = D.default_opts(lanes_per_world=L, forced=f_t.data_ptr(), forced_n=fn_t.data_ptr(), forced_cap=cap)
        r = D.rollout(model, _t(x0), None, n_int, dt, opts=o)
        e = rel_state(r["x"].cpu().numpy(), ref, model.nq)
        print(f"lanes per world {L}: max rel err vs the default team {e.max():.2e}")
        assert e.max() <= 1e-6, (L, e.max())


def test_edge_cases(D):
    import torch
    desc, x0, n_int, dt = _cube_batch(5, horizon=0.2)
    model = D.Model(desc)
    # empty batch
    r = D.rollout(model, _t(np.zeros((0, 13))), None, n_int, dt)
    assert r["x"].shape == (0, 13)
    # ragged batch (5 worlds, 8-lane teams) and a non-finite world
    bad = x0.copy()
    bad[3, 9] = np.nan
    r = D.rollout(model, _t(bad), None, n_int, dt, tape=True)
    st = r["status"].cpu().numpy()
    assert st[3] & D.STATUS["NONFINITE"] and (np.delete(st, 3) == 0).all()
    g, _ = D.rollout_vjp(r["tape"], _t(np.ones_like(bad)))
    g = g.cpu().numpy()
    assert np.isnan(g[3]).all() and np.isfinite(np.delete(g, 3, axis=0)).all()
    # step budget and tape capacity
    r = D.rollout(model, _t(x0), None, n_int, dt, opts=D.default_opts(max_attempts=3))
    assert (r["status"].cpu().numpy() & D.STATUS["MAX_STEPS"]).all()
    r = D.rollout(model, _t(x0), None, n_int, dt, opts=D.default_opts(tape_steps=4), tape=True)
    assert (r["status"].cpu().numpy() & D.STATUS["TAPE_OVERFLOW"]).all()
    g, _ = D.rollout_vjp(r["tape"], _t(np.ones_like(x0)))
    assert torch.isnan(g).all()
    # API errors are reported, not launched
    with pytest.raises(D.DmxError):  # a free joint below another body is not a compiled model shape
        desc2 = W.model_free_box()
        desc2["bodies"].append({"parent": 0, "pos": [0, 0, 0.3], "quat": [1, 0, 0, 0],
                                "inertial": {"type": "sphere", "size": [0.05, 0, 0], "mass": 1.0},
                                "joints": [{"type": "hinge", "axis": [1, 0, 0], "pos": [0, 0, 0]}]})
        D.Model(desc2)
    with pytest.raises(D.DmxError):
        D.rollout(model, _t(x0), None, 0, dt)


def test_autograd_function_matches_vjp(D):
    import torch
    desc, x0, n_int, dt = _cube_batch(3, horizon=0.15)
    model = D.Model(desc)
    xt = _t(x0).requires_grad_(True)
    x, st = D.Rollout.apply(xt, None, model, n_int, dt, D.default_opts())
    loss = x[:, :3].sum()
    loss.backward()
    r = D.rollout(model, _t(x0), None, n_int, dt, tape=True)
    xbar = torch.zeros_like(r["x"])
    xbar[:, :3] = 1.0
    g, _ = D.rollout_vjp(r["tape"], xbar)
    np.testing.assert_array_equal(xt.grad.cpu().numpy(), g.cpu().numpy())


def test_cfd_straight_through(D, oracle):
    """Straight-through CFD: forward unchanged, gradient equals the oracle's
    forward-mode derivative of the CFD field along the same trajectory.  The
    spheres fall to within w_c = 1 cm of the plane without touching (CFD
    rows active only in the gradient), and one lands (contact rows too)."""
    desc = W.model_sphere()
    x0 = np.array([[0.0, 0.0, 0.13, 1, 0, 0, 0, 0.3, 0.0, 0.0, 0, 0, 0],
                   [0.0, 0.0, 0.125, 1, 0, 0, 0, -0.2, 0.1, 0.0, 0, 0, 0],
                   [0.0, 0.0, 0.11, 1, 0, 0, 0, 0.1, 0.0, -0.2, 0, 0, 0]])
    n_int, dt = 1, 0.07
    model = D.Model(desc)
    om = oracle.Model(desc)
    xbar = np.zeros_like(x0)
    xbar[:, 0] = 1.0
    xbar[:, 2] = 1.0
    a = D.rollout(model, _t(x0), None, n_int, dt, tape=True)
    b = D.rollout(model, _t(x0), None, n_int, dt, tape=True, opts=D.default_opts(cfd=1))
    np.testing.assert_array_equal(a["x"].cpu().numpy(), b["x"].cpu().numpy())
    g, _ = D.rollout_vjp(b["tape"], _t(xbar))
    forced, n = tape_steps(b["tape"])
    ref = om.grad_forced_batch(x0, None, n_int, dt, xbar, forced, n, n_threads=3, cfd=1)
    plain = om.grad_forced_batch(x0, None, n_int, dt, xbar, forced, n, n_threads=3, cfd=0)
    eg = rel_grad(g.cpu().numpy(), ref["x0bar"])
    ee = elementwise_grad(g.cpu().numpy(), ref["x0bar"])
    print(f"cfd gradient rel err {eg.max():.3e} (element-wise {ee.max():.2e}); dz/dz0 with CFD "
          f"{ref['x0bar'][:, 2]}, without {plain['x0bar'][:, 2]}")
    assert eg.max() <= 1e-5 and ee.max() <= 1e-5
    assert abs(ref["x0bar"][0, 2] - plain["x0bar"][0, 2]) > 1e-3  # CFD informs the non-touching sphere


@pytest.mark.parametrize("lanes", [0, 8])
def test_cfd_straight_through_cube(D, oracle, lanes):
    """The straight-through CFD gradient of tumbling cubes (8 corner slots,
    CFD rows for corners within w_c of the plane), on the oracle's step
    sequences, for the default team (two lanes per contact) and 8-lane teams
    (one lane per contact)."""
    desc, x0, n_int, dt = _cube_batch(4, horizon=0.3)
    om, tapes = _oracle_tapes(oracle, desc, x0, n_int, dt)
    model = D.Model(desc)
    cap = max(r["n_acc"] for r in tapes)
    forced = np.zeros((x0.shape[0], cap, 2))
    fn = np.zeros(x0.shape[0])
    for w, r in enumerate(tapes):
        forced[w, :r["n_acc"]] = r["tape"][:, :2]
        fn[w] = r["n_acc"]
    f_t, fn_t = _t(forced), _t(fn).int()
    o = D.default_opts(forced=f_t.data_ptr(), forced_n=fn_t.data_ptr(), forced_cap=cap, tape_steps=cap + 8,
                       lanes_per_world=lanes, cfd=1)
    res = D.rollout(model, _t(x0), None, n_int, dt, opts=o, tape=True)
    assert int(res["status"].abs().sum()) == 0
    rng = np.random.default_rng(11)
    xbar = rng.normal(size=x0.shape)
    g, _ = D.rollout_vjp(res["tape"], _t(xbar))
    ref = om.grad_forced_batch(x0, None, n_int, dt, xbar, forced, fn.astype(np.int32), n_threads=4, cfd=1)
    eg = rel_grad(g.cpu().numpy(), ref["x0bar"])
    ee = elementwise_grad(g.cpu().numpy(), ref["x0bar"])
    print(f"cube cfd (lanes {lanes or 'default'}): replayed-sequence gradient rel err {eg.max():.3e} "
          f"(element-wise {ee.max():.2e})")
    assert eg.max() <= 1e-5 and ee.max() <= 1e-5


@pytest.mark.parametrize("case", ["box", "chain"])
def test_cfd_straight_through_box_and_tree(D, oracle, case):
    """The straight-through CFD gradient of the box geom (smoothed plane-box
    rows within w_c) and of the legged chain (foot capsules within w_c), on
    the GPU's own step sequences replayed by the oracle."""
    if case == "box":
        desc, x0, n_int, dt = _box_batch(4, horizon=0.4)
        u = np.zeros((4, 1, 0))
    else:
        desc, x0, u, n_int, dt = _chain(n_worlds=3, n_int=8)
    model = D.Model(desc)
    om = oracle.Model(desc)
    ut = _t(u) if model.nu else None
    res = D.rollout(model, _t(x0), ut, n_int, dt, opts=D.default_opts(cfd=1, tape_steps=8192), tape=True)
    assert int(res["status"].abs().sum()) == 0
    rng = np.random.default_rng(12)
    xbar = rng.normal(size=x0.shape)
    gx, gu = D.rollout_vjp(res["tape"], _t(xbar))
    forced, n = tape_steps(res["tape"])
    cmp = replay_and_compare(om, model.nq, x0, u if model.nu else None, n_int, dt, res["x"].cpu().numpy(), forced,
                             n, xbar, gx.cpu().numpy(), None if gu is None else gu.cpu().numpy(), cfd=1)
    plain = om.grad_forced_batch(x0, u if model.nu else None, n_int, dt, xbar, forced, n, n_threads=4, cfd=0)
    moved = rel_grad(cmp["ref"]["x0bar"], plain["x0bar"])
    print(f"{case} cfd: steps {n.tolist()}; state {cmp['state'].max():.2e}, gradient {cmp['grad'].max():.2e} "
          f"(element-wise {cmp['grad_elem'].max():.2e}); CFD changes the x0 gradient by {moved.max():.2e}")
    assert cmp["state"].max() <= STATE_TOL
    assert cmp["grad"].max() <= GRAD_TOL and cmp["grad_elem"].max() <= GRAD_TOL
    assert moved.max() > 1e-6  # the CFD rows take part in the gradient


@pytest.mark.parametrize("lanes", [0, 8])
def test_full_size_cube_sampled(D, oracle, lanes):
    """The measured configuration (4096 cube worlds, 0.5 s, one launch; the
    default 16-lane teams, which the benchmark's autotuner also picks, and
    8-lane teams):
    every world finishes; then the same launch replays, for 8 sampled worlds,
    the oracle's step sequences (the other worlds replay their own), and the
    sampled end states and gradients match the oracle's."""
    cfg = W.cube_toss(seed=2, n_worlds=4096, horizon=0.5)
    model = D.Model(cfg["model"])
    x0 = cfg["x0"]
    xbar = np.zeros_like(x0)
    xbar[:, :3] = 1.0
    res = D.rollout(model, _t(x0), None, 1, 0.5, tape=True, counters=True,
                    opts=D.default_opts(tape_steps=2048, lanes_per_world=lanes))
    assert int(res["status"].abs().sum()) == 0
    g, _ = D.rollout_vjp(res["tape"], _t(xbar))
    assert np.isfinite(g.cpu().numpy()).all()
    nacc = res["n_acc"].cpu().numpy()
    recs, n = res["tape"].records()
    n_att = nacc + res["n_rej"].cpu().numpy()
    hardest = [int(w) for w in np.argsort(-n_att, kind="stable")[:5]]
    sample = sorted(set([0, 1, 777, 1500, 2048, 3000, 4000, 4095] + hardest))
    om = oracle.Model(cfg["model"])
    ref_tapes = [om.rollout(x0[w], None, 1, 0.5, tape_cap=5000) for w in sample]
    cap = max(int(n.max()), max(r["n_acc"] for r in ref_tapes))
    forced = np.zeros((4096, cap, 2))
    forced[:, :recs.shape[1]] = recs[:, :cap, :2]
    fn = n.astype(np.float64).copy()
    for i, w in enumerate(sample):
        forced[w] = 0.0
        forced[w, :ref_tapes[i]["n_acc"]] = ref_tapes[i]["tape"][:, :2]
        fn[w] = ref_tapes[i]["n_acc"]
    f_t, fn_t = _t(forced), _t(fn).int()
    o = D.default_opts(forced=f_t.data_ptr(), forced_n=fn_t.data_ptr(), forced_cap=cap, tape_steps=cap + 8,
                       lanes_per_world=lanes)
    rep = D.rollout(model, _t(x0), None, 1, 0.5, tape=True, opts=o)
    assert int(rep["status"].abs().sum()) == 0
    gr, _ = D.rollout_vjp(rep["tape"], _t(xbar))
    ref = om.grad_batch(x0[sample], None, 1, 0.5, xbar[sample], n_threads=8)
    ex = rel_state(rep["x"].cpu().numpy()[sample], ref["x"], model.nq)
    eg = rel_grad(gr.cpu().numpy()[sample], ref["x0bar"])
    ee = elementwise_grad(gr.cpu().numpy()[sample], ref["x0bar"])
    print(f"4096 worlds (lanes {lanes or 'default'}): accepted steps mean {nacc.mean():.0f} max {nacc.max()}; "
          f"hardest worlds {hardest} ({n_att[hardest].tolist()} attempts); sampled replay state err "
          f"{ex.max():.2e} grad err {eg.max():.2e} (element-wise {ee.max():.2e})")
    assert ex.max() <= 1e-6 and eg.max() <= 1e-5 and ee.max() <= 1e-5


def test_full_size_chain_sampled(D, oracle):
    """The legged-chain configuration at full size (16384 worlds, 200
    intervals of 10 ms, random torques; one persistent launch, default team):
    every world finishes; the launch then replays, for 3 sampled worlds, the
    oracle's step sequences, and the sampled end states match the oracle's and
    the reverse sweep's x0/u cotangents match the oracle's forward-mode
    derivatives along 16 sampled directions (x0 and u entries)."""
    import torch
    cfg = W.chain_walk(n_worlds=16384, n_intervals=200)
    model = D.Model(cfg["model"])
    x0, u, H, dt = cfg["x0"], cfg["u"], cfg["n_intervals"], cfg["interval_dt"]
    res = D.rollout(model, _t(x0), _t(u), H, dt, tape=True, counters=True,
                    opts=D.default_opts(tape_steps=40 * H + 64))
    assert int(res["status"].abs().sum()) == 0
    nacc = res["n_acc"].cpu().numpy()
    recs_n = res["tape"].info()
    del res
    torch.cuda.empty_cache()
    sample = [0, 8191, 16383]
    om = oracle.Model(cfg["model"])
    ref_tapes = [om.rollout(x0[w], u[w], H, dt, tape_cap=40 * H + 64) for w in sample]
    cap = max(r["n_acc"] for r in ref_tapes)
    forced = np.zeros((len(sample), cap, 2))
    fn = np.zeros(len(sample))
    for i, r in enumerate(ref_tapes):
        forced[i, :r["n_acc"]] = r["tape"][:, :2]
        fn[i] = r["n_acc"]
    f_t, fn_t = _t(forced), _t(fn).int()
    o = D.default_opts(forced=f_t.data_ptr(), forced_n=fn_t.data_ptr(), forced_cap=cap, tape_steps=cap + 8)
    xs, us = x0[sample], u[sample]
    rep = D.rollout(model, _t(xs), _t(us), H, dt, tape=True, opts=o)
    assert int(rep["status"].abs().sum()) == 0
    rng = np.random.default_rng(17)
    xbar = rng.normal(size=xs.shape)
    gx, gu = D.rollout_vjp(rep["tape"], _t(xbar))
    gx, gu = gx.cpu().numpy(), gu.cpu().numpy()
    worst_s, worst_g = 0.0, 0.0
    for i in range(len(sample)):
        nd, nut = 16, H * model.nu
        dx0 = np.zeros((nd, model.nx))
        du = np.zeros((nd, nut))
        for j in range(6):
            dx0[j, rng.integers(model.nx)] = 1.0
        for j in range(6, nd):
            du[j, rng.integers(nut)] = 1.0
        jv = om.rollout_jvp(xs[i], us[i], H, dt, dx0, du)
        worst_s = max(worst_s, rel_state(rep["x"].cpu().numpy()[i], jv["x"], model.nq)[0])
        lhs = jv["tx"] @ xbar[i]                        # <x_bar, J d>
        rhs = dx0 @ gx[i] + du @ gu[i].reshape(-1)      # <J^T x_bar, d>
        worst_g = max(worst_g, np.abs(lhs - rhs).max() / max(np.abs(lhs).max(), 1e-12))
    print(f"chain 16384 x {H}: accepted steps mean {nacc.mean():.0f} max {nacc.max()}, tape {recs_n}; sampled "
          f"replay state err {worst_s:.2e}, cotangent vs forward-mode directions {worst_g:.2e}")
    assert worst_s <= 1e-6 and worst_g <= 1e-5


def test_chain_free_run_full_horizon(D, oracle):
    """16 legged chains over the full 2 s (200 intervals of 10 ms, random
    torques) under the continuous controller: every world's end state against
    the oracle replay of its GPU step sequence, its x0/u cotangents against the
    oracle's forward-mode derivatives along 16 random directions (element by
    element), and the decisions and proposed steps of 4 worlds attempt by
    attempt."""
    cfg = W.chain_walk(seed=3, n_worlds=16, n_intervals=200)
    model = D.Model(cfg["model"])
    om = oracle.Model(cfg["model"])
    x0, u, H, dt = cfg["x0"], cfg["u"], cfg["n_intervals"], cfg["interval_dt"]
    o, (log, logn) = _steplog_opts(D, 16, 16384, tape_steps=40 * H + 64)
    res = D.rollout(model, _t(x0), _t(u), H, dt, tape=True, opts=o)
    assert int(res["status"].abs().sum()) == 0
    rng = np.random.default_rng(31)
    xbar = rng.normal(size=x0.shape)
    gx, gu = D.rollout_vjp(res["tape"], _t(xbar))
    gx, gu = gx.cpu().numpy(), gu.cpu().numpy()
    forced, n = tape_steps(res["tape"])
    xs = res["x"].cpu().numpy()
    worst_s = worst_d = 0.0
    nd, nut = 16, H * model.nu
    for w in range(16):
        dx0 = rng.normal(size=(nd, model.nx))
        du = rng.normal(size=(nd, nut))
        rep = om.rollout(x0[w], u[w], H, dt, forced=forced[w, :n[w]])
        assert rep["status"] == 0
        worst_s = max(worst_s, rel_state(xs[w], rep["x"], model.nq)[0])
        _, jv = om.rollout_jvp_forced(x0[w], u[w], H, dt, forced[w, :n[w]], dx0, du)
        lhs = jv @ xbar[w]                                # <x_bar, J d>
        rhs = dx0 @ gx[w] + du @ gu[w].reshape(-1)        # <J^T x_bar, d>
        worst_d = max(worst_d, elementwise_grad(rhs[None], lhs[None])[0])
    checked, bad_dec, by_rounding, max_rel, bad_ctrl = check_decisions_and_controller(
        oracle, om, x0, u, H, dt, res["tape"].records()[0], n, log.cpu().numpy(), logn.cpu().numpy(),
        worlds=[0, 5, 10, 15])
    print(f"chain 16 x 2 s: accepted steps {n.tolist()}; replay state {worst_s:.2e}; directional derivatives "
          f"{worst_d:.2e}; {checked} attempts: {bad_dec} decisions ({by_rounding} more decided by rounding), "
          f"{bad_ctrl} proposed steps differ; error "
          f"estimates agree to {max_rel:.1e}")
    assert worst_s <= STATE_TOL and worst_d <= GRAD_TOL and bad_dec == 0 and bad_ctrl == 0


# ------------------------------------------------------------------ articulated chain
def _chain(n_worlds=4, n_int=6, z=0.535, seed=3):
    cfg = W.chain_walk(seed=seed, n_worlds=n_worlds, n_intervals=n_int)
    x0 = cfg["x0"].copy()
    x0[:, 1] = z
    rng = np.random.default_rng(seed)
    x0[:, 2:7] += rng.normal(0.0, 0.05, size=(n_worlds, 5))
    return cfg["model"], x0, cfg["u"], n_int, cfg["interval_dt"]


def test_chain_accel_and_single_step_parity(D, oracle):
    desc, x0, u, n_int, dt = _chain()
    om = oracle.Model(desc)
    model = D.Model(desc)
    ys, taus, hs, nxt = [], [], [], []
    for w in range(x0.shape[0]):
        r = om.rollout(x0[w], u[w], n_int, dt, tape_cap=100000)
        assert r["status"] == 0
        tp = r["tape"]
        ys.append(tp[:, 2:]); hs.append(tp[:, 1])
        nxt.append(np.vstack([tp[1:, 2:], r["x"][None]]))
        k = np.minimum((tp[:, 0] / dt + 1e-9).astype(int), n_int - 1)
        tau = np.zeros((len(tp), 7))
        tau[:, 3:7] = u[w][k]
        taus.append(tau)
    ys, taus, hs, nxt = np.vstack(ys), np.vstack(taus), np.concatenate(hs), np.vstack(nxt)
    acc, st = D.accel(model, _t(ys), _t(taus))
    assert int(st.abs().sum()) == 0
    ref = np.stack([om.rhs(y, t[3:7])[0][7:] for y, t in zip(ys, taus)])
    ea = np.linalg.norm(acc.cpu().numpy() - ref, axis=1) / np.maximum(np.linalg.norm(ref, axis=1), 1e-3)
    # one forced step per state, with the interval's torques
    Wn = ys.shape[0]
    forced = np.zeros((Wn, 1, 2))
    forced[:, 0, 1] = hs
    f_t, fn = _t(forced), _t(np.ones(Wn)).int()
    o = D.default_opts(forced=f_t.data_ptr(), forced_n=fn.data_ptr(), forced_cap=1)
    res = D.rollout(model, _t(ys), _t(taus[:, None, 3:7]), 1, 10.0, opts=o)
    assert int(res["status"].abs().sum()) == 0
    es = rel_state(res["x"].cpu().numpy(), nxt, model.nq)
    print(f"chain: {Wn} states, accel max rel err {ea.max():.2e}; single-step max rel err {es.max():.2e}")
    assert ea.max() <= 1e-10 and es.max() <= 1e-10


@pytest.mark.parametrize("case", ["chain", "pendulum"])
def test_tree_replayed_gradient(D, oracle, case):
    if case == "chain":
        desc, x0, u, n_int, dt = _chain(n_worlds=3, n_int=5)
    else:
        desc = W.model_pendulum(3)
        rng = np.random.default_rng(4)
        x0 = np.zeros((3, 8))
        x0[:, :4] = rng.uniform(-0.8, 0.8, size=(3, 4))
        x0[:, 4:] = rng.normal(0, 1.0, size=(3, 4))
        n_int, dt = 5, 0.02
        u = rng.uniform(-0.2, 0.2, size=(3, n_int, 4))
    om = oracle.Model(desc)
    model = D.Model(desc)
    tapes = [om.rollout(x0[w], u[w], n_int, dt, tape_cap=100000) for w in range(x0.shape[0])]
    cap = max(r["n_acc"] for r in tapes)
    forced = np.zeros((x0.shape[0], cap, 2))
    fn = np.zeros(x0.shape[0])
    for w, r in enumerate(tapes):
        forced[w, :r["n_acc"]] = r["tape"][:, :2]
        fn[w] = r["n_acc"]
    f_t, fn_t = _t(forced), _t(fn).int()
    o = D.default_opts(forced=f_t.data_ptr(), forced_n=fn_t.data_ptr(), forced_cap=cap, tape_steps=cap + 8)
    res = D.rollout(model, _t(x0), _t(u), n_int, dt, opts=o, tape=True)
    assert int(res["status"].abs().sum()) == 0
    rng = np.random.default_rng(8)
    xbar = rng.normal(size=x0.shape)
    g, ub = D.rollout_vjp(res["tape"], _t(xbar))
    ref = om.grad_batch(x0, u, n_int, dt, xbar, n_threads=4)
    ex = rel_state(res["x"].cpu().numpy(), ref["x"], model.nq)
    eg = rel_grad(g.cpu().numpy(), ref["x0bar"])
    eu = rel_grad(ub.cpu().numpy().reshape(x0.shape[0], -1), ref["ubar"].reshape(x0.shape[0], -1))
    print(f"{case}: replayed {int(fn.sum())} steps; state {ex.max():.2e}, x0 grad {eg.max():.2e}, u grad {eu.max():.2e}")
    assert ex.max() <= 1e-6 and eg.max() <= 1e-5 and eu.max() <= 1e-5


def test_ragged_horizons_and_work_queue(D, oracle):
    """Per-world horizons in one persistent launch (work queue, longest
    first): each world equals its own uniform-horizon run bit for bit, and
    the oracle's run of that world; u_bar beyond a world's horizon is 0."""
    import torch
    rng = np.random.default_rng(21)
    desc = W.model_cube_corners(ctrl=True)
    model = D.Model(desc)
    n = 24
    x0 = W.cube_toss(seed=4, n_worlds=n, horizon=0.1)["x0"]
    H, dt = 6, 0.02
    nint = rng.integers(1, H + 1, size=n).astype(np.int32)
    u = rng.uniform(-0.5, 0.5, size=(n, H, model.nu))
    order = np.argsort(-nint, kind="stable").astype(np.int32)
    nint_t, order_t = torch.tensor(nint, device="cuda"), torch.tensor(order, device="cuda")
    o = D.default_opts(world_intervals=nint_t.data_ptr(), world_order=order_t.data_ptr(), work_queue=1)
    res = D.rollout(model, _t(x0), _t(u), H, dt, opts=o, tape=True, counters=True)
    xbar = np.zeros_like(x0)
    xbar[:, :3] = 1.0
    gx, gu = D.rollout_vjp(res["tape"], _t(xbar))
    gx, gu = gx.cpu().numpy(), gu.cpu().numpy()
    xr = res["x"].cpu().numpy()
    assert int(res["status"].abs().sum()) == 0
    for k in np.unique(nint):
        idx = np.where(nint == k)[0]
        ru = D.rollout(model, _t(x0[idx]), _t(u[idx, :k]), int(k), dt, opts=D.default_opts(work_queue=-1), tape=True)
        gxu, guu = D.rollout_vjp(ru["tape"], _t(xbar[idx]))
        np.testing.assert_array_equal(xr[idx], ru["x"].cpu().numpy())
        np.testing.assert_array_equal(gx[idx], gxu.cpu().numpy())
        np.testing.assert_array_equal(gu[idx, :k], guu.cpu().numpy())
        assert not gu[idx, k:].any()
    om = oracle.Model(desc)
    # each world against the oracle replay of its own accepted steps
    recs, nrec = res["tape"].records()
    worst_s = worst_g = 0.0
    for w in range(n):
        k = int(nint[w])
        f = np.ascontiguousarray(recs[w:w + 1, :nrec[w], :2])
        ref = om.grad_forced_batch(x0[w:w + 1], u[w:w + 1, :k], k, dt, xbar[w:w + 1], f, nrec[w:w + 1])
        worst_s = max(worst_s, rel_state(xr[w], ref["x"], model.nq).max())
        g = np.concatenate([gx[w], gu[w, :k].ravel()])[None]
        r = np.concatenate([ref["x0bar"][0], ref["ubar"][0].ravel()])[None]
        worst_g = max(worst_g, rel_grad(g, r).max(), elementwise_grad(g, r).max())
    print(f"ragged: horizons {np.bincount(nint).tolist()}; vs the oracle replay of each world's steps: state "
          f"{worst_s:.2e}, gradient {worst_g:.2e}")
    assert worst_s <= 1e-6 and worst_g <= 1e-5
    # the queue on and off give the same bits on a uniform batch
    a = D.rollout(model, _t(x0), _t(u), H, dt, opts=D.default_opts(work_queue=1))
    b = D.rollout(model, _t(x0), _t(u), H, dt, opts=D.default_opts(work_queue=-1))
    np.testing.assert_array_equal(a["x"].cpu().numpy(), b["x"].cpu().numpy())


def test_autotune_picks_a_compiled_team(D):
    desc, x0, n_int, dt = _cube_batch(64, horizon=0.05)
    model = D.Model(desc)
    best, times = D.autotune(model, _t(x0), None, n_int, dt)
    print(f"autotune: {times} -> {best} lanes per world")
    assert best in times and len(times) >= 2 and all(t > 0 for t in times.values())
    a = D.rollout(model, _t(x0), None, n_int, dt)
    b = D.rollout(model, _t(x0), None, n_int, dt, opts=D.default_opts(lanes_per_world=best))
    np.testing.assert_array_equal(a["x"].cpu().numpy(), b["x"].cpu().numpy())


@pytest.mark.parametrize("case", ["cube", "chain"])
def test_checkpoint_tape_recomputes_stages(D, case):
    """A checkpoint-only tape (start states of the accepted steps) gives the
    gradient of the full tape: the reverse sweep solves each step's stages
    again (stage 0 from a cold start, so the bits may differ slightly)."""
    if case == "cube":
        desc, x0, n_int, dt = _cube_batch(32)
        u = None
    else:
        cfg = W.chain_walk(n_worlds=16, n_intervals=20)
        desc, x0, n_int, dt, u = cfg["model"], cfg["x0"], 20, cfg["interval_dt"], cfg["u"]
    model = D.Model(desc)
    ut = None if u is None else _t(u)
    xbar = np.zeros_like(x0)
    xbar[:, :3] = 1.0
    out = {}
    for stages in (1, 0):
        r = D.rollout(model, _t(x0), ut, n_int, dt, opts=D.default_opts(tape_stages=stages, tape_steps=4096),
                      tape=True)
        gx, gu = D.rollout_vjp(r["tape"], _t(xbar))
        out[stages] = (r["x"].cpu().numpy(), gx.cpu().numpy(), None if gu is None else gu.cpu().numpy(),
                       r["tape"].info()[1])
    assert out[1][3] == 3 + model.nx + 6 * model.nv and out[0][3] == 3 + model.nx
    np.testing.assert_array_equal(out[1][0], out[0][0])
    eg = rel_grad(out[0][1], out[1][1])
    eu = 0.0 if u is None else rel_grad(out[0][2].reshape(len(x0), -1), out[1][2].reshape(len(x0), -1)).max()
    print(f"{case}: checkpoint-only vs full tape: x0 grad {eg.max():.2e}, u grad {eu:.2e}")
    assert eg.max() <= 1e-9 and eu <= 1e-9
