"""Parity of the cube-stack kernels (worlds of k free cubes with box-box and
plane-box contacts) with the oracle, through the C ABI.

Tolerances as for single bodies: F(x) at the same state 1e-10 relative (or
ten times the oracle's own change under 4-ulp state perturbations, where the
contact detection is ill-conditioned: top-four vertex ties of the plane-box
rule, clipping points on a side plane); a GPU step fed the oracle's state and
step 1e-10; free runs checked through the oracle replay of the GPU's accepted
steps: end state 1e-6 (or ten times the oracle's own change under 4-ulp
perturbations of the start state, for stacks settling on stiff contacts),
gradient 1e-5 normwise and element by element; worlds of different sizes in
one launch bitwise equal to separate launches.
"""
import numpy as np
import pytest

from paper_2506_14186_amd import workloads as W
from replay_check import GRAD_TOL, STATE_TOL, elementwise_grad, rel_grad, rel_state

pytestmark = pytest.mark.gpu

MAXATT = 200000


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


def _stacks(ks, seed=7, tc=0.003, mu=0.6):
    rng = np.random.default_rng(seed)
    descs, xs = [], []
    for k in ks:
        descs.append(W.model_stack(k, tc=tc, mu=mu))
        xs.append(W.stack_state(rng.normal(0.0, 0.02, size=(k, 2))))
    return descs, xs


def _tossed(k, seed):
    """A stack whose cubes start tilted and moving (contacts of every kind:
    face, edge, plane corners)."""
    rng = np.random.default_rng(seed)
    x = W.stack_state(rng.normal(0.0, 0.02, size=(k, 2)))
    for i in range(k):
        th = rng.normal(0.0, 0.15, 3)
        a = np.linalg.norm(th)
        x[7 * i + 3:7 * i + 7] = np.concatenate([[np.cos(a / 2)], np.sin(a / 2) * th / a])
        x[7 * i + 2] += 0.05 * i
    x[7 * k:] = rng.normal(0.0, 0.3, 6 * k)
    return x


def _stacked(k, seed):
    """A stack at rest with lateral offsets, its cubes given small velocities
    (it stays a stack: only neighbours touch)."""
    rng = np.random.default_rng(seed)
    x = W.stack_state(rng.normal(0.0, 0.02, size=(k, 2)))
    x[7 * k:] = rng.normal(0.0, 0.05, 6 * k)
    return x


def _sens(om, ys, ref, scale, reps=4, seed=3):
    rng = np.random.default_rng(seed)
    sens = np.zeros(len(ys))
    for _ in range(reps):
        for i, y in enumerate(ys):
            yp = y * (1.0 + 4.4e-16 * rng.choice([-1.0, 1.0], size=y.shape))
            sens[i] = max(sens[i], np.linalg.norm(om.rhs(yp)[0][om.nv:] - ref[i]) / scale[i])
    return sens


@pytest.mark.parametrize("k,kind", [(2, "tossed"), (3, "tossed"), (5, "stacked"), (8, "stacked")])
def test_stack_accel_parity(D, oracle, k, kind):
    """F(x) at states along oracle trajectories of tossed stacks (two and
    three cubes: face, edge and corner contacts) and of stacks that stay
    stacked (five and eight cubes)."""
    desc = W.model_stack(k, tc=0.003)
    om = oracle.Model(desc)
    ys = []
    for seed in (1, 2):
        x0 = _tossed(k, seed) if kind == "tossed" else _stacked(k, seed)
        r = om.rollout(x0, None, 1, 0.4, tape_cap=100000)
        assert r["status"] == 0
        ys.append(r["tape"][::7, 2:])
    ys = np.vstack(ys)
    model = D.Model(desc)
    acc, st = D.accel(model, _t(ys))
    assert int(st.abs().sum()) == 0, st
    ref = np.stack([om.rhs(y)[0][om.nv:] for y in ys])
    scale = np.maximum(np.linalg.norm(ref, axis=1), 1e-3)
    err = np.linalg.norm(acc.cpu().numpy() - ref, axis=1) / scale
    sens = _sens(om, ys, ref, scale)
    tol = np.maximum(1e-10, 10.0 * sens)
    nrow = np.array([om.rhs(y)[1]["n_rows"] for y in ys])
    print(f"stack k={k}: {len(ys)} states ({int((nrow > 0).sum())} in contact, up to {nrow.max() // 4} contacts), "
          f"max rel err {err.max():.2e}, max err/tol {(err / tol).max():.2f}")
    assert (err <= tol).all()


@pytest.mark.parametrize("k", [2, 4])
def test_stack_single_step_parity(D, oracle, k):
    """Each oracle step of a tossed stack replayed as a one-step GPU world."""
    desc = W.model_stack(k, tc=0.003)
    om = oracle.Model(desc)
    r = om.rollout(_tossed(k, 3) if k < 4 else _stacked(k, 3), None, 1, 0.3, tape_cap=100000)
    assert r["status"] == 0
    tp = r["tape"][::3]
    ys, hs = tp[:, 2:], tp[:, 1]
    nxt = np.stack([om.rollout(y, None, 1, h, forced=np.array([[0.0, h]]))["x"] for y, h in zip(ys, hs)])
    model = D.Model(desc)
    n = len(ys)
    forced = _t(np.stack([[[0.0, h]] for h in hs]))
    fn = _t(np.ones(n)).int()
    res, sts = [], []
    for i in range(n):
        r1 = D.rollout(model, _t(ys[i:i + 1]), None, 1, float(hs[i]),
                       opts=D.default_opts(forced=forced[i:i + 1].data_ptr(), forced_n=fn[i:i + 1].data_ptr(),
                                           forced_cap=1))
        res.append(r1["x"].cpu().numpy()[0])
        sts.append(int(r1["status"][0]))
    assert not any(sts), sts
    err = rel_state(np.stack(res), nxt, 7 * k)
    # the oracle's own step under 4-ulp perturbations of its start state: at
    # rest on stiff contacts the step is taken at the explicit stability limit
    # and amplifies rounding of the contact forces (tens of newtons balanced
    # to a vanishing net acceleration); both sides may differ by that much
    rng = np.random.default_rng(5)
    sens = np.zeros(n)
    for i, (y, h) in enumerate(zip(ys, hs)):
        for _ in range(2):
            yp = y * (1.0 + 4.4e-16 * rng.choice([-1.0, 1.0], size=y.shape))
            xp = om.rollout(yp, None, 1, h, forced=np.array([[0.0, h]]))["x"]
            sens[i] = max(sens[i], rel_state(xp, nxt[i], 7 * k)[0])
    tol = np.maximum(1e-10, 10.0 * sens)
    print(f"stack k={k}: {n} single steps, max rel err {err.max():.2e}, max err/tol {(err / tol).max():.2f}, "
          f"{int((10 * sens > 1e-10).sum())} states with the oracle's own 4-ulp sensitivity above 1e-11 "
          f"(max {sens.max():.1e})")
    assert (err <= tol).all()


def _free_and_replay(D, oracle, descs, xs, horizon, xbar_fn):
    """One uneven-batch free run on the GPU (forward + reverse) and the
    oracle's replay of every world's accepted steps."""
    models = [D.Model(d) for d in descs]
    x0 = _t(np.concatenate(xs))
    res = D.rollout_batch(models, x0, None, 1, horizon, opts=D.default_opts(max_attempts=MAXATT, tape_steps=8192),
                          tape=True, counters=True)
    st = res["status"].cpu().numpy()
    assert (st == 0).all(), st
    xo = res["x_off"]
    xb = np.concatenate([xbar_fn(d, x) for d, x in zip(descs, xs)])
    gx, _ = D.rollout_batch_vjp(res["tape"], _t(xb))
    recs, n = res["tape"].world_records()
    xg, gg = res["x"].cpu().numpy(), gx.cpu().numpy()

    def one(w):
        d, x = descs[w], xs[w]
        om = oracle.Model(d)
        nx = x.size
        forced = np.ascontiguousarray(recs[w][:, :2])
        ref = om.grad_forced_batch(x[None], None, 1, horizon, xb[xo[w]:xo[w] + nx][None], forced[None],
                                   np.array([n[w]], np.int32), n_threads=1)
        assert ref["status"][0] == 0
        k = nx // 13
        es = rel_state(xg[xo[w]:xo[w] + nx], ref["x"][0], 7 * k)[0]
        eg = rel_grad(gg[xo[w]:xo[w] + nx], ref["x0bar"][0])[0]
        ee = elementwise_grad(gg[xo[w]:xo[w] + nx], ref["x0bar"][0])[0]
        # the oracle's own replay under 4-ulp perturbations of the start state:
        # near rest the velocities are tiny and the steps sit at the stiff
        # contacts' stability limit, so rounding of the contact forces shows
        rng = np.random.default_rng(17 + w)
        sens = 0.0
        for _ in range(2):
            xp = x * (1.0 + 4.4e-16 * rng.choice([-1.0, 1.0], size=x.shape))
            xr = om.rollout(xp, None, 1, horizon, forced=forced[:n[w]])["x"]
            sens = max(sens, rel_state(xr, ref["x"][0], 7 * k)[0])
        return (k, int(n[w]), es, eg, ee, sens)

    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=8) as ex:  # the oracle releases the interpreter lock
        out = list(ex.map(one, range(len(descs))))
    return out, res


def _sum_positions(d, x):
    k = x.size // 13
    xb = np.zeros_like(x)
    for i in range(k):
        xb[7 * i:7 * i + 3] = 1.0
    return xb


def test_stack_free_runs_replayed(D, oracle):
    """Free runs of stacks of 1..4 cubes (and tossed pairs) in one launch,
    every world checked against the oracle replay of its GPU steps."""
    descs, xs = _stacks([1, 2, 3, 4], seed=11)
    # two tossed cubes (face, edge and corner contacts; with two cubes every
    # contact is between neighbours) and stacks with moving cubes
    for seed in (5, 8):
        descs.append(W.model_stack(2, tc=0.002))
        xs.append(_tossed(2, seed))
    descs.append(W.model_stack(3, tc=0.002))
    xs.append(_stacked(3, 6))
    descs.append(W.model_stack(4, tc=0.0015))
    xs.append(_stacked(4, 7))
    out, _ = _free_and_replay(D, oracle, descs, xs, 0.5, _sum_positions)
    for k, n, es, eg, ee, sens in out:
        print(f"k={k}: {n} accepted steps, state {es:.2e} (oracle's 4-ulp sensitivity {sens:.1e}), "
              f"gradient {eg:.2e} (element-wise {ee:.2e})")
    # end state: 1e-6, or ten times the oracle's own 4-ulp sensitivity
    assert all(o[2] <= max(STATE_TOL, 10.0 * o[5]) for o in out)
    assert max(o[3] for o in out) <= GRAD_TOL and max(o[4] for o in out) <= GRAD_TOL


def test_uneven_batch_equals_separate_launches(D):
    """Worlds of 1..6 cubes in one persistent launch give bitwise the same end
    states, step counts and gradients as each model run alone."""
    descs, xs = _stacks([3, 1, 6, 2, 5, 4], seed=13)
    models = [D.Model(d) for d in descs]
    x0 = _t(np.concatenate(xs))
    opts = D.default_opts(max_attempts=MAXATT, tape_steps=4096)
    res = D.rollout_batch(models, x0, None, 1, 0.3, opts=opts, tape=True, counters=True)
    assert int(res["status"].abs().sum()) == 0, res["status"]
    xb = np.concatenate([_sum_positions(d, x) for d, x in zip(descs, xs)])
    gx, _ = D.rollout_batch_vjp(res["tape"], _t(xb))
    xo = res["x_off"]
    for w, (m, x) in enumerate(zip(models, xs)):
        r1 = D.rollout_batch([m], _t(x), None, 1, 0.3, opts=opts, tape=True, counters=True)
        g1, _ = D.rollout_batch_vjp(r1["tape"], _t(_sum_positions(None, x)))
        nx = x.size
        np.testing.assert_array_equal(res["x"].cpu().numpy()[xo[w]:xo[w] + nx], r1["x"].cpu().numpy())
        np.testing.assert_array_equal(gx.cpu().numpy()[xo[w]:xo[w] + nx], g1.cpu().numpy())
        assert int(res["n_acc"][w]) == int(r1["n_acc"][0])


@pytest.mark.parametrize("stages,queue,plain", [(1, 1, 0), (0, 1, 0), (1, -1, 0), (1, 1, 1)],
                         ids=["stages-queue", "checkpoints-queue", "stages-per-block", "plain"])
def test_fused_grad_equals_rollout_then_vjp(D, stages, queue, plain):
    """Forward and reverse of each world in one launch (the cotangent given up
    front) give bitwise the end states, step counts and gradients of the
    forward launch followed by the reverse launch, for every tape policy and
    work distribution; the tape it leaves serves further cotangents and is
    reused in place."""
    descs, xs = _stacks([3, 1, 6, 2, 5, 4, 7, 1, 2], seed=21)
    xs[2] = _tossed(6, 5)
    xs[6] = _tossed(7, 8)
    models = [D.Model(d) for d in descs]
    x0 = _t(np.concatenate(xs))
    xb = _t(np.concatenate([_sum_positions(d, x) for d, x in zip(descs, xs)]))
    xb2 = _t(np.random.default_rng(3).normal(size=xb.numel()))
    opts = D.default_opts(max_attempts=MAXATT, tape_steps=4096, tape_stages=stages, work_queue=queue,
                          launch_mode=plain)
    ref = D.rollout_batch(models, x0, None, 1, 0.2, opts=opts, tape=True, counters=True)
    g_ref, _ = D.rollout_batch_vjp(ref["tape"], xb)
    g2_ref, _ = D.rollout_batch_vjp(ref["tape"], xb2)
    f = D.rollout_batch_grad(models, x0, None, 1, 0.2, xb, opts=opts, counters=True)
    assert int(f["status"].abs().sum()) == 0, f["status"]
    for key in ("x", "status", "n_acc", "n_rej"):
        np.testing.assert_array_equal(f[key].cpu().numpy(), ref[key].cpu().numpy())
    np.testing.assert_array_equal(f["x0_bar"].cpu().numpy(), g_ref.cpu().numpy())
    g2, _ = D.rollout_batch_vjp(f["tape"], xb2)
    np.testing.assert_array_equal(g2.cpu().numpy(), g2_ref.cpu().numpy())
    again = D.rollout_batch_grad(models, x0, None, 1, 0.2, xb2, opts=opts, reuse=f["tape"])
    np.testing.assert_array_equal(again["x0_bar"].cpu().numpy(), g2_ref.cpu().numpy())
    print(f"fused forward+reverse bitwise equal to two launches ({len(models)} worlds, "
          f"{int(ref['n_acc'].sum())} accepted steps)")


def test_fused_grad_stopped_worlds_get_nan(D):
    """Worlds stopped by the attempt cap get NaN gradients in the fused launch,
    as in the reverse launch, the others finite gradients; null arguments are
    refused."""
    descs, xs = _stacks([4, 1, 3], seed=22)
    xs[0] = _tossed(4, 9)
    models = [D.Model(d) for d in descs]
    x0 = _t(np.concatenate(xs))
    xb = _t(np.concatenate([_sum_positions(d, x) for d, x in zip(descs, xs)]))
    opts = D.default_opts(max_attempts=40, tape_steps=4096)
    ref = D.rollout_batch(models, x0, None, 1, 0.2, opts=opts, tape=True, counters=True)
    g_ref, _ = D.rollout_batch_vjp(ref["tape"], xb)
    f = D.rollout_batch_grad(models, x0, None, 1, 0.2, xb, opts=opts, counters=True)
    st = f["status"].cpu().numpy()
    assert st[0] != 0, st
    np.testing.assert_array_equal(st, ref["status"].cpu().numpy())
    g = f["x0_bar"].cpu().numpy()
    np.testing.assert_array_equal(g, g_ref.cpu().numpy())
    xo = f["x_off"]
    for w, x in enumerate(xs):
        gw = g[xo[w]:xo[w] + x.size]
        assert np.isnan(gw).all() if st[w] != 0 else np.isfinite(gw).all(), (w, st[w])
    rc = D._lib.dmx_rollout_batch_grad(None, None, None, None, None, None, None, None, None, None, None, None, None)
    assert rc < 0


def test_work_counters_match_oracle_units(D, oracle):
    """The kernels' work counters, which the benchmark multiplies by the
    per-unit operation counts fitted to the oracle's counter, count the same
    units as the oracle on the same worlds: attempts, right-hand sides and
    contacts (all, and those between two cubes) equal where the step
    sequences are equal; Newton iterations at most the oracle's (the kernels
    start each stage's solve from the previous stage's solution)."""
    descs, xs = _stacks([1, 3, 5], seed=31)
    xs.append(_tossed(4, 12))
    descs.append(W.model_stack(4, tc=0.003, mu=0.6))
    models = [D.Model(d) for d in descs]
    x0 = _t(np.concatenate(xs))
    import torch
    fc = torch.zeros((len(models), len(D.FWD_COUNTERS)), dtype=torch.int64, device="cuda")
    opts = D.default_opts(max_attempts=MAXATT, tape_steps=4096, fwd_counters=fc.data_ptr())
    res = D.rollout_batch(models, x0, None, 1, 0.05, opts=opts, counters=True)
    assert int(res["status"].abs().sum()) == 0
    c = {n: fc[:, i].cpu().numpy() for i, n in enumerate(D.FWD_COUNTERS)}
    for w, (d, x) in enumerate(zip(descs, xs)):
        r = oracle.Model(d).flop_count(x, None, 1, 0.05)
        gpu_att = int(res["n_acc"][w]) + int(res["n_rej"][w])
        print(f"world {w} (k={x.size // 13}): attempts {c['attempts'][w]}/{r['attempts']}, rhs {c['rhs'][w]}/{r['rhs']}, "
              f"contacts {c['rhs_contacts'][w]}/{r['rhs_contacts']} (pairs {c['rhs_contacts_pair'][w]}/"
              f"{r['rhs_contacts_box']}), newton {c['newton_iters'][w]}/{r['newton_iters']}  (GPU/oracle)")
        assert c["attempts"][w] == gpu_att
        if gpu_att != r["attempts"]:
            continue  # step sequences split: units differ with them
        assert c["rhs"][w] == r["rhs"]
        assert abs(int(c["rhs_contacts"][w]) - r["rhs_contacts"]) <= 0.01 * r["rhs_contacts"] + 2
        assert abs(int(c["rhs_contacts_pair"][w]) - r["rhs_contacts_box"]) <= 0.01 * r["rhs_contacts_box"] + 2
        assert c["newton_iters"][w] <= r["newton_iters"]


def test_stack_batch_api_errors(D):
    """Models that are not stacks of cubes are refused by the batch call."""
    sphere = D.Model(W.model_sphere())
    with pytest.raises(D.DmxError):
        D.rollout_batch([sphere], _t(W.sphere_drop()["x0"][0]), None, 1, 0.1)
