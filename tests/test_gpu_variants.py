"""The newer gradient paths under the batch engine's launch variants (the
stack batch's parameter gradient among them): the
optimize-then-discretize adjoint with ragged horizons and a work queue equals
each world's own uniform run bit for bit, and the plain one-world-per-launch
form equals the persistent launch; the box half-size gradient is the same on
checkpoint tapes (stages solved again) as on stage tapes; the Tsitouras pair's
discrete adjoint is the same on both tape kinds."""
import numpy as np
import pytest

from paper_2506_14186_amd import workloads as W

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


def test_otd_ragged_horizons_and_plain_form(D):
    import torch
    rng = np.random.default_rng(23)
    desc = W.model_cube_corners(ctrl=True)
    model = D.Model(desc)
    n, H, dt = 16, 5, 0.02
    x0 = W.cube_toss(seed=5, n_worlds=n, horizon=0.1)["x0"]
    nint = rng.integers(1, H + 1, size=n).astype(np.int32)
    u = rng.uniform(-0.5, 0.5, size=(n, H, model.nu))
    order = np.argsort(-nint, kind="stable").astype(np.int32)
    nint_t, order_t = torch.tensor(nint, device="cuda"), torch.tensor(order, device="cuda")
    o = D.default_opts(world_intervals=nint_t.data_ptr(), world_order=order_t.data_ptr(), work_queue=1,
                       tape_stages=1)
    res = D.rollout(model, _t(x0), _t(u), H, dt, opts=o, tape=True)
    assert int(res["status"].abs().sum()) == 0
    xbar = np.zeros_like(x0)
    xbar[:, :3] = 1.0
    gx, gu = D.rollout_vjp_otd(res["tape"], _t(xbar))
    gx, gu = gx.cpu().numpy(), gu.cpu().numpy()
    for k in np.unique(nint):
        idx = np.where(nint == k)[0]
        ru = D.rollout(model, _t(x0[idx]), _t(u[idx, :k]), int(k), dt,
                       opts=D.default_opts(work_queue=-1, tape_stages=1), tape=True)
        gxu, guu = D.rollout_vjp_otd(ru["tape"], _t(xbar[idx]))
        np.testing.assert_array_equal(gx[idx], gxu.cpu().numpy())
        np.testing.assert_array_equal(gu[idx, :k], guu.cpu().numpy())
        assert not gu[idx, k:].any()
    # plain form: one world per launch, the same kernels
    p = D.rollout(model, _t(x0), _t(u), H, dt, opts=D.default_opts(launch_mode=1, tape_stages=1), tape=True)
    q = D.rollout(model, _t(x0), _t(u), H, dt, opts=D.default_opts(tape_stages=1), tape=True)
    gp, up = D.rollout_vjp_otd(p["tape"], _t(xbar))
    gq, uq = D.rollout_vjp_otd(q["tape"], _t(xbar))
    np.testing.assert_array_equal(gp.cpu().numpy(), gq.cpu().numpy())
    np.testing.assert_array_equal(up.cpu().numpy(), uq.cpu().numpy())


def test_geom_gradient_on_checkpoint_tapes(D):
    desc = W.model_box(tc=0.005, mu=0.5)
    cfg = W.box_toss(seed=6, n_worlds=16, horizon=0.3)
    model = D.Model(desc)
    xb = np.zeros_like(cfg["x0"])
    xb[:, 0], xb[:, 2] = 1.0, 1.0
    out = {}
    for stages in (1, 0):
        r = D.rollout(model, _t(cfg["x0"]), None, 1, 0.3, opts=D.default_opts(tape_stages=stages), tape=True)
        assert int(r["status"].abs().sum()) == 0
        _, _, gh = D.rollout_vjp_geom(r["tape"], _t(xb))
        out[stages] = gh.cpu().numpy()
    err = np.abs(out[0] - out[1]).max() / np.abs(out[1]).max()
    print(f"half-size gradient, checkpoints vs stages: {err:.2e}")
    assert err <= 1e-10


def test_tsit5_adjoint_on_checkpoint_tapes(D):
    cfg = W.chain_walk(seed=3, n_worlds=8, n_intervals=10)
    model = D.Model(cfg["model"])
    xb = np.zeros_like(cfg["x0"])
    xb[:, 0], xb[:, 1] = 1.0, 1.0
    out = {}
    for stages in (1, 0):
        r = D.rollout(model, _t(cfg["x0"]), _t(cfg["u"]), 10, 0.01, opts=D.default_opts(tableau=1, tape_stages=stages),
                      tape=True)
        assert int(r["status"].abs().sum()) == 0
        gx, gu = D.rollout_vjp(r["tape"], _t(xb))
        out[stages] = np.concatenate([gx.cpu().numpy().ravel(), gu.cpu().numpy().ravel()])
    err = np.abs(out[0] - out[1]).max() / np.abs(out[1]).max()
    print(f"Tsitouras adjoint, checkpoints vs stages: {err:.2e}")
    assert err <= 1e-10


def test_stack_parameter_gradient_on_checkpoint_tapes_and_plain_launches(D):
    """The stack batch's model-parameter gradient (friction, solref, mass,
    solimp) on checkpoint tapes (stages solved again in the reverse sweep)
    against stage tapes, and in the one-world-per-launch form against the
    persistent launch (bitwise)."""
    ks = (1, 2, 3)
    rng = np.random.default_rng(31)
    descs = [W.model_stack(k, ctrl=True) for k in ks]
    xs = np.concatenate([W.stack_state(rng.normal(0.0, 0.02, size=(k, 2))) for k in ks])
    u = rng.uniform(-2.0, 2.0, size=6 * len(ks))
    xb = np.concatenate([np.concatenate([np.tile([1.0, 0.5, 2.0, 0, 0, 0, 0], k), np.zeros(6 * k)]) for k in ks])
    models = [D.Model(d) for d in descs]
    out = {}
    for name, kw in (("stages", dict(tape_stages=1)), ("checkpoints", dict(tape_stages=0)),
                     ("plain", dict(tape_stages=1, launch_mode=1))):
        r = D.rollout_batch(models, _t(xs), _t(u), 1, 0.05, opts=D.default_opts(tape_steps=8192, **kw), tape=True)
        assert (r["status"].cpu().numpy() == 0).all()
        _, _, gp = D.rollout_batch_vjp_params(r["tape"], _t(xb))
        out[name] = gp.cpu().numpy()[:, 3:]
    np.testing.assert_array_equal(out["plain"], out["stages"])
    err = np.abs(out["checkpoints"] - out["stages"]).max(axis=0) / np.abs(out["stages"]).max(axis=0)
    print(f"stack parameter gradient, checkpoints vs stages: {err.max():.2e}")
    assert err.max() <= 1e-10
