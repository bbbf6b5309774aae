"""Parity of the GPU optimize-then-discretize adjoint (dmx_rollout_vjp_otd)
with the oracle's, through the C ABI: both solve the continuous adjoint
equations backwards with their own adaptive steps along the continuous
extension of the forward's accepted steps, so where the forward and the
adjoint take the same step sequences they agree to rounding; the bar is the
gradient tolerance of the discrete adjoint's parity (1e-5 relative, element
by element against the largest component), at rtol 1e-10: at looser
tolerances a step decision taken differently at rounding level (in the
forward or in the adjoint, whose right-hand side jumps where contacts switch)
moves both results by their discretization error, which for these contact-
rich tumbles is 1e-3 to 1 at rtol 1e-6 (the cube toss prints the GPU-oracle
difference at 1e-6, 1e-8 and 1e-10: it shrinks about 100x per two decades).  Cases: the paper's cube toss
(box geom), the corner-sphere cube of the benchmark batch with 16-lane
teams, the legged chain with controls (state and control gradients),
bouncing sphere tosses with spin, and the straight-through CFD adjoint of a
sphere skimming the plane, which also
matches the small-step limit of the discrete straight-through gradient
(where the discrete adjoint along the forward's few large steps does not).
"""
import numpy as np
import pytest

from paper_2506_14186_amd import workloads as W
from test_oracle_pins import sphere_state

pytestmark = pytest.mark.gpu
TOL = 1e-5


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


def _compare(name, got, want):
    got, want = np.asarray(got), np.asarray(want)
    scale = np.max(np.abs(want), axis=-1, keepdims=True)
    err = np.abs(got - want) / np.maximum(scale, 1e-12)
    print(f"{name}: max rel err {err.max():.2e}")
    assert err.max() <= TOL, (name, err.max())


def _run(D, desc, x0, u, n_int, dt, xb, **kw):
    model = D.Model(desc)
    opts = D.default_opts(tape_steps=65536, tape_stages=1, **kw)
    r = D.rollout(model, _t(x0), None if u is None else _t(u), n_int, dt, opts=opts, tape=True, counters=True)
    assert int(r["status"].abs().sum()) == 0
    g, gu = D.rollout_vjp_otd(r["tape"], _t(xb))
    return r, g.cpu().numpy(), None if gu is None else gu.cpu().numpy()


def test_otd_cube_toss_matches_oracle(D, oracle):
    desc = W.model_box(tc=0.005, solimp=(0.0, 0.95, 0.001, 0.5, 2.0), mu=0.8)
    x0 = np.zeros((8, 13))
    x0[:, 2], x0[:, 3] = 0.3, 1.0
    x0[:, 7] = np.linspace(-3.0, -1.0, 8)
    x0[:, 11] = np.linspace(-1.0, 1.0, 8)
    xb = np.zeros((8, 13))
    xb[:, 0], xb[:, 2] = 1.0, 0.5
    for rtol in (1e-6, 1e-8, 1e-10):
        r, g, _ = _run(D, desc, x0, None, 1, 1.0, xb, rtol=rtol, atol=rtol)
        ref = oracle.Model(desc).otd_grad_batch(x0, None, 1, 1.0, xb, n_threads=8, rtol=rtol, atol=rtol)
        assert (ref["status"] == 0).all()
        scale = np.max(np.abs(ref["x0bar"]), axis=1, keepdims=True)
        err = np.abs(g - ref["x0bar"]) / scale
        print(f"rtol {rtol:.0e}: per-world max rel err {np.array2string(err.max(1), precision=2)}, forward steps "
              f"gpu {r['n_acc'].cpu().numpy()} oracle {ref['n_acc']}, adjoint steps oracle {ref['adj_accepted']}")
    _compare("cube toss otd rtol 1e-10", g, ref["x0bar"])


def test_otd_corner_cube_batch_matches_oracle(D, oracle):
    cfg = W.cube_toss(seed=2, n_worlds=16, horizon=0.3)
    x0 = cfg["x0"]
    xb = np.zeros_like(x0)
    xb[:, :3] = 1.0
    _, g, _ = _run(D, cfg["model"], x0, None, 1, 0.3, xb, lanes_per_world=16, rtol=1e-10, atol=1e-10)
    ref = oracle.Model(cfg["model"]).otd_grad_batch(x0, None, 1, 0.3, xb, n_threads=8, rtol=1e-10, atol=1e-10)
    _compare("corner cube otd (16-lane teams)", g, ref["x0bar"])


def test_otd_chain_controls_match_oracle(D, oracle):
    cfg = W.chain_walk(seed=3, n_worlds=4, n_intervals=20)
    x0, u = cfg["x0"], cfg["u"]
    xb = np.zeros_like(x0)
    xb[:, 0], xb[:, 1] = 1.0, 1.0
    _, g, gu = _run(D, cfg["model"], x0, u, 20, 0.01, xb, rtol=1e-10, atol=1e-10)
    ref = oracle.Model(cfg["model"]).otd_grad_batch(x0, u, 20, 0.01, xb, n_threads=4, rtol=1e-10, atol=1e-10)
    _compare("chain otd x0", g, ref["x0bar"])
    _compare("chain otd u", gu.reshape(4, -1), ref["ubar"].reshape(4, -1))


def test_otd_cfd_skimming_sphere(D, oracle):
    desc = W.model_sphere()
    x = sphere_state(0.105, vz=0.0, vx=0.3)
    T = 0.03
    xb = np.zeros((1, 13))
    xb[0, 2] = 1.0
    r, g, _ = _run(D, desc, x[None], None, 1, T, xb, cfd=1, rtol=1e-10, atol=1e-10)
    ref = oracle.Model(desc).otd_grad_batch(x[None], None, 1, T, xb, cfd=1, rtol=1e-10, atol=1e-10)
    _compare("skimming sphere otd+cfd", g, ref["x0bar"])
    h = 5e-6
    forced = np.array([[i * h, h] for i in range(int(round(T / h)))])
    _, tx = oracle.Model(desc).rollout_jvp_forced(x, None, 1, T, forced, np.eye(13)[[2, 9]], cfd=1)
    np.testing.assert_allclose(g[0, [2, 9]], tx[:, 2], rtol=1e-5, atol=1e-7)
    dto, _ = D.rollout_vjp(r["tape"], _t(xb))
    off = np.abs(dto.cpu().numpy()[0, [2, 9]] - tx[:, 2]).max()
    print(f"skimming sphere: forward steps {int(r['n_acc'][0])}, otd {g[0, [2, 9]]}, "
          f"small-step limit {tx[:, 2]}, discrete adjoint off by {off:.3g}")
    assert off > 100 * np.abs(g[0, [2, 9]] - tx[:, 2]).max()


def test_otd_refuses_unsupported_tapes(D):
    import torch
    cfg = W.cube_toss(seed=2, n_worlds=2, horizon=0.05)
    model = D.Model(cfg["model"])
    r = D.rollout(model, _t(cfg["x0"]), None, 1, 0.05, opts=D.default_opts(tape_stages=0), tape=True)
    with pytest.raises(D.DmxError):
        D.rollout_vjp_otd(r["tape"], torch.zeros((2, 13), dtype=torch.float64, device="cuda"))
    stack = D.Model(W.model_stack(2))
    x = _t(W.stack_state(np.zeros((2, 2))))
    rb = D.rollout_batch([stack], x, None, 1, 0.02, tape=True)
    with pytest.raises(D.DmxError):
        D._check(D._lib.dmx_rollout_vjp_otd(rb["tape"].h, D._ptr(x), D._ptr(torch.empty_like(x)), None,
                                            D._stream()))


def test_otd_bouncing_sphere_tosses_match_oracle(D, oracle):
    """Spheres thrown onto the plane (bounces between free flights, where the
    adjoint's steps end on the forward's step boundaries on both sides), at
    rtol 1e-10: GPU against the oracle's continuous adjoint."""
    desc = W.model_sphere(radius=0.1, mu=0.8, tc=0.005, solimp=(0.0, 0.95, 0.001, 0.5, 2.0))
    n = 8
    x0 = np.zeros((n, 13))
    x0[:, 2] = 0.3
    x0[:, 3] = 1.0
    x0[:, 7] = np.linspace(-3.0, -1.0, n)
    x0[:, 10] = np.linspace(-5.0, 5.0, n)  # some spin
    xb = np.zeros((n, 13))
    xb[:, 0], xb[:, 1], xb[:, 2] = 1.0, 0.5, 2.0
    _, g, _ = _run(D, desc, x0, None, 1, 1.0, xb, rtol=1e-10, atol=1e-10)
    ref = oracle.Model(desc).otd_grad_batch(x0, None, 1, 1.0, xb, n_threads=8, rtol=1e-10, atol=1e-10)
    _compare("bouncing sphere tosses", g, ref["x0bar"])
