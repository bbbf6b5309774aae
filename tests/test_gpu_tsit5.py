"""GPU rollouts and discrete adjoints with the Tsitouras 5(4) pair (Tsit5, the
paper's solver, App. E.1; solver option tableau = 1) against the oracle's
Tsit5, in the checks used for the Dormand-Prince pair: each GPU free run's
accepted steps replayed by the oracle give the GPU's end state (1e-6) and
gradient (1e-5 normwise and element by element); the corner-sphere cube with
16-lane teams, the box-geom cube and the legged chain with controls.  Stack
batches and the optimize-then-discretize adjoint refuse the option."""
import numpy as np
import pytest

from paper_2506_14186_amd import workloads as W
from replay_check import GRAD_TOL, STATE_TOL, replay_and_compare, tape_steps

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


def _check(D, oracle, name, desc, x0, u, n_int, dt, xb, **kw):
    model = D.Model(desc)
    opts = D.default_opts(tableau=1, tape_steps=8192, **kw)
    r = D.rollout(model, _t(x0), None if u is None else _t(u), n_int, dt, opts=opts, tape=True, counters=True)
    assert int(r["status"].abs().sum()) == 0
    gx, gu = D.rollout_vjp(r["tape"], _t(xb))
    forced, n = tape_steps(r["tape"])
    om = oracle.Model(desc)
    out = replay_and_compare(om, om.nq, x0, u, n_int, dt, r["x"].cpu().numpy(), forced, n, xb, gx.cpu().numpy(),
                             None if gu is None else gu.cpu().numpy(), tableau=1)
    print(f"{name}: state {out['state'].max():.2e}, gradient {out['grad'].max():.2e} "
          f"(elementwise {out['grad_elem'].max():.2e}), accepted steps mean {float(r['n_acc'].double().mean()):.1f}")
    assert out["state"].max() <= STATE_TOL
    assert out["grad"].max() <= GRAD_TOL and out["grad_elem"].max() <= GRAD_TOL
    return r


def test_tsit5_corner_cube_16_lanes(D, oracle):
    cfg = W.cube_toss(seed=2, n_worlds=32, horizon=0.3)
    xb = np.zeros_like(cfg["x0"])
    xb[:, :3] = 1.0
    _check(D, oracle, "corner cube", cfg["model"], cfg["x0"], None, 1, 0.3, xb, lanes_per_world=16)


def test_tsit5_box_cube(D, oracle):
    cfg = W.box_toss(seed=4, n_worlds=16, horizon=0.3)
    xb = np.zeros_like(cfg["x0"])
    xb[:, 0], xb[:, 2] = 1.0, 1.0
    _check(D, oracle, "box cube", cfg["model"], cfg["x0"], None, 1, 0.3, xb)


def test_tsit5_chain_controls(D, oracle):
    cfg = W.chain_walk(seed=3, n_worlds=8, n_intervals=20)
    xb = np.zeros_like(cfg["x0"])
    xb[:, 0], xb[:, 1] = 1.0, 1.0
    _check(D, oracle, "chain", cfg["model"], cfg["x0"], cfg["u"], 20, 0.01, xb)


def test_tsit5_step_counts_near_dopri5(D):
    """On the cube batch the two pairs take comparable numbers of steps."""
    cfg = W.cube_toss(seed=2, n_worlds=256, horizon=0.5)
    model = D.Model(cfg["model"])
    x0 = _t(cfg["x0"])
    n = {}
    for tab in (0, 1):
        r = D.rollout(model, x0, None, 1, 0.5, opts=D.default_opts(tableau=tab), counters=True)
        assert int(r["status"].abs().sum()) == 0
        n[tab] = float((r["n_acc"] + r["n_rej"]).double().mean())
    print(f"attempts per world: Dormand-Prince {n[0]:.1f}, Tsitouras {n[1]:.1f}")
    assert 0.5 < n[1] / n[0] < 2.0


def test_tsit5_refused_where_not_built(D):
    import torch
    stack = D.Model(W.model_stack(2))
    x = _t(W.stack_state(np.zeros((2, 2))))
    with pytest.raises(D.DmxError):
        D.rollout_batch([stack], x, None, 1, 0.02, opts=D.default_opts(tableau=1))
    cfg = W.cube_toss(seed=2, n_worlds=2, horizon=0.05)
    r = D.rollout(D.Model(cfg["model"]), _t(cfg["x0"]), None, 1, 0.05, opts=D.default_opts(tableau=1, tape_stages=1),
                  tape=True)
    with pytest.raises(D.DmxError):
        D.rollout_vjp_otd(r["tape"], torch.zeros((2, 13), dtype=torch.float64, device="cuda"))
    with pytest.raises(D.DmxError):
        D.rollout(D.Model(cfg["model"]), _t(cfg["x0"]), None, 1, 0.05, opts=D.default_opts(tableau=2))
