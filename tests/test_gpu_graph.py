"""Captured rollout segments (dmx_graph_*): every replay, with new inputs
written into the captured buffers and the program's own eager work and
synchronizations in between, gives bitwise the results of the eager calls
(forward end states, statuses, and the reverse sweep's cotangents)."""
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


def _eager(D, models, x0, u, n_int, dt, xbar, uniform_free):
    import torch
    if uniform_free:
        m = models[0]
        W_ = len(models)
        r = D.rollout(m, x0.view(W_, -1), None if u is None else u.view(W_, n_int, -1), n_int, dt, tape=True)
        x0b, ub = D.rollout_vjp(r["tape"], xbar.view(W_, -1))
        return r["x"].reshape(-1), r["status"], x0b.reshape(-1), (None if ub is None else ub.reshape(-1))
    r = D.rollout_batch(models, x0, u, n_int, dt, tape=True)
    x0b, ub = D.rollout_batch_vjp(r["tape"], xbar)
    torch.cuda.synchronize()
    return r["x"], r["status"], x0b, ub


@pytest.mark.parametrize("case", ["stacks", "cubes"])
def test_graph_replays_equal_eager_calls(D, case):
    import torch
    rng = np.random.default_rng(31)
    if case == "stacks":
        ks = [3, 1, 5, 2]
        models = [D.Model(W.model_stack(k, tc=0.003, ctrl=True)) for k in ks]
        x0s = lambda: np.concatenate([W.stack_state(rng.normal(0, 0.01, (k, 2))) for k in ks])  # noqa: E731
        n_int, dt, uniform_free = 4, 0.01, False
    else:
        m = D.Model(W.model_cube_corners(ctrl=True))
        models = [m] * 16
        x0s = lambda: W.cube_toss(seed=int(rng.integers(1 << 20)), n_worlds=16, horizon=0.04)["x0"].reshape(-1)  # noqa: E731
        n_int, dt, uniform_free = 4, 0.01, True
    nu = sum(n_int * mm.nu for mm in models)
    x0 = _t(x0s())
    u = _t(rng.uniform(-1, 1, nu)) if nu else None
    g = D.Graph(models, x0, u, n_int, dt)
    try:
        for rep in range(4):
            x0n, un, xbn = _t(x0s()), (_t(rng.uniform(-1, 1, nu)) if nu else None), _t(rng.normal(0, 1, x0.numel()))
            g.x0.copy_(x0n)
            if nu:
                g.u.copy_(un)
            g.xbar.copy_(xbn)
            g.replay()
            torch.cuda.synchronize()
            xs, st, x0b, ub = _eager(D, models, x0n, un, n_int, dt, xbn, uniform_free)  # eager work in between
            torch.cuda.synchronize()
            assert (st.cpu().numpy() == 0).all()
            assert torch.equal(g.status, st)
            assert torch.equal(g.x, xs), rep
            assert torch.equal(g.x0bar, x0b), rep
            if nu:
                assert torch.equal(g.ubar, ub), rep
        print(f"{case}: 4 replays bitwise equal to the eager calls")
    finally:
        g.close()


def test_autotune_batch_choices(D):
    """The batch autotuner times every candidate (tape policy x work
    distribution, x team size for one free-body model) and its choice runs."""
    import torch
    ks = [4, 2, 6, 1, 3]
    models = [D.Model(W.model_stack(k, tc=0.003)) for k in ks]
    rng = np.random.default_rng(41)
    x0 = _t(np.concatenate([W.stack_state(rng.normal(0, 0.01, (k, 2))) for k in ks]))
    best, tried = D.autotune_batch(models, x0, None, 1, 0.02)
    assert len(tried) == 4 and {(t["tape_stages"], t["work_queue"]) for t in tried} == {(1, 1), (1, -1), (0, 1), (0, -1)}
    assert best["ms"] == min(t["ms"] for t in tried) and best["lanes_per_world"] == 0
    opts = D.default_opts(tape_stages=best["tape_stages"], work_queue=best["work_queue"])
    r = D.rollout_batch(models, x0, None, 1, 0.02, opts=opts, tape=True)
    assert (r["status"].cpu().numpy() == 0).all()
    cube = D.Model(W.model_cube_corners())
    xc = _t(W.cube_toss(seed=3, n_worlds=256, horizon=0.02)["x0"].reshape(-1))
    best_c, tried_c = D.autotune_batch([cube] * 256, xc, None, 1, 0.02)
    teams = sorted({t["lanes_per_world"] for t in tried_c})
    assert len(tried_c) == 4 * len(teams) and best_c["lanes_per_world"] in teams
    print(f"stack batch: {best}; cube batch: {best_c} (teams {teams})")
