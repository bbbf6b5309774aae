"""The allocation-free entry point (dmx_rollout_noalloc) against dmx_rollout
without a tape, through the C ABI: two calls in a row, the second with a
smaller batch, each bitwise equal to dmx_rollout on the same inputs (the
same kernels run; only the home of the work-queue counter differs)."""
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


def _check_pair(D, model, x0, u, n_int, dt, opts):
    import torch
    W_ = x0.shape[0]
    ref = D.rollout(model, x0, u, n_int, dt, opts=opts, counters=True)
    xo = torch.full_like(x0, float("nan"))
    st = torch.full((W_,), -7, dtype=torch.int32, device="cuda")
    na = torch.zeros(W_, dtype=torch.int32, device="cuda")
    D.rollout_noalloc(model, x0, u, n_int, dt, xo, st, opts=opts, n_acc=na)
    torch.cuda.synchronize()
    assert int(ref["status"].abs().sum()) == 0
    np.testing.assert_array_equal(xo.cpu().numpy(), ref["x"].cpu().numpy())
    np.testing.assert_array_equal(st.cpu().numpy(), ref["status"].cpu().numpy())
    np.testing.assert_array_equal(na.cpu().numpy(), ref["n_acc"].cpu().numpy())


def test_noalloc_matches_rollout_cube_batch(D):
    """Cube worlds in a persistent launch with the work queue (more worlds than
    the device holds at once), then a smaller batch reusing the scratch."""
    cfg = W.cube_toss(seed=2, n_worlds=3000, horizon=0.05)
    model = D.Model(cfg["model"])
    opts = D.default_opts(work_queue=1)
    _check_pair(D, model, _t(cfg["x0"]), None, 1, 0.05, opts)
    _check_pair(D, model, _t(cfg["x0"][:37]), None, 1, 0.05, opts)


def test_noalloc_matches_rollout_chain_and_stack(D):
    """A controlled chain batch and a stack batch, each twice (smaller second)."""
    cfg = W.chain_walk(seed=3, n_worlds=300, n_intervals=3)
    model = D.Model(cfg["model"])
    opts = D.default_opts(work_queue=1)
    _check_pair(D, model, _t(cfg["x0"]), _t(cfg["u"]), 3, 0.01, opts)
    _check_pair(D, model, _t(cfg["x0"][:5]), _t(cfg["u"][:5]), 3, 0.01, opts)
    rng = np.random.default_rng(3)
    desc = W.model_stack(3)
    sm = D.Model(desc)
    xs = np.stack([W.stack_state(rng.normal(0, 0.02, (3, 2))) for _ in range(40)])
    _check_pair(D, sm, _t(xs), None, 1, 0.05, opts)
    _check_pair(D, sm, _t(xs[:3]), None, 1, 0.05, opts)
