"""Pins of the oracle's Tsitouras 5(4) pair (Tsit5, the solver of the
paper's experiments, App. E.1; opts tableau=1), independent of its
coefficient table: the fifth-order solution's global error along forced
uniform steps of a swinging double pendulum falls at least 20x per halving
of h (order >= 5; a wrong coefficient drops the order), free fall is
integrated exactly (a polynomial of degree 2), the embedded estimate falls
with h at fifth order (the local error of the fourth-order b-hat), and
adaptive runs meet their tolerance with step counts close to the
Dormand-Prince pair's."""
import numpy as np
import pytest

from paper_2506_14186_amd import workloads as W


def _pendulum(oracle):
    m = oracle.Model(W.model_pendulum())
    x = np.zeros(m.nx)
    x[0], x[1], x[m.nq] = 1.2, -0.4, 0.5
    return m, x


def test_tsit5_global_error_is_fifth_order(oracle):
    m, x = _pendulum(oracle)
    T = 0.4
    ex = m.rollout(x, None, 1, T, rtol=1e-13, atol=1e-13)["x"]
    errs = []
    for n in (8, 16, 32):
        h = T / n
        forced = np.array([[i * h, h] for i in range(n)]).ravel()
        errs.append(np.max(np.abs(m.rollout(x, None, 1, T, forced=forced, tableau=1)["x"] - ex)))
    assert errs[0] / errs[1] > 20 and errs[1] / errs[2] > 20, errs


def test_tsit5_free_fall_exact(oracle):
    m = oracle.Model(W.model_sphere())
    x0 = np.array([0.3, -0.2, 5.0, 1, 0, 0, 0, 0.7, -0.4, 1.5, 0, 0, 0])
    T = 0.6
    r = m.rollout(x0, None, 1, T, tableau=1)
    assert r["status"] == 0
    want = x0[:3] + x0[7:10] * T + np.array([0, 0, -0.5 * 9.81 * T * T])
    np.testing.assert_allclose(r["x"][:3], want, rtol=0, atol=1e-13)


def test_tsit5_error_estimate_order(oracle):
    """One step from the same state with h and h/2: the embedded estimate
    (the difference of the fifth- and fourth-order solutions, ~h^5) falls by
    about 32."""
    m, x = _pendulum(oracle)
    errs = []
    for h in (0.02, 0.01, 0.005):
        r = m.rollout(x, None, 1, h, log_cap=4, tableau=1, h0=h, rtol=1e-3, atol=1e-3)
        errs.append(r["log"][0, 2])
    assert 20 < errs[0] / errs[1] < 50 and 20 < errs[1] / errs[2] < 50, errs


@pytest.mark.parametrize("rtol", [1e-6, 1e-9])
def test_tsit5_adaptive_meets_tolerance(oracle, rtol):
    m, x = _pendulum(oracle)
    ex = m.rollout(x, None, 1, 2.0, rtol=1e-13, atol=1e-13)["x"]
    a = m.rollout(x, None, 1, 2.0, rtol=rtol, atol=rtol, tableau=1)
    b = m.rollout(x, None, 1, 2.0, rtol=rtol, atol=rtol, tableau=0)
    assert np.max(np.abs(a["x"] - ex)) < 100 * rtol
    assert 0.5 < a["n_acc"] / b["n_acc"] < 2.0
