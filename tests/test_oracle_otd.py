"""Pins of the oracle's optimize-then-discretize gradient (App. C.2, eq.
adjoint-equations; with CFD, the straight-through adjoint of App. C.4): the
continuous adjoint equations solved backwards with their own adaptive steps
along the forward's continuous extension.

Each pin is independent of the oracle's formulas: the continuous extension
against quadrature exactness and its observed order of accuracy; the
adjoint against closed forms in free flight (state and control gradients)
and against the fundamental matrix of the linear oscillator of a sustained
constant-impedance contact; the gradient against central differences of the
forward at tolerance 1e-12 on the paper's cube toss; with CFD, against the
discrete straight-through gradient along ever smaller forced steps (both
approach the gradient of the continuous straight-through dynamics).
"""
import numpy as np
import pytest
from scipy.linalg import expm

from paper_2506_14186_amd import workloads as W
from test_oracle_pins import G, _oscillator, sphere_state

NODES = np.array([0.0, 1 / 5, 3 / 10, 4 / 5, 8 / 9, 1.0, 1.0])  # the Dormand-Prince nodes


def test_dense_output_integrates_cubics_exactly(oracle):
    """The continuous extension is a fourth-order interpolant: over a fraction
    theta of a step it integrates polynomial slopes of degree 3 exactly (and
    degree 4 at theta = 1, the fifth-order solution), and vanishes at 0."""
    for th in (0.0, 0.13, 0.5, 0.77, 1.0):
        w = oracle.dense_weights(th)
        for k in range(5 if th == 1.0 else 4):
            assert w @ NODES ** k == pytest.approx(th ** (k + 1) / (k + 1), abs=2e-15), (th, k)
    # not exact beyond: the interior interpolant has order 4, not 5
    assert abs(oracle.dense_weights(0.5) @ NODES ** 4 - 0.5 ** 5 / 5) > 1e-4


def test_dense_output_local_error_is_fifth_order(oracle):
    """Along forced uniform steps of a swinging double pendulum (smooth,
    nonlinear, no contact), x(tau) from the continuous extension at interior
    points converges at h^5: halving h divides the error by about 32."""
    m = oracle.Model(W.model_pendulum())
    x = np.zeros(m.nx)
    x[0], x[1], x[m.nq] = 1.2, -0.4, 0.5
    T, errs = 0.4, []
    for n in (8, 16, 32):
        h = T / n
        forced = np.array([[i * h, h] for i in range(n)]).ravel()
        taus = (np.arange(n) + 0.37) * h
        d = m.dense_states(x, None, 1, T, taus, forced=forced)
        ex = np.array([m.rollout(x, None, 1, t, rtol=1e-13, atol=1e-13)["x"] for t in taus])
        errs.append(np.max(np.abs(d - ex)))
    assert errs[0] / errs[1] > 20 and errs[1] / errs[2] > 20, errs


def test_otd_free_flight_closed_forms(oracle):
    """Cube high above the plane under gravity with forces u on its centre:
    z(T) = z0 + vz0 T - g T^2 / 2 + sum_k u_k dt (T - (k + 1/2) dt) / m, so
    dz/dz0 = 1, dz/dvz0 = T, dx/dvx0 = T and dz/du_k(z) = dt (T - (k + 1/2) dt)
    exactly; the adjoint's steps integrate these polynomials exactly."""
    m = oracle.Model(W.model_cube_corners(ctrl=True))
    n_int, dt = 5, 0.04
    T = n_int * dt
    x0 = np.array([0.1, 0.0, 20.0, 1, 0, 0, 0, 0.3, 0.0, 1.0, 0, 0, 0])
    u = np.zeros((1, n_int, 6))
    u[0, :, 2] = np.linspace(-1, 1, n_int)
    xb = np.zeros((1, 13))
    xb[0, 2], xb[0, 0] = 1.0, 1.0
    r = m.otd_grad_batch(x0[None], u, n_int, dt, xb, rtol=1e-8, atol=1e-8)
    assert r["status"][0] == 0
    g = r["x0bar"][0]
    assert g[2] == pytest.approx(1.0, abs=1e-12) and g[0] == pytest.approx(1.0, abs=1e-12)
    assert g[9] == pytest.approx(T, abs=1e-12) and g[7] == pytest.approx(T, abs=1e-12)
    want = dt * (T - (np.arange(n_int) + 0.5) * dt)  # mass 1
    np.testing.assert_allclose(r["ubar"][0, :, 2], want, rtol=0, atol=1e-12)
    np.testing.assert_allclose(r["ubar"][0, :, 0], want, rtol=0, atol=1e-12)  # x force, same lever in time


def test_otd_sustained_contact_is_oscillator_flow(oracle):
    """In persistent contact with constant impedance the dynamics of (r, r')
    are linear, so d r(T) / d(r, r')(0) is the first row of expm(A T)."""
    d, tc = 0.9, 0.002
    m = oracle.Model(W.model_sphere(mu=0.0, tc=tc, solimp=(d, d, 0.001, 0.5, 2.0)))
    A, rss = _oscillator(d, tc, 1.0, 0.0)
    x0 = sphere_state(0.1 + rss - 2e-6, vz=-0.001)
    T = 0.01
    xb = np.zeros((1, 13))
    xb[0, 2] = 1.0
    r = m.otd_grad_batch(x0[None], None, 1, T, xb, rtol=1e-10, atol=1e-12)
    Phi = expm(A * T)
    np.testing.assert_allclose(r["x0bar"][0, [2, 9]], Phi[0], rtol=1e-7, atol=1e-9)


def test_otd_matches_central_differences_on_the_cube_toss(oracle):
    """The paper's cube toss (solref (0.005, 1), solimp (0, 0.95, 0.001, 0.5,
    2), v_x = -2): the gradient of the toss distance in v_x against central
    differences of the forward at tolerance 1e-12 (the paper's ground truth,
    itself uncertain to about 1e-3 relative here), and against the discrete
    adjoint at the same tolerance (which converges more slowly)."""
    m = oracle.Model(W.model_box(tc=0.005, solimp=(0.0, 0.95, 0.001, 0.5, 2.0), mu=0.8))
    x0 = np.zeros((3, 13))
    x0[:, 2], x0[:, 3] = 0.3, 1.0
    x0[:, 7] = (-2.0, -1.5, -2.5)
    xb = np.zeros((3, 13))
    xb[:, 0] = 1.0
    eps = 1e-6
    fd = []
    for x in x0:
        xp, xm = x.copy(), x.copy()
        xp[7] += eps
        xm[7] -= eps
        fd.append((m.rollout(xp, None, 1, 1.0, rtol=1e-12, atol=1e-12)["x"][0]
                   - m.rollout(xm, None, 1, 1.0, rtol=1e-12, atol=1e-12)["x"][0]) / (2 * eps))
    fd = np.array(fd)
    otd = m.otd_grad_batch(x0, None, 1, 1.0, xb, n_threads=3, rtol=1e-10, atol=1e-10)
    assert (otd["status"] == 0).all()
    np.testing.assert_allclose(otd["x0bar"][:, 7], fd, rtol=3e-3)
    dto = m.grad_batch(x0, None, 1, 1.0, xb, n_threads=3, rtol=1e-8, atol=1e-8)
    otd8 = m.otd_grad_batch(x0, None, 1, 1.0, xb, n_threads=3, rtol=1e-8, atol=1e-8)
    assert np.max(np.abs(otd8["x0bar"][:, 7] - fd)) < np.max(np.abs(dto["x0bar"][:, 7] - fd))


def test_otd_with_cfd_is_the_continuous_straight_through_gradient(oracle):
    """A sphere skimming 5 mm above the plane, inside the CFD width, never
    touching: the forward takes a few large steps (the flight is polynomial).
    The discrete straight-through gradient unrolled along those steps is far
    off (the forward's controller does not see the CFD field, App. C.4);
    along forced ever smaller steps it converges, and the optimize-then-
    discretize gradient, whose adjoint picks its own steps, agrees with that
    limit."""
    m = oracle.Model(W.model_sphere())
    x = sphere_state(0.105, vz=0.0, vx=0.3)
    T = 0.03
    xb = np.zeros((1, 13))
    xb[0, 2] = 1.0
    E = np.eye(13)
    lim = []
    for h in (2e-5, 5e-6):
        n = int(round(T / h))
        forced = np.array([[i * h, h] for i in range(n)])
        xo, tx = m.rollout_jvp_forced(x, None, 1, T, forced, E[[2, 9]], cfd=1)
        assert xo[2] > 0.1
        lim.append(tx[:, 2])
    assert np.max(np.abs(lim[0] - lim[1])) < 1e-5
    otd = m.otd_grad_batch(x[None], None, 1, T, xb, cfd=1, rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(otd["x0bar"][0, [2, 9]], lim[1], rtol=1e-5, atol=1e-7)
    dto = m.grad_batch(x[None], None, 1, T, xb, n_threads=1, cfd=1)
    assert dto["n_acc"][0] < 10
    assert np.max(np.abs(dto["x0bar"][0, [2, 9]] - lim[1])) > 100 * np.max(np.abs(otd["x0bar"][0, [2, 9]] - lim[1]))


def test_otd_resolves_bounces_between_free_flights(oracle):
    """Spheres thrown onto the plane bounce and fly: in flight the adjoint
    equations are nearly linear and the adjoint's own steps grow fast, so a
    step crossing the forward's short steps through a bounce would leave the
    contact out of the gradient.  At rtol 1e-10 the continuous adjoint agrees
    with the forward-mode derivative of the discretized rollout (an
    independent method, itself within 5e-7 of the 1e-12 solve's) to 1e-5."""
    m = oracle.Model(W.model_sphere(radius=0.1, mu=0.8, tc=0.005, solimp=(0.0, 0.95, 0.001, 0.5, 2.0)))
    n = 4
    x0 = np.zeros((n, 13))
    x0[:, 2] = 0.3
    x0[:, 3] = 1.0
    x0[:, 7] = np.linspace(-3.0, -1.0, n)
    xb = np.zeros((n, 13))
    xb[:, 0] = 1.0
    otd = m.otd_grad_batch(x0, None, 1, 1.0, xb, n_threads=4, rtol=1e-10, atol=1e-10)
    dto = m.grad_batch(x0, None, 1, 1.0, xb, n_threads=4, rtol=1e-10, atol=1e-10)
    g_o, g_d = otd["x0bar"][:, 7], dto["x0bar"][:, 7]
    err = np.abs(g_o - g_d) / np.abs(g_d)
    print(f"sphere tosses, dL/dv_x: continuous vs discrete adjoint at rtol 1e-10: {err.max():.2e}")
    assert err.max() <= 1e-5, (g_o, g_d)
