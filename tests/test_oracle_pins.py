"""Pins of the oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: every expected value is a closed
form (free fall, rigid rotation, the damped contact oscillator of the
reference acceleration), an independent derivation (kinetic energy,
Lagrange's equations, slicing quadrature), a brute force (all active sets of
the convex contact problem), or a finite difference.
"""
import itertools

import numpy as np
import pytest
from scipy.integrate import quad
from scipy.linalg import expm
from scipy.optimize import brentq

from paper_2506_14186_amd import workloads as W

G = 9.81


# ------------------------------------------------------------------ helpers (test side)
def qmul(a, b):
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def qrot(th):
    a = np.linalg.norm(th)
    if a == 0:
        return np.array([1.0, 0, 0, 0])
    return np.concatenate([[np.cos(a / 2)], np.sin(a / 2) * th / a])


def qmat(q):
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def sphere_state(z, vz=0.0, vx=0.0, vy=0.0, w=(0, 0, 0)):
    return np.array([0.0, 0.0, z, 1, 0, 0, 0, vx, vy, vz, *w], dtype=float)


# ------------------------------------------------------------------ integrator
def test_free_fall_parabola(oracle):
    """No contact: DOPRI5 reproduces the quadratic free-fall trajectory exactly."""
    m = oracle.Model(W.model_sphere())
    x0 = np.array([0.3, -0.2, 5.0, 1, 0, 0, 0, 0.7, -0.4, 1.5, 0, 0, 0])
    T = 0.6
    r = m.rollout(x0, None, 1, T)
    assert r["status"] == 0
    p = x0[:3] + x0[7:10] * T + 0.5 * np.array([0, 0, -G]) * T * T
    v = x0[7:10] + np.array([0, 0, -G]) * T
    np.testing.assert_allclose(r["x"][:3], p, rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(r["x"][7:10], v, rtol=1e-14, atol=1e-14)


def test_paper_settings_are_the_defaults(oracle):
    """The printed controller and contact settings (tests/golden/paper_settings.json,
    App. E.1) are what the oracle, the library and the cube workloads use: the
    step factor safety * err^-(P+I)/k * err_prev^(P)/k of a PID controller with
    D = 0 has exponents kP + kI = P + I and kP = P; the cube's pairs carry the
    printed solimp and damping ratio (its time constant is the benchmark's)."""
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_settings.json")))
    P, I, Dd = g["pid"]["P"], g["pid"]["I"], g["pid"]["D"]
    assert Dd == 0.0
    assert oracle.DEFAULT_OPTS["kP"] == P and oracle.DEFAULT_OPTS["kI"] == I
    from paper_2506_14186_amd import dmx as D
    o = D.default_opts()
    assert (o.kP, o.kI) == (P, I)
    desc = W.model_cube_corners()
    for pr in desc["pairs"]:
        assert pr["solimp"] == g["cube_toss_contact"]["solimp"]
        assert pr["solref"][1] == g["cube_toss_contact"]["solref"][1]
    assert W.SOLIMP_DEFAULT == g["cube_toss_contact"]["solimp"]


def test_controller_free_fall_step_sequence(oracle):
    """PI controller with P=0.2, I=0.4 (App. E.1) at roundoff-level error:
    growth factor 0.9 * floor^(-0.12) * eprev^(0.04), first with eprev = 1."""
    m = oracle.Model(W.model_sphere())
    x0 = sphere_state(50.0)
    r = m.rollout(x0, None, 1, 2.0, log_cap=100, h_levels=0)
    log = r["log"]
    assert np.all(log[:, 3] == 1.0)  # nothing rejected
    h = log[:, 1]
    assert h[0] == 1e-3
    f1 = 0.9 * (1e-6) ** (-0.12)
    f2 = f1 * (1e-6) ** 0.04
    assert h[1] / h[0] == pytest.approx(f1, rel=1e-12)
    for k in range(2, len(h) - 1):  # the last step is clipped onto t_end
        assert h[k] / h[k - 1] == pytest.approx(min(f2, 10.0), rel=1e-12)
    assert log[-1, 0] + h[-1] == pytest.approx(2.0, rel=1e-15)
    # with the step grid (16 mantissa levels per octave) every proposed step is
    # the largest grid value not above the continuous proposal
    r = m.rollout(x0, None, 1, 2.0, log_cap=100, h_levels=16)
    hq = r["log"][:, 1]
    grid = lambda x: 2.0 ** np.floor(np.log2(x)) * np.floor(x / 2.0 ** np.floor(np.log2(x)) * 16) / 16  # noqa: E731
    assert hq[0] == grid(1e-3)
    for k in range(1, len(hq) - 1):
        f = f1 if k == 1 else min(f2, 10.0)
        assert hq[k] == grid(f * hq[k - 1])


def test_fifth_order_convergence(oracle):
    """Fixed (forced) steps on a smooth contact-free chain: global error falls
    as h^5 (Dormand-Prince weights) and the embedded estimate as h^5."""
    m = oracle.Model(W.model_pendulum(3))
    x0 = np.zeros(m.nx)
    x0[0], x0[1], x0[2] = 0.9, -0.6, 0.05
    x0[4] = 1.5
    u = np.zeros((1, m.nu))
    T = 0.4

    def run(n, T=T):
        h = T / n
        forced = np.array([[k * h, h] for k in range(n)])
        # absolute error scale (atol 1, rtol 0): the log holds the RMS local error estimate
        return m.rollout(x0, u, 1, T, forced=forced.ravel(), log_cap=n, atol=1.0, rtol=0.0)

    ref = run(1280)["x"]
    e = [np.linalg.norm(run(n)["x"] - ref) for n in (40, 80, 160)]
    assert 28 < e[0] / e[1] < 40 and 28 < e[1] / e[2] < 40
    # local error estimate of one step, halving h
    l = [run(1, T=h)["log"][0, 2] for h in (0.01, 0.005, 0.0025)]
    assert 28 < l[0] / l[1] < 36 and 28 < l[1] / l[2] < 36


# ------------------------------------------------------------------ rigid body dynamics
def test_spherical_body_constant_spin(oracle):
    """Isotropic inertia, no torque: q(T) = q0 * exp(w T / 2) for body-frame w."""
    m = oracle.Model(W.model_sphere())
    rng = np.random.default_rng(5)
    q0 = W.uniform_quat(rng, 1)[0]
    w = np.array([1.3, -0.7, 2.1])
    x0 = np.concatenate([[0, 0, 100.0], q0, [0, 0, 0], w])
    T = 0.9
    r = m.rollout(x0, None, 1, T, rtol=1e-10, atol=1e-12)
    qT = qmul(q0, qrot(w * T))
    if qT[0] * r["x"][3] < 0:
        qT = -qT
    np.testing.assert_allclose(r["x"][3:7], qT, atol=1e-13)
    np.testing.assert_allclose(r["x"][10:13], w, atol=1e-13)


def test_axisymmetric_torque_free_precession(oracle):
    """Euler's equations for I1 = I2: w3 constant, (w1, w2) rotate at
    (I3 - I1) w3 / I1 in the body frame."""
    m = oracle.Model(W.model_free_box(half=(0.1, 0.1, 0.25), mass=2.0))
    _, I, _ = m.inertia()
    I1, I3 = I[0, 0, 0], I[0, 2, 2]
    w0 = np.array([0.8, -0.3, 3.0])
    x0 = np.concatenate([[0, 0, 100.0], [1, 0, 0, 0], [0, 0, 0], w0])
    T = 1.3
    r = m.rollout(x0, None, 1, T, rtol=1e-10, atol=1e-12)
    Om = (I3 - I1) * w0[2] / I1
    c = (w0[0] + 1j * w0[1]) * np.exp(1j * Om * T)
    np.testing.assert_allclose(r["x"][10:13], [c.real, c.imag, w0[2]], atol=2e-8)


def test_asymmetric_tumbling_conserves_energy_and_momentum(oracle):
    """Torque-free asymmetric body: energy and |L| = |I w_body| are invariants
    of Euler's equations.  (The world direction of L is not checked: the
    orientation update combines the stage angular velocities before the
    exponential map, as in MuJoCo's Runge-Kutta, which omits the commutator
    term of the rotation and is second order in orientation.)"""
    m = oracle.Model(W.model_free_box())
    mass, I, _ = m.inertia()
    x0 = np.concatenate([[0, 0, 100.0], [0.9, 0.1, -0.3, 0.2], [0.4, -0.2, 1.0], [0.3, 4.0, 0.2]])
    x0[3:7] /= np.linalg.norm(x0[3:7])

    def invariants(x):
        R = qmat(x[3:7])
        w = x[10:13]
        E = 0.5 * mass[0] * x[7:10] @ x[7:10] + 0.5 * w @ I[0] @ w + mass[0] * G * x[2]
        return E, np.linalg.norm(I[0] @ w), np.linalg.norm(R @ (I[0] @ w))

    r = m.rollout(x0, None, 1, 2.0, rtol=1e-10, atol=1e-12)
    E0, L0, Lw0 = invariants(x0)
    E1, L1, Lw1 = invariants(r["x"])
    assert abs(E1 - E0) / abs(E0) < 1e-8
    assert L1 == pytest.approx(L0, rel=1e-8)
    assert Lw1 == pytest.approx(L1, rel=1e-12)  # the rotation matrix stays orthonormal


@pytest.mark.parametrize("kind,size,mass", [("sphere", (0.07, 0, 0), 1.3), ("box", (0.1, 0.15, 0.2), 2.0),
                                            ("capsule", (0.03, 0.125, 0), None)])
def test_primitive_inertia_by_slicing(oracle, kind, size, mass):
    """Mass and inertia of the solid primitives by 1-D slicing quadrature."""
    body = {"parent": -1, "pos": [0, 0, 0], "quat": [1, 0, 0, 0],
            "inertial": {"type": kind, "size": list(size), "mass": mass},
            "joints": [{"type": "free", "axis": [0, 0, 1], "pos": [0, 0, 0]}]}
    desc = {"gravity": [0, 0, -G], "bodies": [body], "geoms": [W._plane()], "pairs": [], "ctrl": {"dofs": []}}
    m = oracle.Model(desc)
    mm, I, _ = m.inertia()
    if kind == "box":
        a, b, c = size
        vol = 8 * a * b * c
        area = lambda z: 4 * a * b  # noqa: E731
        ixx_sec = lambda z: (2 * b) ** 2 / 12  # per unit mass of the slice, about its centre  # noqa: E731
        iyy_sec = lambda z: (2 * a) ** 2 / 12  # noqa: E731
        izz_sec = lambda z: ((2 * a) ** 2 + (2 * b) ** 2) / 12  # noqa: E731
        zmax = c
    else:
        r, h = size[0], size[1]
        rho2 = lambda z: r * r if abs(z) <= h else max(r * r - (abs(z) - h) ** 2, 0.0)  # noqa: E731
        area = lambda z: np.pi * rho2(z)  # noqa: E731
        ixx_sec = iyy_sec = lambda z: rho2(z) / 4  # noqa: E731
        izz_sec = lambda z: rho2(z) / 2  # noqa: E731
        zmax = h + r
    pts = [-zmax, zmax] if kind == "box" else [-zmax, -size[1], size[1], zmax] if kind == "capsule" else [-zmax, zmax]
    integ = lambda f: sum(quad(f, lo, hi, epsabs=0, epsrel=1e-13, limit=200)[0]  # noqa: E731
                          for lo, hi in zip(pts[:-1], pts[1:]) if hi > lo)
    V = integ(area)
    rho = (mass / V) if mass is not None else 1000.0
    if kind == "box":
        V = vol
    assert mm[0] == pytest.approx(rho * V, rel=1e-10)
    Ixx = rho * integ(lambda z: area(z) * (ixx_sec(z) + z * z))
    Iyy = rho * integ(lambda z: area(z) * (iyy_sec(z) + z * z))
    Izz = rho * integ(lambda z: area(z) * izz_sec(z))
    np.testing.assert_allclose(np.diag(I[0]), [Ixx, Iyy, Izz], rtol=1e-9)


def _random_chain_state(m, rng):
    q = rng.uniform(-1.0, 1.0, m.nq)
    v = rng.uniform(-2.0, 2.0, m.nv)
    return q, v


@pytest.mark.parametrize("model", ["chain", "pendulum"])
def test_mass_matrix_is_kinetic_energy_hessian(oracle, model):
    """M_ij from the polarization of the kinetic energy of the body twists."""
    desc = W.model_chain() if model == "chain" else W.model_pendulum(3)
    m = oracle.Model(desc)
    rng = np.random.default_rng(11)
    mass, I, _ = m.inertia()
    for _ in range(3):
        q, _ = _random_chain_state(m, rng)
        M = m.kinematics(q)["M"]

        def T(v):
            k = m.kinematics(q, v)
            e = 0.0
            for b in range(m.nb):
                R = k["xmat"][b]
                w, vb = k["twist"][b, :3], k["twist"][b, 3:]
                e += 0.5 * mass[b] * vb @ vb + 0.5 * w @ (R @ I[b] @ R.T) @ w
            return e

        E = np.eye(m.nv)
        Mt = np.array([[T(E[i] + E[j]) - T(E[i]) - T(E[j]) if i != j else 2 * T(E[i]) for j in range(m.nv)]
                       for i in range(m.nv)])
        np.testing.assert_allclose(M, Mt, rtol=1e-11, atol=1e-13)
        assert np.all(np.linalg.eigvalsh(M) > 0)


@pytest.mark.parametrize("model", ["chain", "pendulum"])
def test_bias_force_matches_lagrange(oracle, model):
    """c = (dM/dt) v - dT/dq + dV/dq by central differences of M(q) and V(q)."""
    desc = W.model_chain() if model == "chain" else W.model_pendulum(3)
    m = oracle.Model(desc)
    mass, _, _ = m.inertia()
    rng = np.random.default_rng(12)
    eps = 1e-6
    for _ in range(3):
        q, v = _random_chain_state(m, rng)
        c = m.kinematics(q, v)["c"]

        def Mq(qq):
            return m.kinematics(qq)["M"]

        def V(qq):
            return -sum(mass[b] * np.array([0, 0, -G]) @ m.kinematics(qq)["xpos"][b] for b in range(m.nb))

        cfd = np.zeros(m.nv)
        for k in range(m.nq):
            dq = np.zeros(m.nq)
            dq[k] = eps
            dM = (Mq(q + dq) - Mq(q - dq)) / (2 * eps)
            cfd += dM @ v * v[k]
            cfd[k] += -0.5 * v @ dM @ v + (V(q + dq) - V(q - dq)) / (2 * eps)
        np.testing.assert_allclose(c, cfd, rtol=1e-6, atol=1e-7)


def test_point_jacobian_is_point_velocity(oracle):
    """J(q) v equals the time derivative of a body-fixed point along v."""
    rng = np.random.default_rng(13)
    m = oracle.Model(W.model_chain())
    eps = 1e-6
    for b in range(m.nb):
        q, v = _random_chain_state(m, rng)
        k = m.kinematics(q)
        c = rng.normal(size=3) * 0.1
        P = k["xpos"][b] + k["xmat"][b] @ c
        J = m.point_jac(q, b, P)

        def pos(qq):
            kk = m.kinematics(qq)
            return kk["xpos"][b] + kk["xmat"][b] @ c

        fd = (pos(q + eps * v) - pos(q - eps * v)) / (2 * eps)
        np.testing.assert_allclose(J @ v, fd, rtol=1e-7, atol=1e-9)
    # free body: integrate the orientation with the body-frame angular velocity
    m = oracle.Model(W.model_free_box())
    q = np.concatenate([[0.1, -0.2, 0.3], W.uniform_quat(rng, 1)[0]])
    v = rng.normal(size=6)
    c = np.array([0.05, -0.07, 0.11])
    R = qmat(q[3:])
    P = q[:3] + R @ c
    J = m.point_jac(q, 0, P)

    def pos(s):
        qq = qmul(q[3:], qrot(s * v[3:]))
        return q[:3] + s * v[:3] + qmat(qq) @ c

    fd = (pos(eps) - pos(-eps)) / (2 * eps)
    np.testing.assert_allclose(J @ v, fd, rtol=1e-7, atol=1e-9)


# ------------------------------------------------------------------ contact solve
def _brute_force_qacc(M, a0, J, aref, D):
    """Enumerate all active sets of the convex piecewise-quadratic problem; the
    KKT-consistent one is the unique minimizer."""
    n = len(aref)
    sols = []
    for mask in itertools.product([0, 1], repeat=n):
        A = np.array(mask, bool)
        H = M + (J[A].T * D[A]) @ J[A]
        b = M @ a0 + (J[A].T * D[A]) @ aref[A]
        x = np.linalg.solve(H, b)
        s = J @ x - aref
        tol = 1e-9 * (1 + np.abs(aref))
        if np.all(s[A] <= tol[A]) and np.all(s[~A] >= -tol[~A]):
            sols.append(x)
    return sols


def test_newton_matches_brute_force_active_sets(oracle):
    rng = np.random.default_rng(21)
    m = oracle.Model(W.model_cube_corners(mu=0.8))
    checked = 0
    for trial in range(200):
        q = W.uniform_quat(rng, 1)[0]
        R = qmat(q)
        corners = np.array([[(1 if k & 1 else -1), (1 if k & 2 else -1), (1 if k & 4 else -1)] for k in range(8)]) * 0.1
        zmin = (corners @ R.T)[:, 2].min() - 0.01
        x = np.concatenate([[0, 0, -zmin - rng.uniform(0.0005, 0.004)], q, rng.normal(size=6)])
        rows = m.rows(x)
        n = len(rows["aref"])
        if n == 0 or n > 12:
            continue
        xd, info = m.rhs(x)
        sols = _brute_force_qacc(rows["M"], rows["a0"], rows["J"], rows["aref"], rows["D"])
        assert len(sols) >= 1
        for s in sols:
            np.testing.assert_allclose(xd[6:], s, rtol=1e-9, atol=1e-9)
        checked += 1
        if checked >= 12:
            break
    assert checked >= 6


def _imp(r, si):
    """MuJoCo's impedance spline of |r| (test-side, for the equilibrium equation)."""
    d0, dw, w, mid, p = si
    x = min(1.0, abs(r) / w)
    y = x ** p / mid ** (p - 1) if x <= mid else 1 - (1 - x) ** p / (1 - mid) ** (p - 1)
    return d0 + y * (dw - d0)


@pytest.mark.parametrize("solimp", [(0.9, 0.95, 0.001, 0.5, 2.0), (0.3, 0.95, 0.002, 0.3, 3.0),
                                    (0.0, 0.95, 0.001, 0.5, 2.0)])
def test_impedance_spline_and_reference_acceleration(oracle, solimp):
    """Sec. 2.1: the rows of a single sphere contact carry the impedance d(r) of
    the solimp spline through D = d / (A (1 - d)) with A = (1 + mu^2) / m, and
    a_ref = -b (J v) - k r with b = 2 / (d_w t_c), k = d / (d_w^2 t_c^2 phi^2).
    Recover d from D at depths on both arms of the spline (and beyond the
    width) and compare with the spline written out; check a_ref row by row."""
    mu, tc, phi, mass, rad = 0.7, 0.004, 0.8, 1.7, 0.05
    desc = W.model_sphere(radius=rad, mass=mass, mu=mu, tc=tc, solimp=solimp, dampratio=phi)
    m = oracle.Model(desc)
    d0, dw, wid, mid, pw = solimp
    A = (1 + mu * mu) / mass
    b = 2.0 / (dw * tc)
    for x in (0.05, 0.2, mid - 1e-3, mid, mid + 1e-3, 0.6, 0.95, 1.0, 1.7):
        r = -x * wid
        st = sphere_state(rad + r, vz=-0.3, vx=0.2, vy=-0.1)
        rows = m.rows(st)
        assert rows["J"].shape[0] == 4 and np.all(rows["D"] == rows["D"][0])
        Dv = rows["D"][0]
        d = Dv * A / (1 + Dv * A)
        assert d == pytest.approx(_imp(r, solimp), rel=1e-12, abs=1e-15), x
        k = d / (dw * dw * tc * tc * phi * phi)
        jv = rows["J"] @ st[7:]
        np.testing.assert_allclose(rows["aref"], -b * jv - k * r, rtol=1e-12, atol=1e-12)
    # no rows without penetration (the CFD field is off)
    assert m.rows(sphere_state(rad + 1e-4))["J"].shape[0] == 0


def test_cfd_impedance_continues_the_spline(oracle):
    """Sec. 4: for 0 <= r < w_c the CFD spline takes d from d_0 at r = 0 to d_c
    at r = w_c (with its own midpoint and power), continuing the penetration
    spline's value d(0) = d_0 without a jump."""
    si = (0.1, 0.95, 0.001, 0.5, 2.0)
    cf = (0.0, 0.1, 0.05, 0.4, 4.0)  # (d_c, d_0, w_c, midpoint, power)
    mu, mass, rad = 0.5, 1.0, 0.05
    desc = W.model_sphere(radius=rad, mass=mass, mu=mu, solimp=si, cfd=cf)
    m = oracle.Model(desc)
    A = (1 + mu * mu) / mass
    dc, dz, wc, mc, pc = cf
    for x in (0.0, 0.1, 0.3, 0.4, 0.5, 0.8, 0.99):
        r = x * wc
        rows = m.rows(sphere_state(rad + r), cfd=True)
        assert rows["J"].shape[0] == 4
        Dv = rows["D"][0]
        d = Dv * A / (1 + Dv * A)
        y = x ** pc / mc ** (pc - 1) if x <= mc else 1 - (1 - x) ** pc / (1 - mc) ** (pc - 1)
        assert d == pytest.approx(dz + y * (dc - dz), rel=1e-12, abs=1e-15), x
    # beyond w_c no row; just inside the surface the penetration spline starts at d_0
    assert m.rows(sphere_state(rad + 1.01 * wc), cfd=True)["J"].shape[0] == 0
    Dv = m.rows(sphere_state(rad - 1e-12), cfd=True)["D"][0]
    assert Dv * A / (1 + Dv * A) == pytest.approx(si[0], rel=1e-6)


def test_resting_sphere_steady_penetration(oracle):
    """At rest the 4 pyramid edges each carry m g / 4; with f = D (-k r),
    D = d / (A (1 - d)), k = d / (dw^2 tc^2 phi^2), A = (1 + mu^2) / m, the
    settled penetration r* solves d(r)^2 r = -(1 + mu^2) g (1 - d) dw^2 tc^2 / 4."""
    desc = W.model_sphere()
    si = desc["pairs"][0]["solimp"]
    tc, phi = desc["pairs"][0]["solref"]
    mu = desc["pairs"][0]["mu"]
    f = lambda r: _imp(r, si) ** 2 * r + (1 + mu * mu) * G * (1 - _imp(r, si)) * si[1] ** 2 * tc ** 2 * phi ** 2 / 4  # noqa: E731
    rstar = brentq(f, -1e-4, -1e-9, xtol=1e-16)
    assert rstar == pytest.approx(-2.186043e-6, rel=1e-6)
    assert _imp(rstar, si) == pytest.approx(0.90000048, abs=1e-8)
    m = oracle.Model(desc)
    r = m.rollout(sphere_state(0.1), None, 1, 0.5, rtol=1e-9, atol=1e-12)
    assert r["status"] == 0
    assert r["x"][2] - 0.1 == pytest.approx(rstar, abs=1e-11)
    np.testing.assert_allclose(r["x"][7:], 0.0, atol=1e-9)


def _oscillator(d, tc, phi, mu, mass=1.0):
    """Frictionless-direction contact with constant impedance d: the 4 identical
    edge rows act with d_eff = 1 / (1 + (1 + mu^2)(1 - d)/(4 d)); the gap obeys
    r'' = -(1 - d_eff) g + d_eff (-b r' - k r)."""
    deff = 1.0 / (1.0 + (1 + mu * mu) * (1 - d) / (4 * d))
    b = 2.0 / (d * tc)
    k = d / (d * d * tc * tc * phi * phi)
    A = np.array([[0.0, 1.0], [-deff * k, -deff * b]])
    rss = -(1 - deff) * G / (deff * k)
    return A, rss


def test_constant_impedance_transient(oracle):
    """Impact with constant impedance follows the linear damped oscillator."""
    d, tc = 0.9, 0.002
    desc = W.model_sphere(mu=0.0, tc=tc, solimp=(d, d, 0.001, 0.5, 2.0))
    m = oracle.Model(desc)
    A, rss = _oscillator(d, tc, 1.0, 0.0)
    r0, v0 = -1e-6, -0.5
    T = 0.004
    res = m.rollout(sphere_state(0.1 + r0, vz=v0), None, 1, T, rtol=1e-11, atol=1e-13, tape_cap=100000)
    tape = res["tape"]
    for t, hh, *y in tape[::7]:
        y = np.array(y)
        z = expm(A * t) @ np.array([r0 - rss, v0]) + np.array([rss, 0.0])
        assert y[2] - 0.1 < 0  # stays in contact over the window
        assert y[2] - 0.1 == pytest.approx(z[0], abs=1e-11)
        assert y[9] == pytest.approx(z[1], abs=1e-8)


# ------------------------------------------------------------------ derivatives
def test_contact_free_gradients(oracle):
    m = oracle.Model(W.model_sphere())
    x0 = np.concatenate([[0.1, 0.2, 10.0], [1, 0, 0, 0], [0.3, -0.1, 0.5], [0, 0, 0]])
    T = 0.7
    E = np.eye(13)
    j = m.rollout_jvp(x0, None, 1, T, E[[2, 7, 9]])
    tx = j["tx"]
    assert tx[0, 2] == pytest.approx(1.0, abs=1e-12)   # dz/dz0
    assert tx[1, 2] == pytest.approx(0.0, abs=1e-12)   # dz/dvx0
    assert tx[1, 0] == pytest.approx(T, abs=1e-12)     # dx/dvx0
    assert tx[2, 2] == pytest.approx(T, abs=1e-12)     # dz/dvz0
    assert tx[2, 9] == pytest.approx(1.0, abs=1e-12)   # dvz/dvz0


def test_sustained_contact_gradient_is_oscillator_flow(oracle):
    """In persistent contact with constant impedance the state map is linear:
    d(r, r')(T)/d(r, r')(0) = expm(A T)."""
    d, tc = 0.9, 0.002
    m = oracle.Model(W.model_sphere(mu=0.0, tc=tc, solimp=(d, d, 0.001, 0.5, 2.0)))
    A, rss = _oscillator(d, tc, 1.0, 0.0)
    x0 = sphere_state(0.1 + rss - 2e-6, vz=-0.001)
    T = 0.01
    E = np.eye(13)
    j = m.rollout_jvp(x0, None, 1, T, E[[2, 9]], rtol=1e-11, atol=1e-13)
    Phi = expm(A * T)
    got = np.array([[j["tx"][0, 2], j["tx"][1, 2]], [j["tx"][0, 9], j["tx"][1, 9]]])
    np.testing.assert_allclose(got, Phi, rtol=1e-7, atol=1e-9)


def _fd_frozen(m, x0, u, n_int, dt, dirs, eps=1e-6, **opts):
    base = m.rollout(x0, u, n_int, dt, tape_cap=200000, **opts)
    forced = base["tape"][:, :2].ravel()
    out = []
    for d in dirs:
        xp = m.rollout(x0 + eps * d, u, n_int, dt, forced=forced, **opts)["x"]
        xm = m.rollout(x0 - eps * d, u, n_int, dt, forced=forced, **opts)["x"]
        out.append((xp - xm) / (2 * eps))
    return np.array(out)


@pytest.mark.parametrize("name", ["cube", "chain"])
def test_rollout_derivative_matches_frozen_step_fd(oracle, name):
    """Forward-mode derivative of the discretized rollout vs central differences
    of the same step sequence replayed (discretize-then-optimize)."""
    rng = np.random.default_rng(31)
    if name == "cube":
        cfg = W.cube_toss(seed=2, n_worlds=4)
        m = oracle.Model(cfg["model"])
        x0 = cfg["x0"][1].copy()
        x0[2] = 0.16
        u, n_int, dt = None, 1, 0.08
    else:
        cfg = W.chain_walk(seed=3, n_worlds=2, n_intervals=4)
        m = oracle.Model(cfg["model"])
        x0 = cfg["x0"][0].copy()
        x0[1] = 0.5299  # feet 0.1 mm into the plane: contact persists over the window
        u, n_int, dt = cfg["u"][0], 4, 0.01
    dirs = rng.normal(size=(3, m.nx))
    # central differences are only valid while no contact switches on or off
    # (the damping term makes the force jump at r = 0)
    if name == "chain":
        tape = m.rollout(x0, u, n_int, dt, tape_cap=100000)["tape"]
        r = np.array([m.contacts(y[2:2 + m.nq])[:, 0] for y in tape])
        assert not np.any(np.diff((r < 0).astype(int), axis=0))
    fd = _fd_frozen(m, x0, u, n_int, dt, dirs)
    j = m.rollout_jvp(x0, u, n_int, dt, dirs)
    assert j["status"] == 0
    np.testing.assert_allclose(j["tx"], fd, rtol=2e-5, atol=2e-6 * np.abs(fd).max())


def test_rhs_tangent_matches_fd_with_and_without_cfd(oracle):
    rng = np.random.default_rng(41)
    m = oracle.Model(W.model_cube_corners())
    q = W.uniform_quat(rng, 1)[0]
    R = qmat(q)
    corners = np.array([[(1 if k & 1 else -1), (1 if k & 2 else -1), (1 if k & 4 else -1)] for k in range(8)]) * 0.1
    zmin = (corners @ R.T)[:, 2].min() - 0.01
    x = np.concatenate([[0, 0, -zmin - 0.002], q, rng.normal(size=6)])
    dirs = rng.normal(size=(3, m.nx))
    eps = 1e-7
    for st in (False, True):
        val, tan = m.rhs_jvp(x, None, dirs, st=st)
        np.testing.assert_array_equal(val, m.rhs(x)[0])  # value is always F
        for i, d in enumerate(dirs):
            fp = m.rhs(x + eps * d, cfd=st)[0]
            fm = m.rhs(x - eps * d, cfd=st)[0]
            np.testing.assert_allclose(tan[i], (fp - fm) / (2 * eps), rtol=1e-5, atol=1e-5 * np.abs(tan[i]).max())


def test_gradient_is_transpose_of_tangent(oracle):
    """<x0bar, dx> = <xbar, J dx> (dot-product test of the batched gradient)."""
    cfg = W.cube_toss(seed=2, n_worlds=2, horizon=0.1)
    m = oracle.Model(cfg["model"])
    x0 = cfg["x0"].copy()
    x0[:, 2] = 0.15
    rng = np.random.default_rng(51)
    xbar = rng.normal(size=x0.shape)
    g = m.grad_batch(x0, None, 1, 0.1, xbar, n_threads=2)
    for w in range(2):
        d = rng.normal(size=m.nx)
        j = m.rollout_jvp(x0[w], None, 1, 0.1, d)
        assert g["x0bar"][w] @ d == pytest.approx(xbar[w] @ j["tx"][0], rel=1e-11)


def test_batch_equals_single(oracle):
    cfg = W.cube_toss(seed=2, n_worlds=3, horizon=0.1)
    m = oracle.Model(cfg["model"])
    b = m.rollout_batch(cfg["x0"], None, 1, 0.1, n_threads=3)
    for w in range(3):
        s = m.rollout(cfg["x0"][w], None, 1, 0.1)
        np.testing.assert_array_equal(b["x"][w], s["x"])


# ------------------------------------------------------------------ contacts from distance
def test_cfd_leaves_forward_unchanged_and_informs_gradient(oracle):
    """Straight-through CFD (Sec. 4): the rollout is unchanged; far from the
    plane (r > w_c throughout) the gradient equals the plain one; passing
    within w_c without touching gives a gradient the plain model lacks."""
    m = oracle.Model(W.model_sphere())
    E = np.eye(13)
    far = sphere_state(1.0, vz=0.5)
    a = m.rollout_jvp(far, None, 1, 0.2, E[[2, 9]], cfd=0)
    b = m.rollout_jvp(far, None, 1, 0.2, E[[2, 9]], cfd=1)
    np.testing.assert_array_equal(a["x"], b["x"])
    np.testing.assert_allclose(a["tx"], b["tx"], rtol=0, atol=1e-14)
    # skim: apex 5 mm above the plane, inside w_c = 1 cm
    skim = sphere_state(0.105, vz=0.0, vx=0.3)
    a = m.rollout_jvp(skim, None, 1, 0.03, E[[2, 7]], cfd=0)
    b = m.rollout_jvp(skim, None, 1, 0.03, E[[2, 7]], cfd=1)
    np.testing.assert_array_equal(a["x"], b["x"])
    assert a["x"][2] > 0.1  # never touched
    assert abs(b["tx"][0, 2] - a["tx"][0, 2]) > 1e-3


def test_box_plane_flat_face_gives_four_equal_corners(oracle):
    """A box resting flat with penetration delta: the four bottom vertices at
    r = -delta, contact points at the midpoints; rotation about the plane
    normal leaves the depths unchanged."""
    delta = 0.003
    hs = (0.1, 0.1, 0.1)
    body = {"parent": -1, "pos": [0, 0, 0], "quat": [1, 0, 0, 0],
            "inertial": {"type": "box", "size": list(hs), "mass": 1.0},
            "joints": [{"type": "free", "axis": [0, 0, 1], "pos": [0, 0, 0]}]}
    desc = {"gravity": [0, 0, -G], "bodies": [body],
            "geoms": [W._plane(), {"body": 0, "type": "box", "size": list(hs), "pos": [0, 0, 0], "quat": [1, 0, 0, 0]}],
            "pairs": [W._pair(0, 1, 0.6, 0.002)], "ctrl": {"dofs": []}}
    m = oracle.Model(desc)
    for ang in (0.0, 0.37, 1.2):
        q = np.concatenate([[0.2, -0.1, 0.1 - delta], qrot(np.array([0, 0, ang]))])
        c = m.contacts(q)
        assert len(c) == 4
        np.testing.assert_allclose(c[:, 0], -delta, atol=1e-15)
        R = qmat(q[3:])
        bottom = np.array([[sx, sy, -0.1] for sy in (-0.1, 0.1) for sx in (-0.1, 0.1)])
        expect = q[:3] + bottom @ R.T + np.array([0, 0, delta / 2])
        np.testing.assert_allclose(c[:, 1:4], expect, atol=1e-14)
        np.testing.assert_allclose(c[:, 4:7], [[0, 0, 1]] * 4, atol=0)


# ------------------------------------------------------------------ CFD position term (softplus)
def _sphere_rows(oracle, z, beta, vz=-0.3):
    desc = W.model_sphere()
    om = oracle.Model(desc)
    x = sphere_state(z, vz=vz)
    rows = om.rows(x, cfd=True, beta=beta)
    plain = om.rows(x, cfd=False)
    pr = desc["pairs"][0]
    return om, x, rows, plain, pr


def test_cfd_position_term_limits(oracle):
    """The CFD field replaces F's position term k relu(-r) of a_ref by a
    softplus (Sec. 4).  Pinned by its limits, which fix its sign and scale
    without the softplus formula: (i) deep in penetration (beta |r| = 50) the
    CFD rows equal F's rows; (ii) at a gap r = +5 mm inside the CFD width the
    position term vanishes (a_ref = -b J v, the damping term alone); (iii) at
    r = 0 it equals k(0) log(2) / beta, the value of any softplus at 0, with
    k(0) = d_0 / (d_w^2 t_c^2 phi^2) and d_0 the CFD spline's value at the
    surface; (iv) between, it decreases with r and grows as beta falls."""
    beta = 1e4
    tc, phi = 0.002, 1.0
    # (i) penetration 5 mm: identical rows (softplus(-r) = -r to rounding)
    om, x, rows, plain, pr = _sphere_rows(oracle, 0.1 - 5e-3, beta)
    assert len(rows["aref"]) == 4 and len(plain["aref"]) == 4
    np.testing.assert_allclose(rows["aref"], plain["aref"], rtol=1e-13)
    np.testing.assert_allclose(rows["D"], plain["D"], rtol=1e-13)
    # (ii) gap 5 mm: F has no rows, the CFD rows carry only the damping term
    om, x, rows, plain, pr = _sphere_rows(oracle, 0.1 + 5e-3, beta)
    assert len(plain["aref"]) == 0 and len(rows["aref"]) == 4
    dw = pr["solimp"][1]
    b = 2.0 / (dw * tc)
    jv = rows["J"] @ x[7:]
    pos = rows["aref"] + b * jv
    assert np.abs(pos).max() <= 1e-12 * np.abs(b * jv).max()
    # (iii) touching: position term k(0) log 2 / beta on every edge
    d0 = pr["cfd"][1]
    om, x, rows, plain, pr = _sphere_rows(oracle, 0.1, beta)
    pos0 = rows["aref"] + b * (rows["J"] @ x[7:])
    k0 = d0 / (dw ** 2 * tc ** 2 * phi ** 2)
    np.testing.assert_allclose(pos0, k0 * np.log(2.0) / beta, rtol=1e-12)
    # (iv) monotone in r and in 1/beta
    vals = []
    for gap in (-2e-4, -5e-5, 0.0, 5e-5, 2e-4):
        _, x, rows, _, _ = _sphere_rows(oracle, 0.1 + gap, beta)
        vals.append((rows["aref"] + b * (rows["J"] @ x[7:]))[0])
    assert all(a > c for a, c in zip(vals, vals[1:]))
    _, x, soft, _, _ = _sphere_rows(oracle, 0.1 + 5e-5, 1e3)
    assert (soft["aref"] + b * (soft["J"] @ x[7:]))[0] > vals[3]


# ------------------------------------------------------------------ failed trial solves
def test_failed_trial_solve_rejects_the_attempt(oracle):
    """Reading of a contact solve that fails at a trial stage (its Newton
    iteration budget is spent): the attempt is rejected as if its error were
    infinite and the step shrinks by the controller's minimum factor; an
    accepted step never contains a failed solve.  With a budget of 4
    iterations some trial stages of tumbling cubes fail; every world still
    finishes, each failed attempt is a rejection followed by a step of
    facmin h (or the landing step), and replaying the accepted steps with the
    full budget reproduces the end state bit for bit (every accepted stage
    solve had converged)."""
    cfg = W.cube_toss(seed=2, n_worlds=8, horizon=0.5)
    om = oracle.Model(cfg["model"])
    failed = 0
    for w in range(8):
        r = om.rollout(cfg["x0"][w], None, 1, 0.5, log_cap=20000, tape_cap=20000, newton_maxit=4)
        assert r["status"] == 0
        lg = r["log"]
        bad = np.where(np.isinf(lg[:, 2]))[0]
        failed += len(bad)
        for i in bad:
            assert lg[i, 3] == 0.0
            t1, h1 = lg[i + 1, 0], lg[i + 1, 1]
            assert t1 == lg[i, 0]
            assert h1 == 0.2 * lg[i, 1] or abs(t1 + h1 - 0.5) < 1e-15
        rep = om.rollout(cfg["x0"][w], None, 1, 0.5, forced=r["tape"][:, :2], newton_maxit=100)
        np.testing.assert_array_equal(rep["x"], r["x"])
    assert failed > 0


# ------------------------------------------------------------------ capsule-plane
def _free_capsule(radius=0.03, half=0.125):
    return {"name": "capsule", "gravity": [0.0, 0.0, -9.81],
            "bodies": [{"parent": -1, "pos": [0.0, 0.0, 0.0], "quat": [1.0, 0.0, 0.0, 0.0],
                        "inertial": {"type": "capsule", "size": [radius, half, 0.0], "mass": None},
                        "joints": [{"type": "free", "axis": [0.0, 0.0, 1.0], "pos": [0.0, 0.0, 0.0]}]}],
            "geoms": [{"body": -1, "type": "plane", "size": [0, 0, 0], "pos": [0, 0, 0], "quat": [1, 0, 0, 0]},
                      {"body": 0, "type": "capsule", "size": [radius, half, 0.0], "pos": [0, 0, 0],
                       "quat": [1, 0, 0, 0]}],
            "pairs": [W._pair(0, 1, 1.0, 0.002)], "ctrl": {"dofs": []}}


@pytest.mark.parametrize("tilt", [0.0, 0.3, np.pi / 2])
def test_capsule_plane_end_spheres(oracle, tilt):
    """Capsule against a plane (reading: both cap-end spheres, +axis end
    first, no case split): for a capsule of radius a and half-length h with
    its centre at height z and its axis tilted by th from the vertical, the
    +axis end sphere is centred at height z + h cos(th) and the other at
    z - h cos(th); the signed distances are those heights minus a, the points
    lie halfway between each end sphere's lowest point and the plane, and the
    normal is the plane's."""
    a, h, z = 0.03, 0.125, 0.2
    om = oracle.Model(_free_capsule(a, h))
    q = np.array([0.1, -0.2, z, np.cos(tilt / 2), np.sin(tilt / 2), 0.0, 0.0])
    c = om.contacts(q)
    assert c.shape[0] == 2
    for row, sgn in zip(c, (1.0, -1.0)):
        end = np.array([0.1, -0.2, z]) + sgn * h * np.array([0.0, -np.sin(tilt), np.cos(tilt)])
        r = end[2] - a
        np.testing.assert_allclose(row[0], r, atol=1e-15)
        np.testing.assert_allclose(row[1:4], end - np.array([0, 0, a + r / 2]), atol=1e-15)
        np.testing.assert_allclose(row[4:7], [0, 0, 1], atol=0)
