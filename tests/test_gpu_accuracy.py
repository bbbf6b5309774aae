"""Gradient accuracy against the tolerance of the adaptive integrator (the
paper's error-versus-runtime study of the cube toss, Fig. 14 and App. B
"Error tolerances set gradient accuracy"): a cube (box geom) thrown at
v_x = -2 m/s (here v_x in [-3, -1], with a tilt) onto the plane with
solref (0.005, 1) and solimp (0, 0.95, 0.001, 0.5, 2), loss = the toss
distance x(T) at T = 1 s, and its gradient with respect to the initial
velocity v_x.  Ground truth: the oracle's gradient of the same rollout at
rtol = atol = 1e-12 (forward mode; central differences of that solve agree
to 5e-3, and the change from 1e-12 to 1e-13 is of the same order: the
active-set changes of the pyramidal friction make the derivative of F jump,
so the discrete gradient converges slowly near those instants).  The GPU
path (forward rollout, discrete adjoint) runs at rtol = atol from 1e-2 to
1e-9; the gradient error must fall with the tolerance (the paper's claim:
the tolerance sets the gradient error) and so must the loss error.  Runtime
of the batch is measured with events on the stream.  The optimize-then-
discretize gradient of the same rollouts (dmx_rollout_vjp_otd) is measured
beside it (App. C.2: the adjoint picks its own steps).
"""
import numpy as np
import pytest

from paper_2506_14186_amd import workloads as W

pytestmark = pytest.mark.gpu

RTOLS = [1e-2, 1e-3, 1e-4, 1e-5, 1e-6, 1e-7, 1e-8, 1e-9]
N = 16


@pytest.fixture(scope="module")
def D():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_14186_amd import dmx
    return dmx


def toss_model():
    return W.model_box(tc=0.005, solimp=(0.0, 0.95, 0.001, 0.5, 2.0), mu=0.8)


def toss_states():
    x0 = np.zeros((N, 13))
    x0[:, 2] = 0.3
    tilt = np.linspace(0.0, 0.3, N)
    x0[:, 3] = np.cos(tilt / 2)
    x0[:, 5] = np.sin(tilt / 2)  # about the y axis
    x0[:, 7] = np.linspace(-3.0, -1.0, N)
    return x0


def test_gradient_error_follows_tolerance(D, oracle):
    import torch
    desc = toss_model()
    x0 = toss_states()
    xb = np.zeros((N, 13))
    xb[:, 0] = 1.0
    om = oracle.Model(desc)
    ref = om.grad_batch(x0, None, 1, 1.0, xb, n_threads=16, rtol=1e-12, atol=1e-12)
    assert (np.asarray(ref["status"]) == 0).all()
    g_true, x_true = ref["x0bar"], ref["x"]
    # the ground truth against central differences of the same adaptive
    # solve (the paper's ground truth) in the initial velocity
    eps = 1e-6
    for w in (0, N // 2, N - 1):
        xp, xm = x0[w].copy(), x0[w].copy()
        xp[7] += eps
        xm[7] -= eps
        fd = (om.rollout(xp, None, 1, 1.0, rtol=1e-12, atol=1e-12)["x"][0]
              - om.rollout(xm, None, 1, 1.0, rtol=1e-12, atol=1e-12)["x"][0]) / (2 * eps)
        assert abs(fd - g_true[w, 7]) <= 5e-3 * abs(g_true[w, 7]), (w, fd, g_true[w, 7])
    model = D.Model(desc)
    x0t = torch.tensor(x0, dtype=torch.float64, device="cuda")
    xbt = torch.tensor(xb, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    rows = []
    for rtol in RTOLS:
        opts = D.default_opts(rtol=rtol, atol=rtol, tape_steps=65536, max_attempts=1000000)
        r = D.rollout(model, x0t, None, 1, 1.0, opts=opts, tape=True, counters=True)
        D.rollout_vjp(r["tape"], xbt)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ev[0].record(stream)
        D.rollout(model, x0t, None, 1, 1.0, opts=opts, reuse=r["tape"])
        ev[1].record(stream)
        g, _ = D.rollout_vjp(r["tape"], xbt)
        ev[2].record(stream)
        go, _ = D.rollout_vjp_otd(r["tape"], xbt)
        ev2 = torch.cuda.Event(enable_timing=True)
        ev2.record(stream)
        torch.cuda.synchronize()
        go = go.cpu().numpy()
        rel_otd = np.abs(go[:, 7] - g_true[:, 7]) / np.abs(g_true[:, 7])
        assert int(r["status"].abs().sum()) == 0
        gg = g.cpu().numpy()
        xg = r["x"].cpu().numpy()
        rel = np.abs(gg[:, 7] - g_true[:, 7]) / np.abs(g_true[:, 7])
        err_l = float(np.max(np.abs(xg[:, 0] - x_true[:, 0])))
        rows.append((rtol, err_l, float(np.median(rel)), float(rel.max()), ev[0].elapsed_time(ev[1]),
                     ev[1].elapsed_time(ev[2]), int(r["n_acc"].max()), int((r["n_acc"] + r["n_rej"]).max()),
                     float(np.median(rel_otd)), float(rel_otd.max()), ev[2].elapsed_time(ev2)))
    print("\n| rtol | loss error (m, max) | dL/dv_x rel. error (median) | (max) | fwd ms | adj ms | "
          "max accepted | max attempts | OTD error (median) | (max) | OTD adj ms |")
    for row in rows:
        print(f"| {row[0]:.0e} | {row[1]:.2e} | {row[2]:.2e} | {row[3]:.2e} | {row[4]:.3f} | {row[5]:.3f} | "
              f"{row[6]} | {row[7]} | {row[8]:.2e} | {row[9]:.2e} | {row[10]:.3f} |")
    loss = {r[0]: r[1] for r in rows}
    med = {r[0]: r[2] for r in rows}
    assert loss[1e-9] <= 1e-5 and loss[1e-9] <= 1e-3 * loss[1e-3]
    assert med[1e-9] <= 2e-2 and med[1e-9] <= 0.1 * med[1e-5]


def test_friction_gradient_error_follows_tolerance(D, oracle):
    """The same tosses and loss, the gradient with respect to the friction
    coefficient (a model parameter, App. E.2): ground truth from central
    differences of the oracle's adaptive solve at rtol = atol = 1e-12; the
    GPU's discrete-adjoint and continuous-adjoint parameter gradients at
    rtol = atol from 1e-2 to 1e-9.  The error must fall with the tolerance."""
    import copy
    import torch
    desc = toss_model()
    x0 = toss_states()
    xb = np.zeros((N, 13))
    xb[:, 0] = 1.0
    mu = desc["pairs"][0]["mu"]
    vals = []
    for s in (+1, -1):
        d = copy.deepcopy(desc)
        d["pairs"][0]["mu"] = mu + s * 1e-6
        vals.append(oracle.Model(d).rollout_batch(x0, None, 1, 1.0, n_threads=16, rtol=1e-12, atol=1e-12)["x"][:, 0])
    g_true = (vals[0] - vals[1]) / 2e-6
    model = D.Model(desc)
    x0t = torch.tensor(x0, dtype=torch.float64, device="cuda")
    xbt = torch.tensor(xb, dtype=torch.float64, device="cuda")
    rows = []
    for rtol in RTOLS:
        opts = D.default_opts(rtol=rtol, atol=rtol, tape_steps=65536, max_attempts=1000000, tape_stages=1)
        r = D.rollout(model, x0t, None, 1, 1.0, opts=opts, tape=True)
        assert int(r["status"].abs().sum()) == 0
        _, _, pd = D.rollout_vjp_params(r["tape"], xbt)
        _, _, po = D.rollout_vjp_otd_params(r["tape"], xbt)
        scale = np.abs(g_true).max()
        e_d = np.abs(pd.cpu().numpy()[:, 3] - g_true) / scale
        e_o = np.abs(po.cpu().numpy()[:, 3] - g_true) / scale
        rows.append((rtol, float(np.median(e_d)), float(e_d.max()), float(np.median(e_o)), float(e_o.max())))
    print("\n| rtol | dL/dmu error, discrete adjoint (median) | (max) | continuous adjoint (median) | (max) |")
    for row in rows:
        print(f"| {row[0]:.0e} | {row[1]:.2e} | {row[2]:.2e} | {row[3]:.2e} | {row[4]:.2e} |")
    med = {r[0]: r[1] for r in rows}
    last = rows[-1]
    assert med[1e-9] <= 1e-2 * med[1e-3]
    assert last[3] <= 1e-5 and last[2] <= 1e-3 and last[4] <= 1e-3



TOSS_SOLIMP = (0.0, 0.95, 0.001, 0.5, 2.0)
PRIMITIVES = {
    "sphere": lambda: W.model_sphere(radius=0.1, mu=0.8, tc=0.005, solimp=TOSS_SOLIMP),
    "capsule": lambda: W.model_capsule(radius=0.05, half_length=0.1, mu=0.8, tc=0.005, solimp=TOSS_SOLIMP),
}


@pytest.mark.parametrize("prim", sorted(PRIMITIVES))
def test_primitive_toss_gradient_error_follows_tolerance(D, oracle, prim):
    """The object tosses of the other primitives (sphere, capsule; the paper's
    tosses of several primitives, Fig. 13) with the same contact setting,
    throws and loss as the box toss above: the toss distance's gradient with
    respect to v_x against the oracle's at rtol 1e-12, for both adjoints, at
    rtol = atol from 1e-2 to 1e-9."""
    import torch
    desc = PRIMITIVES[prim]()
    x0 = toss_states()
    xb = np.zeros((N, 13))
    xb[:, 0] = 1.0
    ref = oracle.Model(desc).grad_batch(x0, None, 1, 1.0, xb, n_threads=16, rtol=1e-12, atol=1e-12)
    assert (np.asarray(ref["status"]) == 0).all()
    g_true, x_true = ref["x0bar"][:, 7], ref["x"][:, 0]
    model = D.Model(desc)
    x0t = torch.tensor(x0, dtype=torch.float64, device="cuda")
    xbt = torch.tensor(xb, dtype=torch.float64, device="cuda")
    rows = []
    for rtol in RTOLS:
        opts = D.default_opts(rtol=rtol, atol=rtol, tape_steps=65536, max_attempts=1000000, tape_stages=1)
        r = D.rollout(model, x0t, None, 1, 1.0, opts=opts, tape=True)
        assert int(r["status"].abs().sum()) == 0
        g, _ = D.rollout_vjp(r["tape"], xbt)
        go, _ = D.rollout_vjp_otd(r["tape"], xbt)
        e_d = np.abs(g.cpu().numpy()[:, 7] - g_true) / np.abs(g_true)
        e_o = np.abs(go.cpu().numpy()[:, 7] - g_true) / np.abs(g_true)
        err_l = float(np.max(np.abs(r["x"].cpu().numpy()[:, 0] - x_true)))
        rows.append((rtol, err_l, float(np.median(e_d)), float(e_d.max()), float(np.median(e_o)), float(e_o.max())))
    print(f"\n{prim}: | rtol | loss error (m, max) | discrete adjoint (median) | (max) | continuous adjoint (median) "
          f"| (max) |")
    for row in rows:
        print(f"| {row[0]:.0e} | {row[1]:.2e} | {row[2]:.2e} | {row[3]:.2e} | {row[4]:.2e} | {row[5]:.2e} |")
    loss = {r[0]: r[1] for r in rows}
    med = {r[0]: r[2] for r in rows}
    assert loss[1e-9] <= 1e-5 and loss[1e-9] <= 1e-3 * loss[1e-3]
    assert med[1e-9] <= 2e-2 and med[1e-9] <= max(0.1 * med[1e-5], 1e-8)
