"""Seeded synthetic workloads: declarative model descriptions and initial data.

This module is the only code shared by the HIP path and the oracle.  It holds
no arithmetic of the method: models are plain dictionaries (geometry, masses,
contact parameters, joint layout), and inputs are draws from
``numpy.random.default_rng(seed)``.  Each consumer turns a description into its
own internal form (inertia tensors, pair tables, invweights ... are computed by
each side independently).

Model dictionary layout
-----------------------
``bodies``  list, parents before children (``parent`` = -1 is the world):
    ``pos``/``quat``  frame relative to the parent frame (quat is w,x,y,z),
    ``inertial``      solid primitive ``{"type", "size", "mass"}`` whose uniform
                      density body gives the mass/inertia about the body origin,
    ``joints``        list of ``{"type": "free"|"hinge"|"slide", "axis", "pos"}``
                      (axis and anchor in the body frame, applied in order).
``geoms``   ``{"body", "type": "plane"|"sphere"|"capsule"|"box", "size", "pos",
            "quat"}``; sizes are MuJoCo-style: sphere (r), capsule (r, half
            length along local z), box (half sizes), plane (unused; normal is
            the local z axis).
``pairs``   ``{"g1", "g2", "mu", "solref": (t_c, damp ratio),
            "solimp": (d0, dw, width, midpoint, power),
            "cfd": (d_c, d_0, w_c, m_c, p_c)}``; the contact normal points from
            g1 to g2.
``ctrl``    ``{"dofs": [...]}``: control i is a generalized force on dof i.
``gravity`` 3-vector.

The workloads follow the soft-contact test problems of the paper (cube and
sphere tosses onto a plane, Sec. 3 and App. E.1; a legged chain and cube stacks
as the multi-contact cases), at the sizes used for measurement.
"""
from __future__ import annotations

import numpy as np

GRAVITY = [0.0, 0.0, -9.81]
# Impedance of the paper's cube and primitive tosses (App. E.1): d(0) = 0, so
# the contact force is continuous when a contact activates at r = 0.
SOLIMP_DEFAULT = [0.0, 0.95, 0.001, 0.5, 2.0]


def _cfd_default(solimp):
    # Contacts-from-distance continuation (d_c, d_0, w_c, m_c, p_c), Sec. 4:
    # from d_0 at r = 0 down to d_c = 0 at r = w_c = 1 cm; d_0 continues the
    # contact impedance d(0) when that is at least 0.01.
    return [0.0, max(float(solimp[0]), 0.01), 0.01, 1.0, 4.0]


def _pair(g1, g2, mu, tc, solimp=None, dampratio=1.0, cfd=None):
    si = list(SOLIMP_DEFAULT if solimp is None else solimp)
    if len(si) == 3:
        si = si + [0.5, 2.0]
    return {"g1": g1, "g2": g2, "mu": float(mu), "solref": [float(tc), float(dampratio)],
            "solimp": [float(s) for s in si],
            "cfd": [float(c) for c in (cfd if cfd is not None else _cfd_default(si))]}


def _plane():
    return {"body": -1, "type": "plane", "size": [0.0, 0.0, 0.0], "pos": [0.0, 0.0, 0.0],
            "quat": [1.0, 0.0, 0.0, 0.0]}


# --------------------------------------------------------------------------
# models
# --------------------------------------------------------------------------

def model_sphere(radius=0.1, mass=1.0, mu=1.0, tc=0.002, solimp=(0.9, 0.95, 0.001),
                 dampratio=1.0, cfd=None):
    """Single free sphere above a plane (sphere toss / ball drop)."""
    return {
        "name": "sphere",
        "gravity": list(GRAVITY),
        "bodies": [{"parent": -1, "pos": [0.0, 0.0, 0.0], "quat": [1.0, 0.0, 0.0, 0.0],
                    "inertial": {"type": "sphere", "size": [radius, 0.0, 0.0], "mass": mass},
                    "joints": [{"type": "free", "axis": [0.0, 0.0, 1.0], "pos": [0.0, 0.0, 0.0]}]}],
        "geoms": [_plane(),
                  {"body": 0, "type": "sphere", "size": [radius, 0.0, 0.0], "pos": [0.0, 0.0, 0.0],
                   "quat": [1.0, 0.0, 0.0, 0.0]}],
        "pairs": [_pair(0, 1, mu, tc, solimp, dampratio, cfd)],
        "ctrl": {"dofs": []},
    }


def model_capsule(radius=0.05, half_length=0.1, mass=1.0, mu=0.8, tc=0.005, solimp=None):
    """Single free capsule (axis along its body z) above a plane (capsule toss)."""
    return {
        "name": "capsule",
        "gravity": list(GRAVITY),
        "bodies": [{"parent": -1, "pos": [0.0, 0.0, 0.0], "quat": [1.0, 0.0, 0.0, 0.0],
                    "inertial": {"type": "capsule", "size": [radius, half_length, 0.0], "mass": mass},
                    "joints": [{"type": "free", "axis": [0.0, 0.0, 1.0], "pos": [0.0, 0.0, 0.0]}]}],
        "geoms": [_plane(),
                  {"body": 0, "type": "capsule", "size": [radius, half_length, 0.0], "pos": [0.0, 0.0, 0.0],
                   "quat": [1.0, 0.0, 0.0, 0.0]}],
        "pairs": [_pair(0, 1, mu, tc, solimp)],
        "ctrl": {"dofs": []},
    }


def model_cube_corners(half=0.1, mass=1.0, corner_radius=0.01, mu=0.8, tc=0.001, solimp=None,
                       ctrl=False):
    """Free cube whose contacts are 8 corner spheres against a plane."""
    geoms = [_plane()]
    pairs = []
    for k in range(8):
        sx = half if (k & 1) else -half
        sy = half if (k & 2) else -half
        sz = half if (k & 4) else -half
        geoms.append({"body": 0, "type": "sphere", "size": [corner_radius, 0.0, 0.0],
                      "pos": [sx, sy, sz], "quat": [1.0, 0.0, 0.0, 0.0]})
        pairs.append(_pair(0, len(geoms) - 1, mu, tc, solimp))
    return {
        "name": "cube_corners",
        "gravity": list(GRAVITY),
        "bodies": [{"parent": -1, "pos": [0.0, 0.0, 0.0], "quat": [1.0, 0.0, 0.0, 0.0],
                    "inertial": {"type": "box", "size": [half, half, half], "mass": mass},
                    "joints": [{"type": "free", "axis": [0.0, 0.0, 1.0], "pos": [0.0, 0.0, 0.0]}]}],
        "geoms": geoms,
        "pairs": pairs,
        "ctrl": {"dofs": [0, 1, 2, 3, 4, 5] if ctrl else []},
    }


def model_box(half=0.1, mass=1.0, mu=0.8, tc=0.001, solimp=None, ctrl=False):
    """Free cube (one stack level) whose contacts come from a box geom against
    the plane (the smoothed plane-box detection: four deepest vertices)."""
    return {
        "name": "box",
        "gravity": list(GRAVITY),
        "bodies": [{"parent": -1, "pos": [0.0, 0.0, 0.0], "quat": [1.0, 0.0, 0.0, 0.0],
                    "inertial": {"type": "box", "size": [half, half, half], "mass": mass},
                    "joints": [{"type": "free", "axis": [0.0, 0.0, 1.0], "pos": [0.0, 0.0, 0.0]}]}],
        "geoms": [_plane(), {"body": 0, "type": "box", "size": [half, half, half], "pos": [0.0, 0.0, 0.0],
                             "quat": [1.0, 0.0, 0.0, 0.0]}],
        "pairs": [_pair(0, 1, mu, tc, solimp)],
        "ctrl": {"dofs": [0, 1, 2, 3, 4, 5] if ctrl else []},
    }


def model_stack(k, half=0.1, mass=1.0, mu=0.6, tc=0.003, solimp=None, ctrl=False):
    """Stack of k free cubes (edge 2 half, mass each) with box geoms: pairs are
    every cube against the plane (cube order), then every cube pair (i, j),
    i < j, in lexicographic order.  With ctrl, the 6 generalized forces act on
    the top cube's free joint."""
    bodies, geoms, pairs = [], [_plane()], []
    for i in range(k):
        bodies.append({"parent": -1, "pos": [0.0, 0.0, 0.0], "quat": [1.0, 0.0, 0.0, 0.0],
                       "inertial": {"type": "box", "size": [half, half, half], "mass": mass},
                       "joints": [{"type": "free", "axis": [0.0, 0.0, 1.0], "pos": [0.0, 0.0, 0.0]}]})
        geoms.append({"body": i, "type": "box", "size": [half, half, half], "pos": [0.0, 0.0, 0.0],
                      "quat": [1.0, 0.0, 0.0, 0.0]})
    for i in range(k):
        pairs.append(_pair(0, 1 + i, mu, tc, solimp))
    for i in range(k):
        for j in range(i + 1, k):
            pairs.append(_pair(1 + i, 1 + j, mu, tc, solimp))
    return {"name": f"stack{k}", "gravity": list(GRAVITY), "bodies": bodies, "geoms": geoms, "pairs": pairs,
            "ctrl": {"dofs": [6 * (k - 1) + d for d in range(6)] if ctrl else []}}


def stack_state(offsets, half=0.1, gap=0.001):
    """Initial state of a stack: cube i centred at (offsets[i], (i + 1/2) edge +
    (i + 1) gap), identity orientation, at rest."""
    k = len(offsets)
    x = np.zeros(13 * k)
    for i in range(k):
        x[7 * i + 0:7 * i + 2] = offsets[i]
        x[7 * i + 2] = half + gap + i * (2.0 * half + gap)
        x[7 * i + 3] = 1.0
    return x


def cube_stacks(seed=4, n_worlds=1024, kmax=32, horizon=1.0, mu=0.6, tc_range=(0.001, 0.005)):
    """Uneven batch of cube stacks: k ~ U{1..kmax} cubes per world, each cube
    offset laterally by N(0, 0.02^2) per axis (independently, not cumulative),
    1 mm gaps, at rest, identity orientation; per-world contact time constant
    t_c ~ U(tc_range); mu as given.  Returns per-world model descriptions and
    states (ragged: 13 k doubles each)."""
    rng = np.random.default_rng(seed)
    ks = rng.integers(1, kmax + 1, size=n_worlds)
    tcs = rng.uniform(tc_range[0], tc_range[1], size=n_worlds)
    models, x0 = [], []
    for w in range(n_worlds):
        k = int(ks[w])
        off = rng.normal(0.0, 0.02, size=(k, 2))
        models.append(model_stack(k, mu=mu, tc=float(tcs[w])))
        x0.append(stack_state(off))
    return {"models": models, "x0": x0, "k": ks, "tc": tcs, "n_intervals": 1, "interval_dt": float(horizon)}


def model_chain(link_half=0.125, radius=0.03, mu=1.0, tc=0.002, solimp=None):
    """Planar legged chain: a horizontal torso capsule with a planar root
    (slide x, slide z, hinge y) and two legs (thigh + shin capsules, hinge y at
    hips and knees).  The shins are the feet that touch the plane."""
    cap = {"type": "capsule", "size": [radius, link_half, 0.0], "mass": None}
    hy = [0.0, 1.0, 0.0]
    ry90 = [float(np.cos(np.pi / 4)), 0.0, float(np.sin(np.pi / 4)), 0.0]  # local z -> world x
    bodies = [
        {"parent": -1, "pos": [0.0, 0.0, 0.0], "quat": [1.0, 0.0, 0.0, 0.0],
         "inertial": {"type": "capsule", "size": [radius, link_half, 0.0], "mass": None,
                      "quat": ry90},
         "joints": [{"type": "slide", "axis": [1.0, 0.0, 0.0], "pos": [0.0, 0.0, 0.0]},
                    {"type": "slide", "axis": [0.0, 0.0, 1.0], "pos": [0.0, 0.0, 0.0]},
                    {"type": "hinge", "axis": hy, "pos": [0.0, 0.0, 0.0]}]},
    ]
    geoms = [_plane(),
             {"body": 0, "type": "capsule", "size": [radius, link_half, 0.0], "pos": [0.0, 0.0, 0.0],
              "quat": ry90}]
    pairs = []
    for side in (-1.0, 1.0):
        thigh = len(bodies)
        bodies.append({"parent": 0, "pos": [side * link_half, 0.0, -link_half],
                       "quat": [1.0, 0.0, 0.0, 0.0], "inertial": dict(cap),
                       "joints": [{"type": "hinge", "axis": hy, "pos": [0.0, 0.0, link_half]}]})
        geoms.append({"body": thigh, "type": "capsule", "size": [radius, link_half, 0.0],
                      "pos": [0.0, 0.0, 0.0], "quat": [1.0, 0.0, 0.0, 0.0]})
        shin = len(bodies)
        bodies.append({"parent": thigh, "pos": [0.0, 0.0, -2 * link_half],
                       "quat": [1.0, 0.0, 0.0, 0.0], "inertial": dict(cap),
                       "joints": [{"type": "hinge", "axis": hy, "pos": [0.0, 0.0, link_half]}]})
        geoms.append({"body": shin, "type": "capsule", "size": [radius, link_half, 0.0],
                      "pos": [0.0, 0.0, 0.0], "quat": [1.0, 0.0, 0.0, 0.0]})
        pairs.append(_pair(0, len(geoms) - 1, mu, tc, solimp))
    return {
        "name": "chain",
        "gravity": list(GRAVITY),
        "bodies": bodies,
        "geoms": geoms,
        "pairs": pairs,
        "ctrl": {"dofs": [3, 4, 5, 6]},
    }


def model_pendulum(n_links=2, half=0.1, radius=0.02):
    """Hinge chain hanging from the world without contacts (dynamics pins)."""
    bodies = []
    geoms = [_plane()]
    for i in range(n_links):
        bodies.append({"parent": i - 1, "pos": [0.0, 0.0, 1.0] if i == 0 else [0.0, 0.0, -2 * half],
                       "quat": [1.0, 0.0, 0.0, 0.0],
                       "inertial": {"type": "capsule", "size": [radius, half, 0.0], "mass": None},
                       "joints": [{"type": "hinge", "axis": [0.0, 1.0, 0.0] if i % 2 == 0 else [1.0, 0.0, 0.0],
                                   "pos": [0.0, 0.0, half]},
                                  {"type": "slide", "axis": [0.0, 0.0, 1.0], "pos": [0.0, 0.0, 0.0]}]
                       if i == n_links - 1 else
                       [{"type": "hinge", "axis": [0.0, 1.0, 0.0] if i % 2 == 0 else [1.0, 0.0, 0.0],
                         "pos": [0.0, 0.0, half]}]})
        geoms.append({"body": i, "type": "capsule", "size": [radius, half, 0.0], "pos": [0.0, 0.0, 0.0],
                      "quat": [1.0, 0.0, 0.0, 0.0]})
    return {"name": "pendulum", "gravity": list(GRAVITY), "bodies": bodies, "geoms": geoms,
            "pairs": [], "ctrl": {"dofs": list(range(n_links + 1))}}


def model_free_box(half=(0.1, 0.15, 0.2), mass=2.0):
    """A free asymmetric box with no contacts (torque-free rigid-body pins)."""
    return {"name": "free_box", "gravity": list(GRAVITY),
            "bodies": [{"parent": -1, "pos": [0.0, 0.0, 0.0], "quat": [1.0, 0.0, 0.0, 0.0],
                        "inertial": {"type": "box", "size": list(half), "mass": mass},
                        "joints": [{"type": "free", "axis": [0.0, 0.0, 1.0], "pos": [0.0, 0.0, 0.0]}]}],
            "geoms": [_plane()], "pairs": [], "ctrl": {"dofs": []}}


# --------------------------------------------------------------------------
# state helpers (layout only)
# --------------------------------------------------------------------------

def nq_nv(model):
    nq = nv = 0
    for b in model["bodies"]:
        for j in b["joints"]:
            if j["type"] == "free":
                nq += 7
                nv += 6
            else:
                nq += 1
                nv += 1
    return nq, nv


def uniform_quat(rng, n):
    """Uniformly distributed unit quaternions (Shoemake's subgroup algorithm), w first."""
    u1, u2, u3 = rng.random(n), rng.random(n), rng.random(n)
    a, b = np.sqrt(1.0 - u1), np.sqrt(u1)
    x = a * np.sin(2 * np.pi * u2)
    y = a * np.cos(2 * np.pi * u2)
    z = b * np.sin(2 * np.pi * u3)
    w = b * np.cos(2 * np.pi * u3)
    return np.stack([w, x, y, z], axis=1)


# --------------------------------------------------------------------------
# configurations
# --------------------------------------------------------------------------

def sphere_drop(seed=1, n_worlds=1, horizon=1.0):
    """Sphere (r 0.1 m, 1 kg) dropped from 0.5 m, v_lin ~ N(0, 0.5) m/s."""
    rng = np.random.default_rng(seed)
    m = model_sphere()
    x0 = np.zeros((n_worlds, 13))
    x0[:, 2] = 0.5
    x0[:, 3] = 1.0
    x0[:, 7:10] = rng.normal(0.0, 0.5, size=(n_worlds, 3))
    return {"model": m, "x0": x0, "u": np.zeros((n_worlds, 1, 0)), "n_intervals": 1,
            "interval_dt": float(horizon)}


def cube_toss(seed=2, n_worlds=4096, horizon=0.5):
    """Cube (edge 0.2 m, 1 kg) with 8 corner spheres, stiff contact t_c 1 ms,
    random orientation, height U(0.2, 0.6) m, linear/angular velocity N(0, 1)."""
    rng = np.random.default_rng(seed)
    m = model_cube_corners()
    x0 = np.zeros((n_worlds, 13))
    x0[:, 2] = rng.uniform(0.2, 0.6, size=n_worlds)
    x0[:, 3:7] = uniform_quat(rng, n_worlds)
    x0[:, 7:13] = rng.normal(0.0, 1.0, size=(n_worlds, 6))
    return {"model": m, "x0": x0, "u": np.zeros((n_worlds, 1, 0)), "n_intervals": 1,
            "interval_dt": float(horizon)}


def box_toss(seed=4, n_worlds=1024, horizon=1.0, mu=0.6, tc=0.003):
    """Single free cubes (edge 0.2 m, 1 kg) with a box geom on a plane: the
    one-level stacks of the stack workload; random orientation, height U(0.2,
    0.6) m, velocity N(0, 1)."""
    rng = np.random.default_rng(seed)
    m = model_box(mu=mu, tc=tc)
    x0 = np.zeros((n_worlds, 13))
    x0[:, 2] = rng.uniform(0.2, 0.6, size=n_worlds)
    x0[:, 3:7] = uniform_quat(rng, n_worlds)
    x0[:, 7:13] = rng.normal(0.0, 1.0, size=(n_worlds, 6))
    return {"model": m, "x0": x0, "u": np.zeros((n_worlds, 1, 0)), "n_intervals": 1,
            "interval_dt": float(horizon)}


def chain_walk(seed=3, n_worlds=16384, n_intervals=200, interval_dt=0.01):
    """Planar legged chain, torso at 0.55 m, legs vertical, at rest; hinge torques
    piecewise constant U(-1, 1) N m over ``n_intervals`` of ``interval_dt``."""
    rng = np.random.default_rng(seed)
    m = model_chain()
    x0 = np.zeros((n_worlds, 14))
    x0[:, 1] = 0.55  # slide-z of the root
    u = rng.uniform(-1.0, 1.0, size=(n_worlds, n_intervals, 4))
    return {"model": m, "x0": x0, "u": u, "n_intervals": n_intervals, "interval_dt": float(interval_dt)}


CONFIGS = {
    "sphere_drop": sphere_drop,
    "cube_toss": cube_toss,
    "chain_walk": chain_walk,
    "box_toss": box_toss,
    "cube_stacks": cube_stacks,
}
