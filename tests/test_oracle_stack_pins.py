"""Pins of the oracle's multi-body worlds: box-box contacts and cube stacks.

The paper names primitive-vs-primitive detection (Sec. 2.1, "Collision
detection") but prints no box-box routine; the oracle's reading is the
separating-axis test with face clipping (its header states it).  These pins
fix it by geometry worked out here independently (the overlap polygon of two
squares, two crossing edges), by invariances the contact set must have
(swapping the boxes, moving both rigidly), and by statics (a resting stack
carries the weight above each level).
"""
import numpy as np
import pytest

from paper_2506_14186_amd import workloads as W

G = 9.81
H = 0.1  # cube half size


def qrot(th):
    th = np.asarray(th, float)
    a = np.linalg.norm(th)
    if a == 0:
        return np.array([1.0, 0, 0, 0])
    return np.concatenate([[np.cos(a / 2)], np.sin(a / 2) * th / a])


def qmat(q):
    w, x, y, z = q / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def qmul(a, b):
    w1, x1, y1, z1 = a
    w2, x2, y2, z2 = b
    return np.array([w1 * w2 - x1 * x2 - y1 * y2 - z1 * z2, w1 * x2 + x1 * w2 + y1 * z2 - z1 * y2,
                     w1 * y2 - x1 * z2 + y1 * w2 + z1 * x2, w1 * z2 + x1 * y2 - y1 * x2 + z1 * w2])


def two_boxes(swap=False, mu=0.6, tc=0.003):
    """Two free cubes and one box-box pair (no plane pair): (A, B), or (B, A)
    when swap (then the reported normal points from B to A)."""
    m = W.model_stack(2, mu=mu, tc=tc)
    m["pairs"] = [W._pair(2, 1, mu, tc) if swap else W._pair(1, 2, mu, tc)]
    return m


def pose(c, q):
    return np.concatenate([c, q / np.linalg.norm(q)])


def square_overlap(ca, cb, th):
    """Vertices of the intersection of the axis-aligned square of half size H
    at ca (2-vector) and the square at cb rotated by th about z: corners of
    either square inside the other, and crossings of their edges."""
    def corners(c, t):
        R = np.array([[np.cos(t), -np.sin(t)], [np.sin(t), np.cos(t)]])
        return [c + R @ np.array(s) * H for s in ((1, 1), (-1, 1), (-1, -1), (1, -1))]

    def inside(p, c, t, tol=1e-12):
        R = np.array([[np.cos(t), -np.sin(t)], [np.sin(t), np.cos(t)]])
        d = R.T @ (p - c)
        return np.all(np.abs(d) <= H + tol)

    A, B = corners(ca, 0.0), corners(cb, th)
    pts = [p for p in A if inside(p, cb, th)] + [p for p in B if inside(p, ca, 0.0)]
    for i in range(4):
        p, r = A[i], A[(i + 1) % 4] - A[i]
        for j in range(4):
            q, s = B[j], B[(j + 1) % 4] - B[j]
            den = r[0] * s[1] - r[1] * s[0]
            if abs(den) < 1e-14:
                continue
            t = ((q - p)[0] * s[1] - (q - p)[1] * s[0]) / den
            u = ((q - p)[0] * r[1] - (q - p)[1] * r[0]) / den
            if -1e-12 <= t <= 1 + 1e-12 and -1e-12 <= u <= 1 + 1e-12:
                pts.append(p + t * r)
    out = []
    for p in pts:  # unique
        if not any(np.linalg.norm(p - o) < 1e-9 for o in out):
            out.append(p)
    return np.array(out)


def same_point_sets(a, b, tol):
    assert len(a) == len(b), (len(a), len(b))
    used = np.zeros(len(b), bool)
    for p in a:
        d = np.linalg.norm(b - p, axis=1) + used * 1e9
        j = int(np.argmin(d))
        assert d[j] <= tol, (p, b)
        used[j] = True


@pytest.mark.parametrize("off,th", [((0.03, -0.02), 0.0), ((0.0, 0.0), 0.0), ((0.05, 0.04), 0.3),
                                    ((0.0, 0.0), np.pi / 4), ((-0.06, 0.01), 1.1)])
def test_face_contacts_are_the_overlap_polygon(oracle, off, th):
    """Cube B resting on cube A, face to face, penetrating by delta, shifted
    laterally and turned about the vertical: the contacts are the corners of
    the overlap polygon of the two squares, all at r = -delta, halfway between
    the faces, normal +z."""
    m = oracle.Model(two_boxes())
    delta = 1.5e-3
    qa = pose([0.0, 0.0, 0.0], qrot([0, 0, 0]))
    cb = np.array([off[0], off[1], 2 * H - delta])
    qb = pose(cb, qrot([0, 0, th]))
    c = m.contacts(np.concatenate([qa, qb]))
    poly = square_overlap(np.zeros(2), cb[:2], th)
    assert 4 <= len(c) <= 8
    np.testing.assert_allclose(c[:, 0], -delta, atol=1e-15)
    np.testing.assert_allclose(c[:, 3], H - delta / 2, atol=1e-15)
    np.testing.assert_allclose(c[:, 4:7], [[0, 0, 1]] * len(c), atol=1e-15)
    same_point_sets(c[:, 1:3], poly, 1e-12)


def test_crossing_edges_give_one_contact(oracle):
    """A turned 45 deg about y (its top is an edge along y), B turned 45 deg
    about x (its bottom is an edge along x), B above A so that the edges cross
    with overlap delta: one contact, normal +z, r = -delta, at the midpoint of
    the crossing (x of A's edge, y of B's edge)."""
    m = oracle.Model(two_boxes())
    delta = 2e-3
    e = H * np.sqrt(2.0)
    ca = np.array([0.01, -0.02, 0.3])
    cb = np.array([-0.03, 0.04, ca[2] + 2 * e - delta])
    q = np.concatenate([pose(ca, qrot([0, np.pi / 4, 0])), pose(cb, qrot([np.pi / 4, 0, 0]))])
    c = m.contacts(q)
    assert len(c) == 1
    np.testing.assert_allclose(c[0, 0], -delta, atol=1e-14)
    np.testing.assert_allclose(c[0, 1:4], [ca[0], cb[1], ca[2] + e - delta / 2], atol=1e-14)
    np.testing.assert_allclose(c[0, 4:7], [0, 0, 1], atol=1e-14)


def _generic_pose(rng):
    """B above a tilted A, slightly tilted itself and penetrating (a unique
    least-overlap face axis)."""
    qa = pose([0.0, 0.0, 0.0], qrot(rng.normal(0, 0.01, 3)))
    qb = pose([rng.normal(0, 0.03), rng.normal(0, 0.03), 2 * H - 0.004], qrot(rng.normal(0, 0.01, 3)))
    return np.concatenate([qa, qb])


def test_swapping_the_boxes_flips_the_normal(oracle):
    rng = np.random.default_rng(5)
    ma, mb = oracle.Model(two_boxes()), oracle.Model(two_boxes(swap=True))
    for _ in range(6):
        q = _generic_pose(rng)
        ca, cb = ma.contacts(q), mb.contacts(q)
        assert len(ca) >= 3 and len(ca) == len(cb)
        same_point_sets(np.c_[ca[:, 0:4], ca[:, 4:7]], np.c_[cb[:, 0:4], -cb[:, 4:7]], 1e-13)


def test_rigid_motion_equivariance(oracle):
    """Moving both boxes by one rotation Q and translation t: r unchanged,
    points Q p + t, normals Q n (the contact set is a property of the pair)."""
    rng = np.random.default_rng(9)
    m = oracle.Model(two_boxes())
    for _ in range(6):
        q = _generic_pose(rng)
        qm = qrot(rng.normal(0, 1.0, 3))
        Q, t = qmat(qm), rng.normal(0, 1.0, 3)
        q2 = q.copy()
        for b in range(2):
            q2[7 * b:7 * b + 3] = Q @ q[7 * b:7 * b + 3] + t
            q2[7 * b + 3:7 * b + 7] = qmul(qm, q[7 * b + 3:7 * b + 7])
        c1, c2 = m.contacts(q), m.contacts(q2)
        assert len(c1) == len(c2) >= 3
        moved = np.c_[c1[:, 0], c1[:, 1:4] @ Q.T + t, c1[:, 4:7] @ Q.T]
        same_point_sets(moved, c2[:, 0:7], 1e-12)


def test_separated_boxes_touch_only_in_the_cfd_field(oracle):
    """A gap g below the CFD width w_c = 1 cm: no contact for F, and the
    contacts-from-distance field sees the four corners at r = +g."""
    m = oracle.Model(two_boxes())
    g = 4e-3
    q = np.concatenate([pose([0, 0, 0], qrot([0, 0, 0])), pose([0.02, 0.01, 2 * H + g], qrot([0, 0, 0]))])
    assert len(m.contacts(q)) == 0
    c = m.contacts(q, cfd=True)
    assert len(c) == 4
    np.testing.assert_allclose(c[:, 0], g, atol=1e-15)
    q[9] = 2 * H + 0.011  # beyond w_c
    assert len(m.contacts(q, cfd=True)) == 0


def test_resting_stack_carries_the_weight_above(oracle):
    """Three cubes (1 kg) settled on the plane: the normal contact forces sum
    to 3 m g at the plane, 2 m g between cubes 1 and 2 and m g between cubes
    2 and 3 (statics of the resting stack), and every acceleration vanishes."""
    k = 3
    desc = W.model_stack(k, tc=0.003)
    m = oracle.Model(desc)
    x0 = W.stack_state([[0.01, -0.005], [-0.004, 0.008], [0.006, 0.002]])
    r = m.rollout(x0, None, 1, 1.5)
    assert r["status"] == 0
    x = r["x"]
    xd, info = m.rhs(x)
    assert np.abs(xd[6 * k:]).max() < 1e-6 * G
    f = info["forces"].reshape(-1, 4).sum(axis=1)  # per contact: normal part of its 4 edge forces
    c = m.contacts(x[:7 * k])
    act = c[c[:, 0] < 0]
    z = act[:, 3]
    levels = {0.0: 3 * G, 2 * H: 2 * G, 4 * H: G}
    for zl, w in levels.items():
        sel = np.abs(z - zl) < 0.01
        assert sel.sum() >= 4
        np.testing.assert_allclose(f[sel].sum(), w, rtol=1e-6)


def test_contact_capacity_and_overflow_flag(oracle):
    """More than 256 contacts within reach (six coincident cubes give 15
    pairs of 8 corners, plus two big stacks of them): the first 256 in pair
    order make rows and the status flags the overflow, without ending the
    world."""
    k = 40
    desc = W.model_stack(k)
    m = oracle.Model(desc)
    q = np.zeros(7 * k)
    for i in range(k):
        q[7 * i:7 * i + 3] = [0.0, 0.0, 1.0 + 1e-3 * (i % 2)]
        q[7 * i + 3:7 * i + 7] = qrot([0, 0, 0.01 * i])
    x = np.concatenate([q, np.zeros(6 * k)])
    xd, info = m.rhs(x)
    assert info["status"] & oracle.STATUS_BITS["CONTACT_OVERFLOW"]
    assert info["n_rows"] == 4 * 256
    r = m.rollout(x, None, 1, 1e-3)
    assert r["status"] == oracle.STATUS_BITS["CONTACT_OVERFLOW"]


def test_box_box_tangent_matches_fd(oracle):
    """The derivative of F through the box-box contact geometry (face
    clipping; combinatorics held fixed) against central differences."""
    rng = np.random.default_rng(17)
    m = oracle.Model(W.model_stack(2, tc=0.003))
    q = np.concatenate([pose([0, 0, H - 2e-4], qrot(rng.normal(0, 0.02, 3))),
                        pose([0.03, -0.02, 3 * H - 1e-3], qrot(rng.normal(0, 0.04, 3)))])
    x = np.concatenate([q, rng.normal(0, 0.05, 12)])
    dirs = rng.normal(size=(3, m.nx))
    xd, jv = m.rhs_jvp(x, None, dirs)
    eps = 1e-7
    for d in range(3):
        fp, _ = m.rhs(x + eps * dirs[d])
        fm, _ = m.rhs(x - eps * dirs[d])
        fd = (fp - fm) / (2 * eps)
        np.testing.assert_allclose(jv[d], fd, rtol=1e-5, atol=1e-6 * np.abs(fd).max())
