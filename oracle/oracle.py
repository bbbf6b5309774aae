"""ctypes wrapper of the oracle simulator (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` use this module.  It converts a declarative model description
(see ``paper_2506_14186_amd.workloads``) into the oracle's own model struct and
calls the plain FP64 simulator in ``orc_sim.cpp``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SOURCES = ["orc_sim.cpp"]
_HEADERS = ["orc_api.h", "orc_math.hpp"]

JOINT = {"free": 0, "hinge": 1, "slide": 2}
GEOM = {"plane": 0, "sphere": 1, "capsule": 2, "box": 3}

STATUS_BITS = {"MAX_STEPS": 1, "DT_UNDERFLOW": 2, "NONFINITE": 4, "SOLVER_MAXIT": 8, "CONTACT_OVERFLOW": 16}


def build(force=True):
    """Compile the oracle with g++ (FP64, no fast-math, no FMA contraction)."""
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-pthread", "-ffp-contract=off",
           "-fno-fast-math", "-o", LIB_PATH] + [os.path.join(_HERE, s) for s in _SOURCES]
    subprocess.check_call(cmd)
    return LIB_PATH


def dense_weights(theta):
    """Weights of the stage slopes in the Dormand-Prince continuous extension."""
    w = np.zeros(7)
    lib().orc_dense_weights(float(theta), _p(w))
    return w


def flop_cholesky(A):
    """Counted operations of the oracle's Cholesky factorization and solve of A."""
    A = np.ascontiguousarray(np.asarray(A, np.float64))
    return int(lib().orc_flop_cholesky(_p(A), A.shape[0]))


class _ModelDef(C.Structure):
    _fields_ = [("nb", C.c_int), ("nj", C.c_int), ("ng", C.c_int), ("npair", C.c_int), ("nu", C.c_int)] + [
        (n, C.c_void_p) for n in (
            "body_parent", "body_pos", "body_quat", "body_iner_type", "body_iner_size", "body_iner_quat",
            "body_mass", "jnt_body", "jnt_type", "jnt_axis", "jnt_pos", "geom_body", "geom_type", "geom_size",
            "geom_pos", "geom_quat", "pair_g1", "pair_g2", "pair_mu", "pair_solref", "pair_solimp", "pair_cfd",
            "ctrl_dof")] + [("gravity", C.c_double * 3)]


class _Opts(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("rtol", "atol", "h0", "safety", "facmin", "facmax", "kP", "kI",
                                           "err_order", "err_floor")] + [
        ("max_attempts", C.c_longlong), ("newton_maxit", C.c_int), ("cfd", C.c_int), ("softplus_beta", C.c_double),
        ("h_levels", C.c_int), ("tableau", C.c_int)]


DEFAULT_OPTS = dict(rtol=1e-6, atol=1e-8, h0=1e-3, safety=0.9, facmin=0.2, facmax=10.0, kP=0.2, kI=0.4,
                    err_order=5.0, err_floor=1e-6, max_attempts=1_000_000, newton_maxit=100, cfd=0,
                    softplus_beta=1e4, h_levels=0, tableau=0)

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.orc_model_new.restype = P
        L.orc_model_new.argtypes = [C.POINTER(_ModelDef)]
        L.orc_model_free.argtypes = [P]
        L.orc_model_sizes.argtypes = [P, P]
        L.orc_model_inertia.argtypes = [P, P, P, P]
        L.orc_kinematics.argtypes = [P, P, P, P, P, P, P, P]
        L.orc_contacts.argtypes = [P, P, P]
        L.orc_contacts_cfd.argtypes = [P, P, C.c_int, P]
        L.orc_point_jac.argtypes = [P, P, C.c_int, P, P]
        L.orc_rhs.argtypes = [P, P, P, C.c_int, P, P, P]
        L.orc_rows.argtypes = [P, P, P, C.c_int, C.c_double, P, P, P, P, P]
        L.orc_rhs_jvp.argtypes = [P, P, P, C.c_int, C.c_double, C.c_int, P, P, P, P]
        L.orc_rollout.argtypes = [P, P, P, C.c_int, C.c_double, C.POINTER(_Opts), P, C.c_int, P, P,
                                  C.c_int, P, C.c_int, P]
        L.orc_rollout_jvp.argtypes = [P, P, P, C.c_int, C.c_double, C.POINTER(_Opts), C.c_int, P, P, P, P, P]
        L.orc_rollout_batch.argtypes = [P, C.c_int, P, P, C.c_int, C.c_double, C.POINTER(_Opts), P, P, C.c_int]
        L.orc_grad_batch.argtypes = [P, C.c_int, P, P, C.c_int, C.c_double, C.POINTER(_Opts), P, P, P, P, P,
                                     C.c_int]
        L.orc_grad_forced_batch.argtypes = [P, C.c_int, P, P, C.c_int, C.c_double, C.POINTER(_Opts), P, P, C.c_int,
                                            P, P, P, P, P, C.c_int]
        L.orc_rollout_jvp_forced.argtypes = [P, P, P, C.c_int, C.c_double, C.POINTER(_Opts), P, C.c_int, C.c_int,
                                             P, P, P, P]
        L.orc_attempt.argtypes = [P, P, P, C.c_double, C.POINTER(_Opts), P, P]
        L.orc_flop_count.argtypes = [P, P, P, C.c_int, C.c_double, C.POINTER(_Opts), P]
        L.orc_flop_cholesky.argtypes = [P, C.c_int]
        L.orc_otd_grad_batch.argtypes = [P, C.c_int, P, P, C.c_int, C.c_double, C.POINTER(_Opts), P, P, P, P, P,
                                         C.c_int]
        L.orc_dense_weights.argtypes = [C.c_double, P]
        L.orc_dense_states.argtypes = [P, P, P, C.c_int, C.c_double, C.POINTER(_Opts), P, C.c_int, C.c_int, P, P]
        L.orc_flop_cholesky.restype = C.c_longlong
        L.orc_next_step.argtypes = [C.POINTER(_Opts), C.c_double, C.c_double, C.c_double, C.c_int, P]
        L.orc_next_step.restype = C.c_double
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data if a is not None and a.size else None


def _f64(x, n=None):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float64).ravel())
    return a


def _i32(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.int32).ravel())


def make_opts(**kw):
    d = dict(DEFAULT_OPTS)
    d.update(kw)
    o = _Opts()
    for k, v in d.items():
        setattr(o, k, v)
    return o


class Model:
    """The oracle's model, built from a workload dictionary."""

    def __init__(self, desc):
        self.desc = desc
        bodies, geoms, pairs = desc["bodies"], desc["geoms"], desc["pairs"]
        self._keep = []
        jb, jt, ja, jp = [], [], [], []
        for bi, b in enumerate(bodies):
            for j in b["joints"]:
                jb.append(bi)
                jt.append(JOINT[j["type"]])
                ja.append(j["axis"])
                jp.append(j["pos"])
        itype = [GEOM[b["inertial"]["type"]] for b in bodies]
        isize = [list(b["inertial"]["size"]) + [0.0] * (3 - len(b["inertial"]["size"])) for b in bodies]
        iquat = [b["inertial"].get("quat", [1.0, 0.0, 0.0, 0.0]) for b in bodies]
        imass = [b["inertial"]["mass"] if b["inertial"]["mass"] is not None else -1.0 for b in bodies]
        arrs = dict(
            body_parent=_i32([b["parent"] for b in bodies]), body_pos=_f64([b["pos"] for b in bodies]),
            body_quat=_f64([b["quat"] for b in bodies]), body_iner_type=_i32(itype), body_iner_size=_f64(isize),
            body_iner_quat=_f64(iquat), body_mass=_f64(imass), jnt_body=_i32(jb), jnt_type=_i32(jt),
            jnt_axis=_f64(ja), jnt_pos=_f64(jp), geom_body=_i32([g["body"] for g in geoms]),
            geom_type=_i32([GEOM[g["type"]] for g in geoms]),
            geom_size=_f64([list(g["size"]) + [0.0] * (3 - len(g["size"])) for g in geoms]),
            geom_pos=_f64([g["pos"] for g in geoms]), geom_quat=_f64([g["quat"] for g in geoms]),
            pair_g1=_i32([p["g1"] for p in pairs]), pair_g2=_i32([p["g2"] for p in pairs]),
            pair_mu=_f64([p["mu"] for p in pairs]), pair_solref=_f64([p["solref"] for p in pairs]),
            pair_solimp=_f64([p["solimp"] for p in pairs]), pair_cfd=_f64([p["cfd"] for p in pairs]),
            ctrl_dof=_i32(desc["ctrl"]["dofs"]))
        d = _ModelDef()
        d.nb, d.nj, d.ng, d.npair, d.nu = len(bodies), len(jb), len(geoms), len(pairs), len(desc["ctrl"]["dofs"])
        for k, a in arrs.items():
            setattr(d, k, _p(a))
        for i in range(3):
            d.gravity[i] = desc["gravity"][i]
        self._keep = arrs
        self._def = d
        self.h = lib().orc_model_new(C.byref(d))
        sz = np.zeros(4, np.int32)
        lib().orc_model_sizes(self.h, _p(sz))
        self.nq, self.nv, self.nu, self.ncmax = (int(s) for s in sz)
        self.nx = self.nq + self.nv
        self.nb = len(bodies)

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().orc_model_free(self.h)
        except Exception:
            pass

    # -------------------------------------------------------------- pieces
    def inertia(self):
        m, I, w = np.zeros(self.nb), np.zeros((self.nb, 3, 3)), np.zeros(self.nb)
        lib().orc_model_inertia(self.h, _p(m), _p(I), _p(w))
        return m, I, w

    def kinematics(self, q, v=None):
        q = _f64(q)
        v = _f64(v) if v is not None else np.zeros(self.nv)
        xpos, xmat = np.zeros((self.nb, 3)), np.zeros((self.nb, 3, 3))
        M, c, tw = np.zeros((self.nv, self.nv)), np.zeros(self.nv), np.zeros((self.nb, 6))
        lib().orc_kinematics(self.h, _p(q), _p(v), _p(xpos), _p(xmat), _p(M), _p(c), _p(tw))
        return dict(xpos=xpos, xmat=xmat, M=M, c=c, twist=tw)

    def contacts(self, q, cfd=False):
        """Candidate contacts at q, rows (r, pos[3], n[3], t1[3], t2[3])."""
        out = np.zeros((max(self.ncmax, 1), 13))
        n = lib().orc_contacts_cfd(self.h, _p(_f64(q)), int(cfd), _p(out))
        return out[:n]

    def point_jac(self, q, body, point):
        J = np.zeros((3, self.nv))
        lib().orc_point_jac(self.h, _p(_f64(q)), int(body), _p(_f64(point)), _p(J))
        return J

    def rhs(self, x, u=None, cfd=False):
        u = _f64(u if u is not None else np.zeros(max(self.nu, 1)))
        xd = np.zeros(2 * self.nv)
        info = np.zeros(4, np.int32)
        forces = np.zeros(4 * max(self.ncmax, 1) + 4)
        lib().orc_rhs(self.h, _p(_f64(x)), _p(u), int(cfd), _p(xd), _p(info), _p(forces))
        return xd, dict(n_rows=int(info[0]), n_active=int(info[1]), newton_it=int(info[2]), status=int(info[3]),
                        forces=forces[:info[0]].copy())

    def rows(self, x, u=None, cfd=False, beta=1e4):
        u = _f64(u if u is not None else np.zeros(max(self.nu, 1)))
        nrmax = 4 * max(self.ncmax, 1)
        M, a0 = np.zeros((self.nv, self.nv)), np.zeros(self.nv)
        J, aref, D = np.zeros((nrmax, self.nv)), np.zeros(nrmax), np.zeros(nrmax)
        n = lib().orc_rows(self.h, _p(_f64(x)), _p(u), int(cfd), float(beta), _p(M), _p(a0), _p(J), _p(aref), _p(D))
        return dict(M=M, a0=a0, J=J[:n], aref=aref[:n], D=D[:n])

    def rhs_jvp(self, x, u, dx, du=None, st=False, beta=1e4):
        dx = np.atleast_2d(_f64(dx).reshape(-1, self.nx))
        nd = dx.shape[0]
        u = _f64(u if u is not None else np.zeros(max(self.nu, 1)))
        du = _f64(du if du is not None else np.zeros((nd, max(self.nu, 1))))
        xd, dxd = np.zeros(2 * self.nv), np.zeros((nd, 2 * self.nv))
        lib().orc_rhs_jvp(self.h, _p(_f64(x)), _p(u), int(st), float(beta), nd, _p(dx), _p(du), _p(xd), _p(dxd))
        return xd, dxd

    # -------------------------------------------------------------- rollouts
    def _controls(self, u, n_int, W):
        """Contiguous controls [W][n_int][nu]: zeros when u is None (every
        routine reads n_int * nu values per world), at least one element."""
        n = W * n_int * self.nu
        if u is None or not np.size(u):
            return np.zeros(max(1, n))
        u = _f64(u)
        assert u.size == n, (u.size, n)
        return u

    def rollout(self, x0, u, n_int, dt, forced=None, tape_cap=0, log_cap=0, **opts):
        o = make_opts(**opts)
        x0 = _f64(x0)
        u = self._controls(u, n_int, 1)
        xo = np.zeros(self.nx)
        cnt = np.zeros(5, np.int64)
        tape = np.zeros((tape_cap, 2 + self.nx)) if tape_cap else None
        log = np.zeros((log_cap, 4)) if log_cap else None
        fz = _f64(forced) if forced is not None else None
        nf = 0 if forced is None else len(fz) // 2
        lib().orc_rollout(self.h, _p(x0), _p(u), int(n_int), float(dt), C.byref(o), _p(fz), nf, _p(xo), _p(cnt),
                          tape_cap, _p(tape), log_cap, _p(log))
        res = dict(x=xo, n_acc=int(cnt[0]), n_rej=int(cnt[1]), n_rhs=int(cnt[2]), newton_it=int(cnt[3]),
                   status=int(cnt[4]))
        if tape is not None:
            res["tape"] = tape[:min(tape_cap, res["n_acc"])]
        if log is not None:
            res["log"] = log[:min(log_cap, res["n_acc"] + res["n_rej"])]
        return res

    def otd_grad_batch(self, x0, u, n_int, dt, xbar, n_threads=8, **opts):
        """Optimize-then-discretize gradients of sum(xbar * x(T)): x0bar [W, nx]
        (quaternion parts tangent at q0), ubar [W, n_int, nu], and the adjoint's
        attempts and accepted steps."""
        o = make_opts(**opts)
        x0 = np.ascontiguousarray(np.asarray(x0, np.float64).reshape(-1, self.nx))
        W = x0.shape[0]
        nut = n_int * self.nu
        u = self._controls(u, n_int, W)
        xb = np.ascontiguousarray(np.asarray(xbar, np.float64).reshape(W, self.nx))
        xo, x0b = np.zeros((W, self.nx)), np.zeros((W, self.nx))
        ub = np.zeros(max(1, W * nut))
        cnt = np.zeros((W, 4), np.int64)
        lib().orc_otd_grad_batch(self.h, W, _p(x0), _p(u), int(n_int), float(dt), C.byref(o), _p(xb), _p(xo), _p(x0b),
                                 _p(ub), _p(cnt), int(n_threads))
        return dict(x=xo, x0bar=x0b, ubar=ub[:W * nut].reshape(W, n_int, self.nu), adj_attempts=cnt[:, 0],
                    adj_accepted=cnt[:, 1], n_acc=cnt[:, 2], status=cnt[:, 3])

    def dense_states(self, x0, u, n_int, dt, taus, forced=None, **opts):
        """x(tau) at the given times from the continuous extension of the rollout's accepted steps."""
        o = make_opts(**opts)
        taus = _f64(taus)
        u = self._controls(u, n_int, 1)
        fz = _f64(forced) if forced is not None else None
        nf = 0 if forced is None else len(fz) // 2
        out = np.zeros((taus.size, self.nx))
        st = lib().orc_dense_states(self.h, _p(_f64(x0)), _p(u), int(n_int), float(dt), C.byref(o), _p(fz), nf,
                                    taus.size, _p(taus), _p(out))
        assert st == 0, st
        return out

    FLOP_PHASES = ("step", "rhs", "newton", "line_search", "other")

    def flop_count(self, x0, u, n_int, dt, **opts):
        """Floating-point operations of the forward rollout by phase, and its
        work units (attempts, rhs, newton_iters, contacts per rhs, active
        contacts per Newton iteration, contacts per line-search segment)."""
        o = make_opts(**opts)
        x0 = _f64(x0)
        u = self._controls(u, n_int, 1)
        out = np.zeros(16, np.int64)
        lib().orc_flop_count(self.h, _p(x0), _p(u), int(n_int), float(dt), C.byref(o), _p(out))
        res = {f"flops_{p}": int(out[i]) for i, p in enumerate(self.FLOP_PHASES)}
        res.update(attempts=int(out[5]), rhs=int(out[6]), newton_iters=int(out[7]), rhs_contacts=int(out[8]),
                   newton_contacts=int(out[9]), ls_contacts=int(out[10]), n_acc=int(out[11]), status=int(out[12]),
                   rhs_contacts_box=int(out[13]), newton_contacts_box=int(out[14]), ls_contacts_box=int(out[15]))
        return res

    def rollout_jvp(self, x0, u, n_int, dt, dx0, du=None, **opts):
        o = make_opts(**opts)
        dx0 = np.atleast_2d(np.asarray(dx0, np.float64).reshape(-1, self.nx))
        nd = dx0.shape[0]
        nut = n_int * self.nu
        du = _f64(du) if du is not None else np.zeros(nd * max(nut, 1))
        u = self._controls(u, n_int, 1)
        xo, tx = np.zeros(self.nx), np.zeros((nd, self.nx))
        cnt = np.zeros(5, np.int64)
        lib().orc_rollout_jvp(self.h, _p(_f64(x0)), _p(u), int(n_int), float(dt), C.byref(o), nd, _p(_f64(dx0)),
                              _p(du), _p(xo), _p(tx), _p(cnt))
        return dict(x=xo, tx=tx, n_acc=int(cnt[0]), n_rej=int(cnt[1]), status=int(cnt[4]))

    def rollout_jvp_forced(self, x0, u, n_int, dt, forced, dx0, du=None, **opts):
        """Tangents [n_dir][nx] of the final state along (dx0, du) for the frozen
        step sequence forced [n][2]; returns (x_out, tangents)."""
        o = make_opts(**opts)
        dx0 = np.ascontiguousarray(np.atleast_2d(np.asarray(dx0, np.float64).reshape(-1, self.nx)))
        nd = dx0.shape[0]
        nut = n_int * self.nu
        du = _f64(du) if du is not None else np.zeros(nd * max(nut, 1))
        u = self._controls(u, n_int, 1)
        fz = np.ascontiguousarray(forced, np.float64)
        xo, tx = np.zeros(self.nx), np.zeros((nd, self.nx))
        st = lib().orc_rollout_jvp_forced(self.h, _p(_f64(x0)), _p(u), int(n_int), float(dt), C.byref(o), _p(fz),
                                          int(fz.shape[0]), nd, _p(dx0), _p(du), _p(xo), _p(tx))
        assert st == 0, st
        return xo, tx

    def rollout_batch(self, x0, u, n_int, dt, n_threads=1, **opts):
        o = make_opts(**opts)
        x0 = np.ascontiguousarray(x0, np.float64)
        W = x0.shape[0]
        u = self._controls(u, n_int, W)
        xo = np.zeros_like(x0)
        cnt = np.zeros((W, 5), np.int64)
        lib().orc_rollout_batch(self.h, W, _p(x0), _p(u), int(n_int), float(dt), C.byref(o), _p(xo), _p(cnt),
                                int(n_threads))
        return dict(x=xo, n_acc=cnt[:, 0], n_rej=cnt[:, 1], n_rhs=cnt[:, 2], newton_it=cnt[:, 3], status=cnt[:, 4])

    def grad_batch(self, x0, u, n_int, dt, xbar, n_threads=1, **opts):
        o = make_opts(**opts)
        x0 = np.ascontiguousarray(x0, np.float64)
        W = x0.shape[0]
        nut = n_int * self.nu
        u = self._controls(u, n_int, W)
        xbar = np.ascontiguousarray(np.broadcast_to(xbar, x0.shape), np.float64)
        xo, x0b = np.zeros_like(x0), np.zeros_like(x0)
        ub = np.zeros((W, max(nut, 1)))
        cnt = np.zeros((W, 5), np.int64)
        lib().orc_grad_batch(self.h, W, _p(x0), _p(u), int(n_int), float(dt), C.byref(o), _p(xbar), _p(xo),
                             _p(x0b), _p(ub), _p(cnt), int(n_threads))
        return dict(x=xo, x0bar=x0b, ubar=ub[:, :nut].reshape(W, n_int, self.nu), n_acc=cnt[:, 0],
                    n_rej=cnt[:, 1], n_rhs=cnt[:, 2], status=cnt[:, 4])

    def grad_forced_batch(self, x0, u, n_int, dt, xbar, forced, forced_n, n_threads=1, **opts):
        """Gradients along given accepted-step sequences: forced [W][cap][2]
        (t_n, h_n), forced_n [W] steps per world (the controller is off)."""
        o = make_opts(**opts)
        x0 = np.ascontiguousarray(x0, np.float64)
        W = x0.shape[0]
        nut = n_int * self.nu
        u = self._controls(u, n_int, W)
        xbar = np.ascontiguousarray(np.broadcast_to(xbar, x0.shape), np.float64)
        fz = np.ascontiguousarray(forced, np.float64)
        fn = _i32(forced_n)
        xo, x0b = np.zeros_like(x0), np.zeros_like(x0)
        ub = np.zeros((W, max(nut, 1)))
        cnt = np.zeros((W, 5), np.int64)
        lib().orc_grad_forced_batch(self.h, W, _p(x0), _p(u), int(n_int), float(dt), C.byref(o), _p(fz), _p(fn),
                                    int(fz.shape[1]), _p(xbar), _p(xo), _p(x0b), _p(ub), _p(cnt), int(n_threads))
        return dict(x=xo, x0bar=x0b, ubar=ub[:, :nut].reshape(W, n_int, self.nu), n_acc=cnt[:, 0],
                    status=cnt[:, 4])

    def attempt(self, y, u, h, **opts):
        """One attempt from y with step h: (5th-order state, error norm, status)."""
        o = make_opts(**opts)
        u = _f64(u if u is not None and np.size(u) else np.zeros(max(self.nu, 1)))
        yn = np.zeros(self.nx)
        err = C.c_double()
        st = lib().orc_attempt(self.h, _p(_f64(y)), _p(u), float(h), C.byref(o), _p(yn), C.byref(err))
        return yn, err.value, st


def next_step(err, eprev, h, accepted, **opts):
    """The oracle controller's next proposed step and its new memory e_prev."""
    o = make_opts(**opts)
    ep = C.c_double()
    hn = lib().orc_next_step(C.byref(o), float(err), float(eprev), float(h), int(accepted), C.byref(ep))
    return hn, ep.value
