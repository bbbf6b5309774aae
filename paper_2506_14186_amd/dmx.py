"""Thin Python binding of the dmx C ABI (include/dmx.h).

Argument marshalling only: every step of the rollout and of its gradient runs
in the HIP kernels of ``libdmx.so``.  Tensors are PyTorch CUDA tensors (FP64,
contiguous) used as device buffers; the library works on the current torch
stream.  If the library is missing this module raises on import.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdmx.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc, gfx950)")

_lib = C.CDLL(LIB_PATH)
_P = C.c_void_p

JOINT = {"free": 0, "hinge": 1, "slide": 2}
GEOM = {"plane": 0, "sphere": 1, "capsule": 2, "box": 3}
STATUS = {"MAX_STEPS": 1, "DT_UNDERFLOW": 2, "NONFINITE": 4, "SOLVER_MAXIT": 8, "CONTACT_OVERFLOW": 16,
          "TAPE_OVERFLOW": 32, "CONTACT_GRAPH": 64}


class ModelDesc(C.Structure):
    _fields_ = [("nbody", C.c_int32), ("njnt", C.c_int32), ("ngeom", C.c_int32), ("npair", C.c_int32),
                ("nu", C.c_int32)] + [(n, _P) for n in (
                    "body_parent", "body_pos", "body_quat", "body_iner_type", "body_iner_size", "body_iner_quat",
                    "body_mass", "jnt_body", "jnt_type", "jnt_axis", "jnt_pos", "geom_body", "geom_type",
                    "geom_size", "geom_pos", "geom_quat", "pair_g1", "pair_g2", "pair_mu", "pair_solref",
                    "pair_solimp", "pair_cfd", "ctrl_dof")] + [("gravity", C.c_double * 3)]


class SolverOpts(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("rtol", "atol", "h0", "safety", "facmin", "facmax", "kP", "kI",
                                           "err_order", "err_floor")] + [
        ("max_attempts", C.c_int64), ("newton_maxit", C.c_int32), ("cfd", C.c_int32),
        ("softplus_beta", C.c_double), ("tape_steps", C.c_int64), ("lanes_per_world", C.c_int32),
        ("forced", _P), ("forced_n", _P), ("forced_cap", C.c_int32), ("steplog", _P), ("log_n", _P),
        ("log_cap", C.c_int32), ("fwd_counters", _P), ("adj_counters", _P), ("launch_mode", C.c_int32),
        ("h_levels", C.c_int32), ("fail_state", _P), ("world_intervals", _P), ("world_order", _P),
        ("work_queue", C.c_int32), ("tape_stages", C.c_int32), ("tableau", C.c_int32)]

FWD_COUNTERS = ("attempts", "rhs", "rhs_contacts", "newton_iters", "newton_contacts", "newton_edges",
                "ls_contacts", "rhs_contacts_pair", "newton_contacts_pair")
ADJ_COUNTERS = ("steps", "vjps", "vjp_contacts", "vjp_edges")


_lib.dmx_last_error.restype = C.c_char_p
_lib.dmx_default_opts.argtypes = [C.POINTER(SolverOpts)]
_lib.dmx_model_create.argtypes = [C.POINTER(ModelDesc), C.POINTER(_P)]
_lib.dmx_model_info.argtypes = [_P, _P, _P, _P, _P]
_lib.dmx_model_destroy.argtypes = [_P]
_lib.dmx_rollout.argtypes = [_P, C.c_int32, C.c_int32, C.c_double, C.POINTER(SolverOpts), _P, _P, _P, _P, _P, _P,
                             C.POINTER(_P), _P]
_lib.dmx_rollout_vjp.argtypes = [_P, _P, _P, _P, _P]
_lib.dmx_rollout_vjp_otd.argtypes = [_P, _P, _P, _P, _P]
_lib.dmx_rollout_vjp_geom.argtypes = [_P, _P, _P, _P, _P, _P]
_lib.dmx_rollout_vjp_otd_geom.argtypes = [_P, _P, _P, _P, _P, _P]
_lib.dmx_rollout_vjp_params.argtypes = [_P, _P, _P, _P, _P, _P]
_lib.dmx_rollout_vjp_otd_params.argtypes = [_P, _P, _P, _P, _P, _P]
_lib.dmx_accel.argtypes = [_P, C.c_int32, _P, _P, C.c_int32, _P, _P, _P]
_lib.dmx_autotune.argtypes = [_P, C.c_int32, C.c_int32, C.c_double, _P, _P, _P, _P, _P, _P, _P]
_lib.dmx_tape_info.argtypes = [_P, _P, _P]
_lib.dmx_tape_data.argtypes = [_P, _P, _P]
_lib.dmx_tape_destroy.argtypes = [_P]
_lib.dmx_tape_layout.argtypes = [_P, _P, _P]
_lib.dmx_batch_layout.argtypes = [_P, _P, _P, _P, _P]
_lib.dmx_rollout_batch.argtypes = [_P, C.POINTER(SolverOpts), _P, _P, _P, _P, _P, _P, C.POINTER(_P), _P]
_lib.dmx_rollout_noalloc.argtypes = [_P, C.c_int32, C.c_int32, C.c_double, C.POINTER(SolverOpts), _P, _P, _P, _P,
                                     _P, _P, _P]
_lib.dmx_rollout_batch_grad.argtypes = [_P, C.POINTER(SolverOpts), _P, _P, _P, _P, _P, _P, _P, _P, _P,
                                        C.POINTER(_P), _P]
for _f in ("dmx_model_create", "dmx_model_info", "dmx_rollout", "dmx_rollout_vjp", "dmx_tape_info",
           "dmx_tape_data", "dmx_accel", "dmx_autotune", "dmx_tape_layout", "dmx_batch_layout",
           "dmx_rollout_batch", "dmx_rollout_noalloc", "dmx_rollout_batch_grad", "dmx_rollout_vjp_otd",
           "dmx_rollout_vjp_geom", "dmx_rollout_vjp_otd_geom", "dmx_rollout_vjp_params",
           "dmx_rollout_vjp_otd_params"):
    getattr(_lib, _f).restype = C.c_int32

EXPORTS = ["dmx_default_opts", "dmx_model_create", "dmx_model_info", "dmx_model_destroy", "dmx_rollout",
           "dmx_rollout_vjp", "dmx_tape_info", "dmx_tape_data", "dmx_tape_destroy", "dmx_accel", "dmx_autotune",
           "dmx_last_error", "dmx_batch_layout", "dmx_rollout_batch", "dmx_tape_layout", "dmx_rollout_noalloc",
           "dmx_rollout_batch_grad", "dmx_rollout_vjp_otd", "dmx_rollout_vjp_geom",
           "dmx_rollout_vjp_otd_geom", "dmx_rollout_vjp_params", "dmx_rollout_vjp_otd_params"]


class Batch(C.Structure):
    _fields_ = [("n_worlds", C.c_int32), ("models", _P), ("n_intervals", C.c_int32), ("interval_dt", C.c_double)]


class DmxError(RuntimeError):
    pass


def _check(code):
    if code < 0:
        raise DmxError(f"dmx error {code}: {_lib.dmx_last_error().decode()}")
    return code


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def default_opts(**kw):
    o = SolverOpts()
    _lib.dmx_default_opts(C.byref(o))
    names = {f[0] for f in SolverOpts._fields_}
    for k, v in kw.items():
        if k not in names:
            raise TypeError(f"unknown solver option {k!r}")
        setattr(o, k, v)
    return o


def _f64(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64).ravel())


def _i32(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.int32).ravel())


class Model:
    """A compiled model on the current device (wraps dmx_model_create)."""

    def __init__(self, desc):
        bodies, geoms, pairs = desc["bodies"], desc["geoms"], desc["pairs"]
        jb, jt, ja, jp = [], [], [], []
        for bi, b in enumerate(bodies):
            for j in b["joints"]:
                jb.append(bi)
                jt.append(JOINT[j["type"]])
                ja.append(j["axis"])
                jp.append(j["pos"])
        pad3 = lambda s: list(s) + [0.0] * (3 - len(s))  # noqa: E731
        arrs = dict(
            body_parent=_i32([b["parent"] for b in bodies]), body_pos=_f64([b["pos"] for b in bodies]),
            body_quat=_f64([b["quat"] for b in bodies]),
            body_iner_type=_i32([GEOM[b["inertial"]["type"]] for b in bodies]),
            body_iner_size=_f64([pad3(b["inertial"]["size"]) for b in bodies]),
            body_iner_quat=_f64([b["inertial"].get("quat", [1.0, 0.0, 0.0, 0.0]) for b in bodies]),
            body_mass=_f64([b["inertial"]["mass"] if b["inertial"]["mass"] is not None else -1.0 for b in bodies]),
            jnt_body=_i32(jb), jnt_type=_i32(jt), jnt_axis=_f64(ja), jnt_pos=_f64(jp),
            geom_body=_i32([g["body"] for g in geoms]), geom_type=_i32([GEOM[g["type"]] for g in geoms]),
            geom_size=_f64([pad3(g["size"]) for g in geoms]), geom_pos=_f64([g["pos"] for g in geoms]),
            geom_quat=_f64([g["quat"] for g in geoms]), pair_g1=_i32([p["g1"] for p in pairs]),
            pair_g2=_i32([p["g2"] for p in pairs]), pair_mu=_f64([p["mu"] for p in pairs]),
            pair_solref=_f64([p["solref"] for p in pairs]), pair_solimp=_f64([p["solimp"] for p in pairs]),
            pair_cfd=_f64([p["cfd"] for p in pairs]), ctrl_dof=_i32(desc["ctrl"]["dofs"]))
        d = ModelDesc()
        d.nbody, d.njnt, d.ngeom, d.npair, d.nu = len(bodies), len(jb), len(geoms), len(pairs), len(
            desc["ctrl"]["dofs"])
        for k, a in arrs.items():
            setattr(d, k, a.ctypes.data if a.size else None)
        for i in range(3):
            d.gravity[i] = desc["gravity"][i]
        h = _P()
        _check(_lib.dmx_model_create(C.byref(d), C.byref(h)))
        self.h = h
        sz = (C.c_int32 * 4)()
        _check(_lib.dmx_model_info(h, C.byref(sz, 0), C.byref(sz, 4), C.byref(sz, 8), C.byref(sz, 12)))
        self.nq, self.nv, self.nu, self.ncon = list(sz)
        self.nx = self.nq + self.nv

    def __del__(self):
        if getattr(self, "h", None):
            try:
                _lib.dmx_model_destroy(self.h)
            except Exception:
                pass
            self.h = None


class Tape:
    def __init__(self, h, model, W, n_int):
        self.h, self.model, self.W, self.n_int = h, model, W, n_int

    def info(self):
        s, r = C.c_int64(), C.c_int32()
        _check(_lib.dmx_tape_info(self.h, C.byref(s), C.byref(r)))
        return s.value, r.value

    def layout(self):
        """Per-world record offsets and lengths (doubles)."""
        off = np.zeros(self.W, np.int64)
        rec = np.zeros(self.W, np.int32)
        _check(_lib.dmx_tape_layout(self.h, off.ctypes.data, rec.ctypes.data))
        return off, rec

    def world_records(self):
        """Ragged tapes: per world the records [n_steps][rec] (host), and n_steps [W]."""
        cap, _ = self.info()
        off, rec = self.layout()
        rp, npp = C.c_void_p(), C.c_void_p()
        _check(_lib.dmx_tape_data(self.h, C.byref(rp), C.byref(npp)))
        torch.cuda.synchronize()
        n = torch.as_tensor(_DevArray(npp.value, (self.W,), "<i4"), device="cuda").cpu().numpy()
        total = int(off[-1] + cap * rec[-1]) if self.W else 0
        flat = torch.as_tensor(_DevArray(rp.value, (max(total, 1),), "<f8"), device="cuda")
        out = []
        for w in range(self.W):
            seg = flat[int(off[w]):int(off[w]) + int(n[w]) * int(rec[w])]
            out.append(seg.cpu().numpy().reshape(int(n[w]), int(rec[w])))
        return out, n

    def records(self):
        """(records [W][steps][rec] float64, n_steps [W] int32) copied to the host."""
        cap, rec = self.info()
        if getattr(self, "ragged", False):
            per, n = self.world_records()
            width = max(r.shape[1] for r in per)
            out = np.zeros((self.W, max(int(n.max()), 1), width))
            for w, r in enumerate(per):
                out[w, :r.shape[0], :r.shape[1]] = r
            return out, n
        rp, npp = C.c_void_p(), C.c_void_p()
        _check(_lib.dmx_tape_data(self.h, C.byref(rp), C.byref(npp)))
        torch.cuda.synchronize()
        n = torch.as_tensor(_DevArray(npp.value, (self.W,), "<i4"), device="cuda").cpu().numpy()
        recs = torch.as_tensor(_DevArray(rp.value, (self.W, cap, rec), "<f8"), device="cuda")
        nmax = int(n.max()) if self.W else 0
        return recs[:, :max(nmax, 1)].cpu().numpy(), n

    def __del__(self):
        if getattr(self, "h", None):
            try:
                _lib.dmx_tape_destroy(self.h)
            except Exception:
                pass
            self.h = None


class _DevArray:
    """A library-owned device buffer exposed to torch (read-only view)."""

    def __init__(self, ptr, shape, typestr):
        self.__cuda_array_interface__ = {"shape": tuple(shape), "typestr": typestr, "data": (int(ptr), False),
                                         "version": 3, "strides": None}


def autotune(model, x0, u, n_int, dt):
    """Time every compiled team size on this batch (CUDA float64 tensors) and
    make the fastest the model's default.  Returns (best, {lanes: ms})."""
    W = x0.shape[0]
    best, n = C.c_int32(), C.c_int32()
    lanes, ms = (C.c_int32 * 8)(), (C.c_double * 8)()
    _check(_lib.dmx_autotune(model.h, W, int(n_int), float(dt), _ptr(x0), _ptr(u), _stream(), C.byref(best),
                             C.byref(n), lanes, ms))
    return best.value, {lanes[i]: ms[i] for i in range(min(n.value, 8))}


def rollout(model, x0, u, n_int, dt, opts=None, tape=False, counters=False, reuse=None):
    """Forward rollout.  x0 [W, nx] and u [W, n_int, nu] CUDA float64.
    Returns dict(x, status[, tape][, n_acc, n_rej]).  ``reuse``: a Tape of the
    same model and batch size whose buffers are overwritten (no allocation)."""
    x0 = x0.contiguous()
    W = x0.shape[0]
    assert x0.dtype == torch.float64 and x0.is_cuda and x0.shape[1] == model.nx
    if model.nu:
        u = u.contiguous()
        assert u.dtype == torch.float64 and u.is_cuda and tuple(u.shape) == (W, n_int, model.nu)
    else:
        u = None
    x_out = torch.empty_like(x0)
    status = torch.empty(W, dtype=torch.int32, device=x0.device)
    nacc = torch.zeros(W, dtype=torch.int32, device=x0.device) if counters else None
    nrej = torch.zeros(W, dtype=torch.int32, device=x0.device) if counters else None
    o = opts if opts is not None else default_opts()
    th = _P(reuse.h.value if isinstance(reuse.h, _P) else reuse.h) if reuse is not None else _P()
    tape = tape or reuse is not None
    _check(_lib.dmx_rollout(model.h, W, int(n_int), float(dt), C.byref(o), _ptr(x0), _ptr(u), _ptr(x_out),
                            _ptr(status), _ptr(nacc), _ptr(nrej), C.byref(th) if tape else None, _stream()))
    res = {"x": x_out, "status": status}
    if counters:
        res["n_acc"], res["n_rej"] = nacc, nrej
    if reuse is not None:
        reuse.n_int = n_int
        reuse.keep = (x0, u)  # the tape reads u during the reverse sweep
        res["tape"] = reuse
    elif tape:
        res["tape"] = Tape(th, model, W, n_int)
        res["tape"].keep = (x0, u)
    return res


def rollout_noalloc(model, x0, u, n_int, dt, x_out, status, opts=None, n_acc=None, n_rej=None):
    """Forward rollout without a tape that allocates no device memory (the
    library's static scratch holds its work-queue counter); every output
    buffer is the caller's: x_out [W, nx] float64, status [W] int32 (and
    optionally n_acc, n_rej [W] int32), CUDA tensors."""
    W = x0.shape[0]
    assert x0.is_contiguous() and x_out.is_contiguous() and status.is_contiguous()
    o = opts if opts is not None else default_opts()
    _check(_lib.dmx_rollout_noalloc(model.h, W, int(n_int), float(dt), C.byref(o), _ptr(x0),
                                    _ptr(u) if model.nu else None, _ptr(x_out), _ptr(status), _ptr(n_acc),
                                    _ptr(n_rej), _stream()))


def batch_layout(models, n_int):
    """Offsets of each world's state and controls in the packed arrays of an
    uneven batch, and the totals."""
    arr = (_P * len(models))(*[m.h for m in models])
    b = Batch(len(models), C.cast(arr, _P), int(n_int), 1.0)
    xo = np.zeros(len(models), np.int64)
    uo = np.zeros(len(models), np.int64)
    nx, nu = C.c_int64(), C.c_int64()
    _check(_lib.dmx_batch_layout(C.byref(b), xo.ctypes.data, uo.ctypes.data, C.byref(nx), C.byref(nu)))
    return xo, uo, nx.value, nu.value


class BatchTape(Tape):
    """Tape of an uneven batch (per-world records of different lengths)."""

    def __init__(self, h, models, n_int, xo, uo, nx, nu):
        super().__init__(h, models[0], len(models), n_int)
        self.models, self.ragged = models, True
        self.xo, self.uo, self.nx, self.nu = xo, uo, nx, nu


def rollout_batch(models, x0, u, n_int, dt, opts=None, tape=False, counters=False, reuse=None):
    """Forward rollout of an uneven batch: models (list, one per world), x0
    packed states [sum nx_w] and u packed controls [sum n_int nu_w] (or None),
    CUDA float64.  Returns dict(x, status[, tape][, n_acc, n_rej])."""
    W = len(models)
    xo, uo, nx, nu = batch_layout(models, n_int)
    x0 = x0.contiguous()
    assert x0.dtype == torch.float64 and x0.is_cuda and x0.numel() == nx
    if nu:
        u = u.contiguous()
        assert u.dtype == torch.float64 and u.numel() == nu
    else:
        u = None
    arr = (_P * W)(*[m.h for m in models])
    b = Batch(W, C.cast(arr, _P), int(n_int), float(dt))
    x_out = torch.empty_like(x0)
    status = torch.empty(W, dtype=torch.int32, device=x0.device)
    nacc = torch.zeros(W, dtype=torch.int32, device=x0.device) if counters else None
    nrej = torch.zeros(W, dtype=torch.int32, device=x0.device) if counters else None
    o = opts if opts is not None else default_opts()
    th = _P(reuse.h.value if isinstance(reuse.h, _P) else reuse.h) if reuse is not None else _P()
    tape = tape or reuse is not None
    _check(_lib.dmx_rollout_batch(C.byref(b), C.byref(o), _ptr(x0), _ptr(u), _ptr(x_out), _ptr(status),
                                  _ptr(nacc), _ptr(nrej), C.byref(th) if tape else None, _stream()))
    res = {"x": x_out, "status": status, "x_off": xo, "u_off": uo}
    if counters:
        res["n_acc"], res["n_rej"] = nacc, nrej
    if reuse is not None:
        reuse.keep = (x0, u)
        res["tape"] = reuse
    elif tape:
        res["tape"] = BatchTape(th, models, n_int, xo, uo, nx, nu)
        res["tape"].keep = (x0, u)
    return res


def rollout_batch_grad(models, x0, u, n_int, dt, x_out_bar, opts=None, counters=False, reuse=None):
    """Forward rollout and reverse sweep of an uneven batch in one launch for
    a final-state cotangent x_out_bar given up front (packed, CUDA float64).
    Returns dict(x, status, x0_bar, u_bar, tape[, n_acc, n_rej]); the tape
    serves later rollout_batch_vjp calls and reuse=."""
    W = len(models)
    xo, uo, nx, nu = batch_layout(models, n_int)
    x0 = x0.contiguous()
    assert x0.dtype == torch.float64 and x0.is_cuda and x0.numel() == nx
    xb = x_out_bar.contiguous()
    assert xb.dtype == torch.float64 and xb.is_cuda and xb.numel() == nx
    if nu:
        u = u.contiguous()
        assert u.dtype == torch.float64 and u.numel() == nu
    else:
        u = None
    arr = (_P * W)(*[m.h for m in models])
    b = Batch(W, C.cast(arr, _P), int(n_int), float(dt))
    x_out = torch.empty_like(x0)
    x0b = torch.empty_like(x0)
    ub = torch.empty(nu, dtype=torch.float64, device=x0.device) if nu else None
    status = torch.empty(W, dtype=torch.int32, device=x0.device)
    nacc = torch.zeros(W, dtype=torch.int32, device=x0.device) if counters else None
    nrej = torch.zeros(W, dtype=torch.int32, device=x0.device) if counters else None
    o = opts if opts is not None else default_opts()
    th = _P(reuse.h.value if isinstance(reuse.h, _P) else reuse.h) if reuse is not None else _P()
    _check(_lib.dmx_rollout_batch_grad(C.byref(b), C.byref(o), _ptr(x0), _ptr(u), _ptr(xb), _ptr(x_out),
                                       _ptr(status), _ptr(nacc), _ptr(nrej), _ptr(x0b), _ptr(ub), C.byref(th),
                                       _stream()))
    res = {"x": x_out, "status": status, "x0_bar": x0b, "u_bar": ub, "x_off": xo, "u_off": uo}
    if counters:
        res["n_acc"], res["n_rej"] = nacc, nrej
    if reuse is not None:
        reuse.keep = (x0, u)
        res["tape"] = reuse
    else:
        res["tape"] = BatchTape(th, models, n_int, xo, uo, nx, nu)
        res["tape"].keep = (x0, u)
    return res


def rollout_batch_vjp(tape, x_out_bar):
    """Packed x0_bar and u_bar of sum(x_out_bar * x_out) for an uneven batch."""
    xb = x_out_bar.contiguous()
    x0b = torch.empty_like(xb)
    ub = torch.empty(tape.nu, dtype=torch.float64, device=xb.device) if tape.nu else None
    _check(_lib.dmx_rollout_vjp(tape.h, _ptr(xb), _ptr(x0b), _ptr(ub), _stream()))
    return x0b, ub


def rollout_batch_vjp_params(tape, x_out_bar):
    """Packed x0_bar, u_bar and the model-parameter gradient [W, 12] (columns
    PARAMS) of sum(x_out_bar * x_out) for an uneven batch."""
    xb = x_out_bar.contiguous()
    x0b = torch.empty_like(xb)
    ub = torch.empty(tape.nu, dtype=torch.float64, device=xb.device) if tape.nu else None
    pb = torch.empty((tape.W, len(PARAMS)), dtype=torch.float64, device=xb.device)
    _check(_lib.dmx_rollout_vjp_params(tape.h, _ptr(xb), _ptr(x0b), _ptr(ub), _ptr(pb), _stream()))
    return x0b, ub, pb


def accel(model, x, tau=None, cfd=False):
    """Accelerations F(x) at independent states x [n, nx] (and generalized forces tau [n, nv])."""
    x = x.contiguous()
    n = x.shape[0]
    acc = torch.empty((n, model.nv), dtype=torch.float64, device=x.device)
    st = torch.empty(n, dtype=torch.int32, device=x.device)
    tau = tau.contiguous() if tau is not None else None
    _check(_lib.dmx_accel(model.h, n, _ptr(x), _ptr(tau), int(cfd), _ptr(acc), _ptr(st), _stream()))
    return acc, st


def rollout_vjp(tape, x_out_bar):
    """x0_bar [W, nx], u_bar [W, n_int, nu] of sum(x_out_bar * x_out)."""
    xb = x_out_bar.contiguous()
    m = tape.model
    x0b = torch.empty_like(xb)
    ub = torch.empty((tape.W, tape.n_int, m.nu), dtype=torch.float64, device=xb.device) if m.nu else None
    _check(_lib.dmx_rollout_vjp(tape.h, _ptr(xb), _ptr(x0b), _ptr(ub), _stream()))
    return x0b, ub


def rollout_vjp_geom(tape, x_out_bar):
    """x0_bar [W, nx], u_bar [W, n_int, nu] and the box geom half sizes' gradient
    [W, 3] of sum(x_out_bar * x_out) through the recorded discretization."""
    xb = x_out_bar.contiguous()
    m = tape.model
    x0b = torch.empty_like(xb)
    hb = torch.empty((tape.W, 3), dtype=torch.float64, device=xb.device)
    ub = torch.empty((tape.W, tape.n_int, m.nu), dtype=torch.float64, device=xb.device) if m.nu else None
    _check(_lib.dmx_rollout_vjp_geom(tape.h, _ptr(xb), _ptr(x0b), _ptr(ub), _ptr(hb), _stream()))
    return x0b, ub, hb


def rollout_vjp_otd_geom(tape, x_out_bar):
    """Optimize-then-discretize x0_bar, u_bar and the box half sizes' gradient [W, 3]."""
    xb = x_out_bar.contiguous()
    m = tape.model
    x0b = torch.empty_like(xb)
    hb = torch.empty((tape.W, 3), dtype=torch.float64, device=xb.device)
    ub = torch.empty((tape.W, tape.n_int, m.nu), dtype=torch.float64, device=xb.device) if m.nu else None
    _check(_lib.dmx_rollout_vjp_otd_geom(tape.h, _ptr(xb), _ptr(x0b), _ptr(ub), _ptr(hb), _stream()))
    return x0b, ub, hb


PARAMS = ("half_x", "half_y", "half_z", "friction", "solref_timeconst", "solref_dampratio", "mass",
          "solimp_d0", "solimp_dwidth", "solimp_width", "solimp_midpoint", "solimp_power")


def _params(fn, tape, x_out_bar):
    xb = x_out_bar.contiguous()
    m = tape.model
    x0b = torch.empty_like(xb)
    pb = torch.empty((tape.W, len(PARAMS)), dtype=torch.float64, device=xb.device)
    ub = torch.empty((tape.W, tape.n_int, m.nu), dtype=torch.float64, device=xb.device) if m.nu else None
    _check(fn(tape.h, _ptr(xb), _ptr(x0b), _ptr(ub), _ptr(pb), _stream()))
    return x0b, ub, pb


def rollout_vjp_params(tape, x_out_bar):
    """x0_bar, u_bar and the model-parameter gradient [W, 12] (columns PARAMS)
    of sum(x_out_bar * x_out) through the recorded discretization."""
    return _params(_lib.dmx_rollout_vjp_params, tape, x_out_bar)


def rollout_vjp_otd_params(tape, x_out_bar):
    """Optimize-then-discretize x0_bar, u_bar and model-parameter gradient [W, 12]."""
    return _params(_lib.dmx_rollout_vjp_otd_params, tape, x_out_bar)


def rollout_vjp_otd(tape, x_out_bar):
    """Optimize-then-discretize x0_bar [W, nx] (quaternion parts tangent at
    x0), u_bar [W, n_int, nu] of sum(x_out_bar * x_out)."""
    xb = x_out_bar.contiguous()
    m = tape.model
    x0b = torch.empty_like(xb)
    ub = torch.empty((tape.W, tape.n_int, m.nu), dtype=torch.float64, device=xb.device) if m.nu else None
    _check(_lib.dmx_rollout_vjp_otd(tape.h, _ptr(xb), _ptr(x0b), _ptr(ub), _stream()))
    return x0b, ub


class Rollout(torch.autograd.Function):
    """x_out = rollout(x0, u); backward runs the discrete adjoint kernel."""

    @staticmethod
    def forward(ctx, x0, u, model, n_int, dt, opts):
        r = rollout(model, x0, u if model.nu else None, n_int, dt, opts=opts, tape=True)
        ctx.tape = r["tape"]
        ctx.has_u = model.nu > 0
        ctx.mark_non_differentiable(r["status"])
        return r["x"], r["status"]

    @staticmethod
    def backward(ctx, xb, _sb):
        x0b, ub = rollout_vjp(ctx.tape, xb)
        return x0b, (ub if ctx.has_u else None), None, None, None, None


# ------------------------------------------------------------------ serving
class ServerOpts(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_int64), ("max_inflight", C.c_int32), ("n_streams", C.c_int32),
                ("steps_per_interval", C.c_int32), ("max_batch_worlds", C.c_int32),
                ("stack_steps_per_interval", C.c_int32)]


class Request(C.Structure):
    _fields_ = [("model", _P), ("n_worlds", C.c_int32), ("n_intervals", C.c_int32), ("interval_dt", C.c_double),
                ("x0", _P), ("u", _P), ("target", C.c_double * 3), ("ctrl_weight", C.c_double),
                ("want_grad", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("cost", _P), ("grad_u", _P), ("world_status", _P), ("t_submit", C.c_double),
                ("t_start", C.c_double), ("t_done", C.c_double)]


_lib.dmx_default_server_opts.argtypes = [C.POINTER(ServerOpts)]
_lib.dmx_server_create.argtypes = [C.POINTER(ServerOpts), C.POINTER(_P)]
_lib.dmx_submit.argtypes = [_P, C.POINTER(Request), C.POINTER(C.c_uint64)]
_lib.dmx_poll.argtypes = [_P, C.c_uint64, C.POINTER(Result)]
_lib.dmx_server_stats.argtypes = [_P, _P, _P, _P]
_lib.dmx_server_destroy.argtypes = [_P]
for _f in ("dmx_server_create", "dmx_submit", "dmx_poll", "dmx_server_stats"):
    getattr(_lib, _f).restype = C.c_int32
EXPORTS += ["dmx_default_server_opts", "dmx_server_create", "dmx_submit", "dmx_poll", "dmx_server_stats",
            "dmx_server_destroy"]
DMX_PENDING = 1


class Server:
    """Request loop on the current device (wraps dmx_server_*)."""

    def __init__(self, **kw):
        o = ServerOpts()
        _lib.dmx_default_server_opts(C.byref(o))
        names = {f[0] for f in ServerOpts._fields_}
        for k, v in kw.items():
            if k not in names:
                raise TypeError(f"unknown server option {k!r}")
            setattr(o, k, v)
        h = _P()
        _check(_lib.dmx_server_create(C.byref(o), C.byref(h)))
        self.h = h
        self._pending = {}

    def submit(self, model, x0, u, dt, target=(0.0, 0.0, 0.0), ctrl_weight=1e-3, want_grad=True):
        x0 = _f64(x0)
        u = np.ascontiguousarray(u, dtype=np.float64) if model.nu else np.zeros((1, 1, 0))
        N, H = u.shape[0], u.shape[1]
        q = Request()
        q.model, q.n_worlds, q.n_intervals, q.interval_dt = model.h, N, H, float(dt)
        q.x0, q.u = x0.ctypes.data, (u.ctypes.data if u.size else None)
        for i in range(3):
            q.target[i] = float(target[i])
        q.ctrl_weight, q.want_grad = float(ctrl_weight), int(want_grad)
        t = C.c_uint64()
        _check(_lib.dmx_submit(self.h, C.byref(q), C.byref(t)))
        self._pending[t.value] = (np.zeros(N), np.zeros((N, H, model.nu)), np.zeros(N, np.int32))
        return t.value

    def poll(self, ticket):
        cost, grad, st = self._pending.get(ticket) or (np.zeros(1), np.zeros((1, 1, 0)), np.zeros(1, np.int32))
        r = Result()
        r.cost, r.grad_u, r.world_status = cost.ctypes.data, (grad.ctypes.data if grad.size else None), st.ctypes.data
        code = _check(_lib.dmx_poll(self.h, C.c_uint64(ticket), C.byref(r)))
        if code == DMX_PENDING:
            return None
        self._pending.pop(ticket, None)
        return {"cost": cost, "grad_u": grad, "status": st, "t_submit": r.t_submit, "t_start": r.t_start,
                "t_done": r.t_done}

    def stats(self):
        q, i, b = C.c_int32(), C.c_int32(), C.c_int64()
        _check(_lib.dmx_server_stats(self.h, C.byref(q), C.byref(i), C.byref(b)))
        return q.value, i.value, b.value

    def close(self):
        if getattr(self, "h", None):
            _lib.dmx_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_lib.dmx_graph_create.argtypes = [C.POINTER(Batch), C.POINTER(SolverOpts), _P, _P, _P, _P, _P, _P, _P, _P,
                                  C.POINTER(_P)]
_lib.dmx_graph_create.restype = C.c_int32
_lib.dmx_graph_launch.argtypes = [_P, _P]
_lib.dmx_graph_launch.restype = C.c_int32
_lib.dmx_graph_tape.argtypes = [_P]
_lib.dmx_graph_tape.restype = _P
_lib.dmx_graph_destroy.argtypes = [_P]
EXPORTS += ["dmx_graph_create", "dmx_graph_launch", "dmx_graph_tape", "dmx_graph_destroy"]


class Graph:
    """A captured rollout segment (wraps dmx_graph_*): the forward rollout of
    `models` (one per world) over n_int intervals of dt and, with grad, its
    reverse sweep, recorded once over fixed device buffers.  Write new inputs
    into .x0, .u and .xbar in place (e.g. x0.copy_(...)), then replay(); the
    results appear in .x, .status, .x0bar and .ubar."""

    def __init__(self, models, x0, u, n_int, dt, opts=None, grad=True):
        W = len(models)
        nx = sum(m.nx for m in models)
        nu = sum(int(n_int) * m.nu for m in models)
        self.x0 = x0.contiguous().clone()
        assert self.x0.dtype == torch.float64 and self.x0.is_cuda and self.x0.numel() == nx
        self.u = None
        if nu:
            self.u = u.contiguous().clone()
            assert self.u.dtype == torch.float64 and self.u.numel() == nu
        self.x = torch.empty_like(self.x0)
        self.status = torch.empty(W, dtype=torch.int32, device=self.x0.device)
        self.xbar = torch.zeros_like(self.x0) if grad else None
        self.x0bar = torch.empty_like(self.x0) if grad else None
        self.ubar = torch.empty_like(self.u) if (grad and nu) else None
        self._arr = (_P * W)(*[m.h for m in models])
        self.models = models
        b = Batch(W, C.cast(self._arr, _P), int(n_int), float(dt))
        o = opts if opts is not None else default_opts()
        h = _P()
        _check(_lib.dmx_graph_create(C.byref(b), C.byref(o), _ptr(self.x0), _ptr(self.u), _ptr(self.x),
                                     _ptr(self.status), _ptr(self.xbar), _ptr(self.x0bar), _ptr(self.ubar),
                                     _stream(), C.byref(h)))
        self.h = h

    def replay(self):
        _check(_lib.dmx_graph_launch(self.h, _stream()))

    def close(self):
        if getattr(self, "h", None):
            _lib.dmx_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Tuning(C.Structure):
    _fields_ = [("lanes_per_world", C.c_int32), ("tape_stages", C.c_int32), ("work_queue", C.c_int32),
                ("ms", C.c_double)]


_lib.dmx_autotune_batch.argtypes = [C.POINTER(Batch), _P, _P, _P, C.POINTER(Tuning), C.POINTER(C.c_int32),
                                    C.POINTER(Tuning)]
_lib.dmx_autotune_batch.restype = C.c_int32
EXPORTS += ["dmx_autotune_batch"]


def autotune_batch(models, x0, u, n_int, dt):
    """Launch choices (tape policy, work distribution, team size) timed on
    this batch (dmx_autotune_batch).  Returns (best, tried): dicts with
    lanes_per_world, tape_stages, work_queue and ms."""
    W = len(models)
    arr = (_P * W)(*[m.h for m in models])
    b = Batch(W, C.cast(arr, _P), int(n_int), float(dt))
    x0 = x0.contiguous()
    u = u.contiguous() if u is not None else None
    best, tried, n = Tuning(), (Tuning * 32)(), C.c_int32()
    _check(_lib.dmx_autotune_batch(C.byref(b), _ptr(x0), _ptr(u), _stream(), C.byref(best), C.byref(n), tried))
    as_dict = lambda t: {f[0]: getattr(t, f[0]) for f in Tuning._fields_}  # noqa: E731
    return as_dict(best), [as_dict(tried[i]) for i in range(min(n.value, 32))]
