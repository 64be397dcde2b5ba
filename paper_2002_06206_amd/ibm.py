"""Python binding of the C ABI in include/ibm.h (ctypes; argument marshalling only).

Every function named ``ibm_*`` here calls the C entry point of the same name in
libibm.so with device pointers taken from torch tensors and the current torch
stream; torch is used for device memory and streams only.  All arithmetic of the
step runs in the library's gfx950 kernels.  If libibm.so is missing or cannot be
loaded this module raises at import: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libibm.so")

PERIODIC, INFLOW, OUTFLOW, SLIP = 0, 1, 2, 3
FP64, MIXED = 0, 1
SOLVER_PCG_JACOBI, SOLVER_FCG_CNN, SOLVER_FCG_JACOBI, SOLVER_RBSOR = 0, 1, 2, 3
BCM_BICGSTAB, BCM_SOR = 0, 1
SCHEME_AB2, SCHEME_CN = 0, 1
OK, NOT_CONVERGED = 0, 1


class IBMError(RuntimeError):
    pass


class Grid(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("dx", ctypes.c_double), ("origin", ctypes.c_double * 3)]


class BC(ctypes.Structure):
    _fields_ = [("face", ctypes.c_int32 * 6), ("u_in", ctypes.c_double * 3)]


class SolverOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("kind", ctypes.c_int32),
                ("inner_tol", ctypes.c_double), ("inner_max_iter", ctypes.c_int32),
                ("stall_factor", ctypes.c_double), ("check_every", ctypes.c_int32),
                ("force_stall", ctypes.c_int32), ("omega", ctypes.c_double), ("inner_restart", ctypes.c_int32),
                ("pad", ctypes.c_int32)]


class StepParams(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("dt_prev", ctypes.c_double), ("nu", ctypes.c_double),
                ("c1", ctypes.c_double),
                ("csm_on", ctypes.c_int32), ("step", ctypes.c_int32), ("body_force", ctypes.c_double * 3),
                ("poisson", SolverOpts), ("scheme", ctypes.c_int32), ("mom_max_iter", ctypes.c_int32),
                ("mom_tol", ctypes.c_double), ("quick", ctypes.c_double), ("p_prev", ctypes.c_void_p)]


class Stats(ctypes.Structure):
    _fields_ = [("iters_inner", ctypes.c_int32), ("iters_outer", ctypes.c_int32),
                ("fallback_used", ctypes.c_int32), ("status", ctypes.c_int32),
                ("rel_residual", ctypes.c_double), ("div_l2", ctypes.c_double), ("div_linf", ctypes.c_double),
                ("umax", ctypes.c_double), ("iters_momentum", ctypes.c_int32 * 3),
                ("iters_fallback", ctypes.c_int32)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_ if f != "pad"}
        d["iters_momentum"] = list(d["iters_momentum"])
        return d


PROGRESS_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_int64, ctypes.c_double)


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libibm.so is not built (run: python -m paper_2002_06206_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    P3 = vp * 3
    sig = {
        "ibm_create": ([ctypes.POINTER(Grid), ctypes.POINTER(BC), ctypes.c_int32, ctypes.POINTER(vp)], ctypes.c_int),
        "ibm_destroy": ([vp], ctypes.c_int),
        "ibm_last_error": ([], ctypes.c_char_p),
        "ibm_alloc_count": ([ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
        "ibm_tag_geometry": ([vp, vp, ctypes.c_int64, ctypes.c_double, vp, vp, vp], ctypes.c_int),
        "ibm_build_stencils": ([vp, vp, vp, ctypes.c_int32, vp, vp, ctypes.POINTER(ctypes.c_int64), vp],
                               ctypes.c_int),
        "ibm_cut_points": ([vp, vp, vp], ctypes.c_int),
        "ibm_init_state": ([vp, P3, P3, vp, P3, ctypes.POINTER(ctypes.c_double), vp, vp], ctypes.c_int),
        "ibm_step": ([vp, P3, P3, vp, P3, vp, ctypes.POINTER(StepParams), ctypes.POINTER(Stats), vp],
                     ctypes.c_int),
        "ibm_poisson_solve": ([vp, vp, vp, ctypes.POINTER(SolverOpts), ctypes.POINTER(Stats), vp], ctypes.c_int),
        "ibm_apply_laplacian": ([vp, vp, vp, vp], ctypes.c_int),
        "ibm_get_nut": ([vp, vp, vp], ctypes.c_int),
        "ibm_get_rhs": ([vp, vp, vp], ctypes.c_int),
        "ibm_forces": ([vp, P3, vp, vp, ctypes.c_double, vp, ctypes.POINTER(ctypes.c_double), vp], ctypes.c_int),
        "ibm_forces_noalloc": ([vp, P3, vp, vp, ctypes.c_double, vp, vp, vp], ctypes.c_int),
        "ibm_shepard_force": ([vp, vp, ctypes.c_int64, vp, ctypes.c_int32, vp, ctypes.POINTER(ctypes.c_double), vp],
                              ctypes.c_int),
        "ibm_timing_enable": ([vp, ctypes.c_int32], ctypes.c_int),
        "ibm_timing_read": ([vp, ctypes.POINTER(ctypes.c_double), ctypes.c_int32], ctypes.c_int),
        "ibm_timing_slot": ([vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_double), ctypes.c_int32], ctypes.c_int),
        "ibm_prepare_crank_nicolson": ([vp], ctypes.c_int),
        "ibm_momentum_apply": ([vp, P3, P3, vp, ctypes.c_double, ctypes.c_double, P3, vp], ctypes.c_int),
        "ibm_momentum_solve": ([vp, P3, P3, P3, vp, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), vp], ctypes.c_int),
        "ibm_set_progress": ([vp, PROGRESS_FN, vp], ctypes.c_int),
        "ibm_cnn_create": ([ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(vp)], ctypes.c_int),
        "ibm_cnn_destroy": ([vp], ctypes.c_int),
        "ibm_cnn_set_weights": ([vp, vp, ctypes.c_int64], ctypes.c_int),
        "ibm_cnn_get_weights": ([vp, vp, ctypes.c_int64], ctypes.c_int),
        "ibm_cnn_forward": ([vp, vp, vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp], ctypes.c_int),
        "ibm_cnn_backward": ([vp, vp, vp, vp, vp], ctypes.c_int),
        "ibm_cnn_loss": ([vp, vp, vp, vp, ctypes.c_double, ctypes.POINTER(ctypes.c_double), vp, vp], ctypes.c_int),
        "ibm_cnn_train_step": ([vp, vp, vp, vp, ctypes.c_float, ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                                vp],
                               ctypes.c_int),
        "ibm_cnn_precondition": ([vp, vp, vp, vp, ctypes.c_double, vp], ctypes.c_int),
        "ibm_ctx_set_preconditioner": ([vp, vp], ctypes.c_int),
        "ibm_bcm_create": ([ctypes.POINTER(ctypes.c_int32), ctypes.c_int32, ctypes.c_double,
                            ctypes.POINTER(ctypes.c_double), vp, ctypes.POINTER(vp)], ctypes.c_int),
        "ibm_bcm_destroy": ([vp], ctypes.c_int),
        "ibm_bcm_info": ([vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                          ctypes.POINTER(ctypes.c_int64), vp, vp], ctypes.c_int),
        "ibm_bcm_exchange": ([vp, vp, vp], ctypes.c_int),
        "ibm_bcm_laplacian": ([vp, vp, vp, vp], ctypes.c_int),
        "ibm_bcm_sor": ([vp, vp, vp, ctypes.c_double, ctypes.c_int32, vp], ctypes.c_int),
        "ibm_bcm_set_blocked": ([vp, ctypes.c_int32, vp, vp], ctypes.c_int),
        "ibm_bcm_solve": ([vp, ctypes.c_int32, vp, vp, ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                           ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double), vp],
                          ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


_lib = _load()
EXPORTED = ("ibm_create", "ibm_destroy", "ibm_last_error", "ibm_alloc_count", "ibm_tag_geometry", "ibm_build_stencils",
            "ibm_cut_points", "ibm_init_state", "ibm_step", "ibm_poisson_solve", "ibm_apply_laplacian",
            "ibm_get_nut", "ibm_get_rhs", "ibm_forces", "ibm_forces_noalloc", "ibm_shepard_force", "ibm_timing_enable", "ibm_timing_read",
            "ibm_timing_slot", "ibm_set_progress", "ibm_prepare_crank_nicolson", "ibm_momentum_apply",
            "ibm_momentum_solve",
            "ibm_cnn_create", "ibm_cnn_destroy", "ibm_cnn_set_weights", "ibm_cnn_get_weights", "ibm_cnn_forward",
            "ibm_cnn_backward", "ibm_cnn_loss", "ibm_cnn_train_step", "ibm_cnn_precondition",
            "ibm_ctx_set_preconditioner", "ibm_bcm_create", "ibm_bcm_destroy", "ibm_bcm_info", "ibm_bcm_exchange",
            "ibm_bcm_laplacian", "ibm_bcm_sor", "ibm_bcm_set_blocked", "ibm_bcm_solve")
CNN_NWEIGHTS = 7776


def lib():
    return _lib


def _check(rc, what):
    if rc < 0:
        msg = _lib.ibm_last_error()
        raise IBMError("%s failed (%d): %s" % (what, rc, msg.decode() if msg else ""))
    return rc


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise IBMError("fields must be contiguous CUDA (HIP) tensors")
    return ctypes.c_void_p(t.data_ptr())


def _p3(ts):
    return (ctypes.c_void_p * 3)(*[t.data_ptr() for t in ts])


# ------------------------------------------------------------ C ABI, same names

def ibm_create(n, dx, origin, bc, u_in=(0.0, 0.0, 0.0), precision=FP64):
    g = Grid((ctypes.c_int32 * 3)(*n), float(dx), (ctypes.c_double * 3)(*origin))
    b = BC((ctypes.c_int32 * 6)(*bc), (ctypes.c_double * 3)(*u_in))
    out = ctypes.c_void_p()
    _check(_lib.ibm_create(ctypes.byref(g), ctypes.byref(b), int(precision), ctypes.byref(out)), "ibm_create")
    return out


def alloc_count():
    """Device and pinned-host allocations the library has made in this process."""
    n = ctypes.c_int64(0)
    _check(_lib.ibm_alloc_count(ctypes.byref(n)), "ibm_alloc_count")
    return int(n.value)


def ibm_destroy(ctx):
    return _check(_lib.ibm_destroy(ctx), "ibm_destroy")


def ibm_tag_geometry(ctx, tri, blocked, theta=None, bary_eps=0.0):
    assert tri.dtype == torch.float64 and blocked.dtype == torch.uint8
    return _check(_lib.ibm_tag_geometry(ctx, _ptr(tri), tri.shape[0] if tri.numel() else 0, float(bary_eps),
                                        _ptr(blocked), _ptr(theta), _stream()), "ibm_tag_geometry")


def ibm_build_stencils(ctx, blocked, theta=None, deadend=False, flags=None, label=None):
    ncut = ctypes.c_int64(0)
    _check(_lib.ibm_build_stencils(ctx, _ptr(blocked), _ptr(theta), int(bool(deadend)), _ptr(flags), _ptr(label),
                                   ctypes.byref(ncut), _stream()), "ibm_build_stencils")
    return int(ncut.value)


def ibm_cut_points(ctx, xyz):
    return _check(_lib.ibm_cut_points(ctx, _ptr(xyz), _stream()), "ibm_cut_points")


def ibm_init_state(ctx, u, U, p, h, u0, wall=None):
    return _check(_lib.ibm_init_state(ctx, _p3(u), _p3(U), _ptr(p), _p3(h), (ctypes.c_double * 3)(*u0),
                                      _ptr(wall), _stream()), "ibm_init_state")


def ibm_step(ctx, u, U, p, h, params: StepParams, wall=None, want_stats=True):
    st = Stats()
    rc = _check(_lib.ibm_step(ctx, _p3(u), _p3(U), _ptr(p), _p3(h), _ptr(wall), ctypes.byref(params),
                              ctypes.byref(st) if want_stats else None, _stream()), "ibm_step")
    return rc, (st.as_dict() if want_stats else None)


def ibm_poisson_solve(ctx, b, x, opts: SolverOpts):
    st = Stats()
    rc = _check(_lib.ibm_poisson_solve(ctx, _ptr(b), _ptr(x), ctypes.byref(opts), ctypes.byref(st), _stream()),
                "ibm_poisson_solve")
    return rc, st.as_dict()


def ibm_apply_laplacian(ctx, x, y):
    return _check(_lib.ibm_apply_laplacian(ctx, _ptr(x), _ptr(y), _stream()), "ibm_apply_laplacian")


def ibm_get_nut(ctx, out):
    return _check(_lib.ibm_get_nut(ctx, _ptr(out), _stream()), "ibm_get_nut")


def ibm_get_rhs(ctx, out):
    return _check(_lib.ibm_get_rhs(ctx, _ptr(out), _stream()), "ibm_get_rhs")


def ibm_forces(ctx, u, p, nu, nut=None, wall=None):
    out = (ctypes.c_double * 6)()
    _check(_lib.ibm_forces(ctx, _p3(u), _ptr(p), _ptr(nut), float(nu), _ptr(wall), out, _stream()), "ibm_forces")
    return list(out[:3]), list(out[3:])


def ibm_forces_noalloc(ctx, u, p, nu, out, nut=None, wall=None):
    """ibm_forces without allocation or host wait: the six sums (F_p xyz, F_v xyz) go to
    the device tensor out (6 doubles) on the current stream."""
    return _check(_lib.ibm_forces_noalloc(ctx, _p3(u), _ptr(p), _ptr(nut), float(nu), _ptr(wall), _ptr(out),
                                          _stream()), "ibm_forces_noalloc")


def ibm_shepard_force(ctx, tri, p, side=None, thin_filter=False):
    """Near-field pressure force (eq. (force)) of triangles tri (ntri, 3, 3, FP64,
    device) on the cell pressure p; fills side (ntri, 2) when given; thin_filter applies
    the filter Z of eq. (force_filter).  Returns the force as three floats."""
    out = (ctypes.c_double * 3)()
    ntri = int(tri.shape[0]) if tri is not None else 0
    _check(_lib.ibm_shepard_force(ctx, _ptr(tri), ntri, _ptr(p), int(bool(thin_filter)), _ptr(side), out, _stream()),
           "ibm_shepard_force")
    return list(out)


def ibm_prepare_crank_nicolson(ctx):
    return _check(_lib.ibm_prepare_crank_nicolson(ctx), "ibm_prepare_crank_nicolson")


def ibm_momentum_apply(ctx, q, U, nut, nu, dt, out):
    """out = (I - dt/2 L) q for the three velocity components (eq. (crank-nicolson));
    q, out: three cell fields of the context's cell type; nut: cell field or None."""
    return _check(_lib.ibm_momentum_apply(ctx, _p3(q), _p3(U), _ptr(nut), float(nu), float(dt), _p3(out),
                                          _stream()), "ibm_momentum_apply")


def ibm_momentum_solve(ctx, b, x, U, nut, nu, dt, tol, max_iter):
    """BiCGStab for (I - dt/2 L) x = b, x in/out (initial guess / solution); returns
    (return code, iterations per component)."""
    it = (ctypes.c_int32 * 3)()
    rc = _check(_lib.ibm_momentum_solve(ctx, _p3(b), _p3(x), _p3(U), _ptr(nut), float(nu), float(dt), float(tol),
                                        int(max_iter), it, _stream()), "ibm_momentum_solve")
    return rc, list(it)


def ibm_timing_slot(ctx, slot, reset=False):
    """(milliseconds, launches) accumulated in one timed slot."""
    out = (ctypes.c_double * 2)()
    _check(_lib.ibm_timing_slot(ctx, int(slot), out, int(bool(reset))), "ibm_timing_slot")
    return float(out[0]), int(out[1])


def ibm_timing_enable(ctx, on=True):
    return _check(_lib.ibm_timing_enable(ctx, int(bool(on))), "ibm_timing_enable")


def ibm_set_progress(ctx, fn):
    """fn(iterations, rr) or None; returns the ctypes callback, which the caller keeps alive."""
    cb = PROGRESS_FN(lambda user, it, rr: fn(int(it), float(rr))) if fn is not None else PROGRESS_FN()
    _check(_lib.ibm_set_progress(ctx, cb, None), "ibm_set_progress")
    return cb


def ibm_timing_read(ctx, reset=False):
    out = (ctypes.c_double * 10)()
    _check(_lib.ibm_timing_read(ctx, out, int(bool(reset))), "ibm_timing_read")
    v = list(out)
    return {"ms": v[0:3], "launches": [int(x) for x in v[3:6]], "real_iters": int(v[6]), "cells": int(v[7]),
            "cuts": int(v[8]), "precision": int(v[9])}


CNN_INFERENCE_ONLY = 1


def ibm_cnn_create(max_cells, flags=0):
    out = ctypes.c_void_p()
    _check(_lib.ibm_cnn_create(int(max_cells), int(flags), ctypes.byref(out)), "ibm_cnn_create")
    return out


def ibm_cnn_destroy(net):
    return _check(_lib.ibm_cnn_destroy(net), "ibm_cnn_destroy")


def ibm_cnn_set_weights(net, w):
    import numpy as np
    a = np.ascontiguousarray(w, dtype=np.float32)
    return _check(_lib.ibm_cnn_set_weights(net, a.ctypes.data_as(ctypes.c_void_p), a.size), "ibm_cnn_set_weights")


def ibm_cnn_get_weights(net):
    import numpy as np
    a = np.empty(CNN_NWEIGHTS, dtype=np.float32)
    _check(_lib.ibm_cnn_get_weights(net, a.ctypes.data_as(ctypes.c_void_p), a.size), "ibm_cnn_get_weights")
    return a


def ibm_cnn_forward(net, x_bf16, y, n):
    """x_bf16: (nz, ny, nx, 2) torch.bfloat16 (or int16 bit patterns); y: (nz, ny, nx) float32."""
    return _check(_lib.ibm_cnn_forward(net, _ptr(x_bf16), _ptr(y), int(n[0]), int(n[1]), int(n[2]), _stream()),
                  "ibm_cnn_forward")


def ibm_cnn_backward(net, dy, dw, dx=None):
    return _check(_lib.ibm_cnn_backward(net, _ptr(dy), _ptr(dw), _ptr(dx), _stream()), "ibm_cnn_backward")


def ibm_cnn_loss(net, ctx, b, p, dw=None, omega=0.0):
    loss = ctypes.c_double()
    _check(_lib.ibm_cnn_loss(net, ctx, _ptr(b), _ptr(p), float(omega), ctypes.byref(loss), _ptr(dw), _stream()),
           "ibm_cnn_loss")
    return loss.value


def ibm_cnn_train_step(net, ctx, b, p, lr, omega=0.0):
    loss = ctypes.c_double()
    _check(_lib.ibm_cnn_train_step(net, ctx, _ptr(b), _ptr(p), float(lr), float(omega), ctypes.byref(loss),
                                   _stream()), "ibm_cnn_train_step")
    return loss.value


def ibm_cnn_precondition(net, ctx, r, z, omega=0.0):
    return _check(_lib.ibm_cnn_precondition(net, ctx, _ptr(r), _ptr(z), float(omega), _stream()),
                  "ibm_cnn_precondition")


def ibm_ctx_set_preconditioner(ctx, net):
    return _check(_lib.ibm_ctx_set_preconditioner(ctx, net), "ibm_ctx_set_preconditioner")


# ------------------------------------------------------------- convenience

def solver_opts(tol=1e-10, max_iter=20000, kind=SOLVER_PCG_JACOBI, inner_tol=1e-2, inner_max_iter=200,
                stall_factor=2.0, check_every=16, force_stall=0, omega=0.0, inner_restart=0):
    return SolverOpts(tol, max_iter, kind, inner_tol, inner_max_iter, stall_factor, check_every, force_stall,
                      float(omega), int(inner_restart), 0)


def step_params(dt, nu, c1=1.0 / 20.0, csm=True, step=0, body=(0.0, 0.0, 0.0), dt_prev=0.0, scheme="ab2",
                mom_tol=1e-10, mom_max_iter=200, quick=0.0, p_prev=None, **solver):
    """p_prev: None, or a float64 device tensor holding the previous pressure (the solve
    then starts from 2 p - p_prev, and p_prev receives p)."""
    sc = {"ab2": SCHEME_AB2, "cn": SCHEME_CN}[scheme]
    if p_prev is not None and p_prev.dtype != torch.float64:
        raise IBMError("p_prev must be a float64 tensor")
    return StepParams(dt, dt_prev, nu, c1, int(bool(csm)), int(step), (ctypes.c_double * 3)(*body),
                      solver_opts(**solver), sc, int(mom_max_iter), float(mom_tol), float(quick),
                      None if p_prev is None else _ptr(p_prev))


class Solver:
    """Owns one context and the flow state on the current HIP device."""

    def __init__(self, n, dx, origin, bc, u_in=(0.0, 0.0, 0.0), precision=FP64, device=None):
        self.n = tuple(int(v) for v in n)
        self.shape = (self.n[2], self.n[1], self.n[0])
        self.dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.precision = precision
        self.ftype = torch.float64 if precision == FP64 else torch.float32
        self.ctx = ibm_create(self.n, dx, origin, bc, u_in, precision)
        self.ncut = 0

    def close(self):
        if self.ctx is not None:
            ibm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def tag(self, tri, want_theta=True, bary_eps=0.0):
        """Blocked bits and (when want_theta) the dense theta; the context keeps its own
        compact tagging for the next build either way."""
        tri_t = torch.as_tensor(tri, dtype=torch.float64).to(self.dev).contiguous()
        blocked = torch.zeros(self.shape, dtype=torch.uint8, device=self.dev)
        theta = torch.empty(self.shape + (6,), dtype=torch.float64, device=self.dev) if want_theta else None
        ibm_tag_geometry(self.ctx, tri_t.reshape(-1, 3, 3), blocked, theta, bary_eps)
        del tri_t
        return blocked, theta

    def build(self, blocked, theta=None, deadend=False):
        flags = torch.empty(self.shape, dtype=torch.int16, device=self.dev)
        label = torch.empty(self.shape, dtype=torch.int32, device=self.dev)
        self.ncut = ibm_build_stencils(self.ctx, blocked, theta, deadend, flags, label)
        return flags, label

    def cut_points(self):
        X = torch.empty((max(self.ncut, 1), 3), dtype=torch.float64, device=self.dev)
        ibm_cut_points(self.ctx, X)
        return X[: self.ncut]

    def new_state(self, u0, wall=None):
        z = lambda dt: torch.empty(self.shape, dtype=dt, device=self.dev)  # noqa: E731
        st = {"u": [z(self.ftype) for _ in range(3)], "U": [z(torch.float64) for _ in range(3)],
              "p": z(torch.float64), "h": [z(self.ftype) for _ in range(3)]}
        ibm_init_state(self.ctx, st["u"], st["U"], st["p"], st["h"], u0, wall)
        return st

    def step(self, st, params, wall=None, want_stats=True):
        if params.scheme == SCHEME_CN:
            self.prepare_crank_nicolson()
        return ibm_step(self.ctx, st["u"], st["U"], st["p"], st["h"], params, wall, want_stats)

    def prepare_crank_nicolson(self):
        """Allocates the Crank-Nicolson workspace once (set-up, outside the time step)."""
        if not getattr(self, "_cn_ready", False):
            ibm_prepare_crank_nicolson(self.ctx)
            self._cn_ready = True

    def poisson(self, b, x, **opts):
        return ibm_poisson_solve(self.ctx, b, x, solver_opts(**opts))

    def laplacian(self, x):
        y = torch.empty_like(x)
        ibm_apply_laplacian(self.ctx, x, y)
        return y

    def nut(self):
        out = torch.empty(self.shape, dtype=self.ftype, device=self.dev)
        ibm_get_nut(self.ctx, out)
        return out

    def rhs(self):
        out = torch.empty(self.shape, dtype=torch.float64, device=self.dev)
        ibm_get_rhs(self.ctx, out)
        return out

    def forces(self, st, nu, wall=None):
        return ibm_forces(self.ctx, st["u"], st["p"], nu, None, wall)

    def momentum_apply(self, q, U, nut, nu, dt, out):
        return ibm_momentum_apply(self.ctx, q, U, nut, nu, dt, out)

    def momentum_solve(self, b, x, U, nut, nu, dt, tol=1e-10, max_iter=200):
        self.prepare_crank_nicolson()
        return ibm_momentum_solve(self.ctx, b, x, U, nut, nu, dt, tol, max_iter)

    def shepard_force(self, tri, p, side=None, thin_filter=False):
        return ibm_shepard_force(self.ctx, tri, p, side, thin_filter)


class Network:
    """Owns one learned-preconditioner network on the current HIP device."""

    def __init__(self, max_cells, weights=None, inference_only=False):
        self.net = ibm_cnn_create(max_cells, CNN_INFERENCE_ONLY if inference_only else 0)
        if weights is not None:
            ibm_cnn_set_weights(self.net, weights)

    def close(self):
        if self.net is not None:
            ibm_cnn_destroy(self.net)
            self.net = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def weights(self):
        return ibm_cnn_get_weights(self.net)

    @weights.setter
    def weights(self, w):
        ibm_cnn_set_weights(self.net, w)

    def train_step(self, solver: "Solver", b, p, lr, omega=0.0):
        return ibm_cnn_train_step(self.net, solver.ctx, b, p, lr, omega)

    def loss(self, solver: "Solver", b, p, dw=None, omega=0.0):
        return ibm_cnn_loss(self.net, solver.ctx, b, p, dw, omega)

    def attach(self, solver: "Solver"):
        ibm_ctx_set_preconditioner(solver.ctx, self.net)


class BCM:
    """Building-cube grid (Sec. 2.2) on the current HIP device: two levels of n^3-cell
    cubes, halo exchange and the 7-point operator (ibm_bcm_*)."""

    def __init__(self, K, n, dx0, origin, refine):
        import numpy as np
        ref = np.ascontiguousarray(np.asarray(refine, dtype=np.uint8).reshape(K[2], K[1], K[0]))
        out = ctypes.c_void_p()
        _check(_lib.ibm_bcm_create((ctypes.c_int32 * 3)(*K), int(n), float(dx0), (ctypes.c_double * 3)(*origin),
                                   ref.ctypes.data_as(ctypes.c_void_p), ctypes.byref(out)), "ibm_bcm_create")
        self.grid = out
        nc, size, nh = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(_lib.ibm_bcm_info(self.grid, ctypes.byref(nc), ctypes.byref(size), ctypes.byref(nh), None, None),
               "ibm_bcm_info")
        self.ncubes, self.size, self.nhalo = nc.value, size.value, nh.value
        lv = np.zeros(self.ncubes, dtype=np.int32)
        org = np.zeros((self.ncubes, 3), dtype=np.int32)
        _check(_lib.ibm_bcm_info(self.grid, None, None, None, lv.ctypes.data_as(ctypes.c_void_p),
                                 org.ctypes.data_as(ctypes.c_void_p)), "ibm_bcm_info")
        self.levels, self.origins = lv, org
        self.n = int(n)

    def exchange(self, data):
        return _check(_lib.ibm_bcm_exchange(self.grid, _ptr(data), _stream()), "ibm_bcm_exchange")

    def laplacian(self, x, y):
        return _check(_lib.ibm_bcm_laplacian(self.grid, _ptr(x), _ptr(y), _stream()), "ibm_bcm_laplacian")

    def sor(self, b, x, omega, sweeps):
        return _check(_lib.ibm_bcm_sor(self.grid, _ptr(b), _ptr(x), float(omega), int(sweeps), _stream()),
                      "ibm_bcm_sor")

    def set_blocked(self, level, blocked):
        """Blocked bits of one level's uniform grid over the domain (uint8 device tensor,
        (nz, ny, nx) of that level) for the cubes of that level."""
        assert blocked.dtype == torch.uint8 and blocked.is_contiguous()
        return _check(_lib.ibm_bcm_set_blocked(self.grid, int(level), _ptr(blocked), _stream()),
                      "ibm_bcm_set_blocked")

    def solve(self, b, x, kind=BCM_BICGSTAB, omega=1.0, tol=1e-8, max_iter=10000, check_every=16):
        """L x = b on the cube interiors (ibm_bcm_solve); x (cube storage) in/out.
        Returns (rc, iterations or sweeps, true relative residual)."""
        it, rel = ctypes.c_int32(), ctypes.c_double()
        rc = _check(_lib.ibm_bcm_solve(self.grid, int(kind), _ptr(b), _ptr(x), float(omega), float(tol),
                                       int(max_iter), int(check_every), ctypes.byref(it), ctypes.byref(rel),
                                       _stream()), "ibm_bcm_solve")
        return rc, it.value, rel.value

    def close(self):
        if self.grid:
            ibm_bcm_destroy(self.grid)
            self.grid = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ibm_bcm_destroy(grid):
    return _check(_lib.ibm_bcm_destroy(grid), "ibm_bcm_destroy")
