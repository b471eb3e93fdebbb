"""Python binding of the KFBI HIP library (``include/kfbi.h``).

Argument marshalling only: every step of the method runs in the HIP kernels of
``libkfbi.so``.  PyTorch supplies device memory and the stream.  There is no
CPU fallback: importing this module fails when the library is not built.
"""
from __future__ import annotations

import ctypes as ct
import os
import threading

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libkfbi.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2404_15249_amd.build`")

_lib = ct.CDLL(LIB_PATH)

OK = 0
NOT_CONVERGED = 1
ERR_GEOMETRY = -2
ERR_BUDGET = -5
ERR_NONFINITE = -6


class KfbiError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class GeometryError(KfbiError):
    pass


class NonfiniteError(KfbiError):
    """A NaN or Inf in the data of a call (KFBI_ERR_NONFINITE); nothing was written."""


class _Desc(ct.Structure):
    _fields_ = [("lo", ct.c_double), ("hi", ct.c_double), ("n", ct.c_int), ("kappa", ct.c_double),
                ("m", ct.c_int), ("xy", ct.POINTER(ct.c_double)), ("tol", ct.c_double),
                ("restart", ct.c_int), ("max_iter", ct.c_int), ("precision", ct.c_int),
                ("refine_steps", ct.c_int)]

class _Desc3(ct.Structure):
    _fields_ = [("n", ct.c_int), ("lo", ct.c_double), ("hi", ct.c_double), ("kappa", ct.c_double),
                ("axes", ct.c_double * 3), ("tol", ct.c_double), ("restart", ct.c_int), ("max_iter", ct.c_int)]


class _GsDesc(ct.Structure):
    _fields_ = [("lo", ct.c_double), ("hi", ct.c_double), ("n", ct.c_int), ("m", ct.c_int), ("xy", ct.c_void_p),
                ("gamma", ct.c_double), ("kill", ct.c_double), ("eps0", ct.c_double), ("eps1", ct.c_double),
                ("eps2", ct.c_double), ("dt", ct.c_double), ("tol", ct.c_double), ("restart", ct.c_int),
                ("max_iter", ct.c_int)]


FP64 = 0            # KFBI_FP64
FP32_REFINED = 1    # KFBI_FP32_REFINED
_PRECISION = {"fp64": FP64, "fp32": FP32_REFINED}


class Tiles(ct.Structure):
    """Launch shapes of a problem's kernels (``kfbi_tiles``)."""
    _fields_ = [("modes_per_group", ct.c_int), ("modes_groups", ct.c_int), ("dst_cols", ct.c_int),
                ("apply_us", ct.c_double), ("grid_solve_us", ct.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_vp = ct.c_void_p
_sigs = {
    "kfbi_ctx_create": [ct.c_int, _vp, ct.POINTER(_vp)],
    "kfbi_ctx_destroy": [_vp],
    "kfbi_ctx_sync": [_vp],
    "kfbi_prob_create": [_vp, ct.POINTER(_Desc), ct.POINTER(_vp)],
    "kfbi_prob_destroy": [_vp],
    "kfbi_prob_info": [_vp, ct.POINTER(ct.c_int), ct.POINTER(ct.c_int), ct.POINTER(ct.c_int), ct.POINTER(ct.c_size_t)],
    "kfbi_prob_mask": [_vp, _vp],
    "kfbi_prob_crossings": [_vp, _vp, _vp, _vp, _vp],
    "kfbi_prob_irregular": [_vp, _vp],
    "kfbi_prob_points": [_vp, _vp, _vp],
    "kfbi_apply": [_vp, _vp, _vp],
    "kfbi_apply_noalloc": [_vp, _vp, _vp],
    "kfbi_solve": [_vp, _vp, _vp, _vp, _vp, _vp, _vp, ct.POINTER(ct.c_int), ct.POINTER(ct.c_double)],
    "kfbi_gmres": [_vp, _vp, _vp, ct.c_double, ct.c_int, ct.POINTER(ct.c_int), ct.POINTER(ct.c_int),
                   ct.POINTER(ct.c_double)],
    "kfbi_correct": [_vp, _vp, _vp, _vp],
    "kfbi_fast_solve": [_vp, _vp, _vp],
    "kfbi_interface_solve": [_vp, _vp, _vp, _vp, _vp, _vp],
    "kfbi_interface_solve_jumps": [_vp, _vp, _vp, _vp, _vp, _vp],
    "kfbi_richardson": [_vp, _vp, _vp, ct.c_double, ct.c_double, ct.c_int, ct.POINTER(ct.c_int),
                        ct.POINTER(ct.c_double)],
    "kfbi_bicgstab": [_vp, _vp, _vp, ct.c_double, ct.c_int, ct.POINTER(ct.c_int), ct.POINTER(ct.c_int),
                      ct.POINTER(ct.c_double)],
    "kfbi_solve_method": [_vp, ct.c_int, ct.c_double, _vp, _vp, _vp, _vp, _vp, _vp, ct.POINTER(ct.c_int),
                          ct.POINTER(ct.c_double)],
    "kfbi_apply_neumann": [_vp, _vp, _vp],
    "kfbi_interface_solve_neumann": [_vp, _vp, _vp, _vp, _vp, _vp, _vp],
    "kfbi_gmres_neumann": [_vp, _vp, _vp, ct.c_double, ct.c_int, ct.POINTER(ct.c_int), ct.POINTER(ct.c_int),
                           ct.POINTER(ct.c_double)],
    "kfbi_solve_neumann": [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, ct.POINTER(ct.c_int), ct.POINTER(ct.c_double)],
    "kfbi_batch_create": [_vp, ct.c_int, ct.c_int, ct.c_size_t, ct.POINTER(_vp)],
    "kfbi_batch_destroy": [_vp],
    "kfbi_batch_estimate_bytes": [ct.c_int, ct.c_int, ct.c_int, ct.POINTER(ct.c_size_t)],
    "kfbi_batch_admit": [_vp, _vp, _vp, _vp, _vp, ct.POINTER(ct.c_int)],
    "kfbi_batch_step": [_vp, ct.c_int],
    "kfbi_batch_poll": [_vp, _vp, _vp, _vp],
    "kfbi_batch_finish": [_vp, ct.c_int, _vp, _vp, _vp],
    "kfbi_batch_info": [_vp, ct.POINTER(ct.c_int), ct.POINTER(ct.c_size_t)],
    "kfbi_prob_autotune": [_vp, ct.c_int, ct.POINTER(Tiles)],
    "kfbi_prob_get_tiles": [_vp, ct.POINTER(Tiles)],
    "kfbi_prob_set_tiles": [_vp, ct.POINTER(Tiles)],
    "kfbi3_prob_create": [_vp, ct.POINTER(_Desc3), ct.POINTER(_vp)],
    "kfbi3_prob_destroy": [_vp],
    "kfbi3_prob_info": [_vp, ct.POINTER(ct.c_int), ct.POINTER(ct.c_int), ct.POINTER(ct.c_size_t)],
    "kfbi3_prob_points": [_vp, _vp, _vp],
    "kfbi3_prob_mask": [_vp, _vp],
    "kfbi3_prob_irregular": [_vp, _vp],
    "kfbi3_jumps": [_vp, _vp, _vp, _vp],
    "kfbi3_apply": [_vp, _vp, _vp],
    "kfbi3_interface_solve": [_vp, _vp, _vp, _vp, _vp, _vp],
    "kfbi3_solve": [_vp, _vp, _vp, _vp, _vp, _vp, _vp, ct.POINTER(ct.c_int), ct.POINTER(ct.c_double)],
    "kfbi3_gmres": [_vp, _vp, _vp, ct.c_double, ct.c_int, ct.POINTER(ct.c_int), ct.POINTER(ct.c_int),
                    ct.POINTER(ct.c_double)],
    "kfbi_gs_create": [_vp, ct.POINTER(_GsDesc), ct.POINTER(_vp)],
    "kfbi_gs_destroy": [_vp],
    "kfbi_gs_info": [_vp, ct.POINTER(ct.c_int), ct.POINTER(ct.c_int), ct.POINTER(ct.c_longlong)],
    "kfbi_gs_set_state": [_vp, _vp, _vp, _vp, _vp],
    "kfbi_gs_get_state": [_vp, _vp, _vp, _vp, _vp],
    "kfbi_gs_step": [_vp, ct.c_int],
    "kfbi_prob_set_reorth": [_vp, ct.c_double],
    "kfbi_set_timing": [_vp, ct.c_int],
    "kfbi_apply_timing": [_vp, ct.POINTER(ct.c_double), ct.POINTER(ct.c_double), ct.POINTER(ct.c_double),
                          ct.POINTER(ct.c_int)],
}
for _name, _args in _sigs.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = ct.c_int
_lib.kfbi_status_str.argtypes = [ct.c_int]
_lib.kfbi_status_str.restype = ct.c_char_p
_lib.kfbi_last_error.argtypes = []
_lib.kfbi_last_error.restype = ct.c_char_p

EXPORTED = tuple(_sigs) + ("kfbi_status_str", "kfbi_last_error")


def _check(status, allow=(OK,)):
    if status in allow:
        return status
    msg = _lib.kfbi_last_error().decode() or _lib.kfbi_status_str(status).decode()
    if status == ERR_GEOMETRY:
        raise GeometryError(status, msg)
    if status == ERR_NONFINITE:
        raise NonfiniteError(status, msg)
    raise KfbiError(status, msg)


def _dptr(t, name, numel=None):
    """Device pointer of a contiguous float64 CUDA tensor (None -> NULL)."""
    if t is None:
        return None
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float64 tensor on the GPU")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")
    return _vp(t.data_ptr())


class Context:
    """A device and the HIP stream the library enqueues on.

    By default the context owns a dedicated torch stream (default priority).
    Every call orders itself after the caller's current stream and makes the
    current stream wait for the library's work, so tensors flow between torch
    and the library without explicit synchronisation.  A caller that makes the
    context's stream its current torch stream (``torch.cuda.set_stream``) has
    one stream, and the calls skip that ordering.
    """

    def __init__(self, device: int = 0, stream: torch.cuda.Stream | None = None):
        self.device = device
        if stream is not None and stream.cuda_stream == 0:
            # the C library reads a null stream as "make your own": the two would differ
            raise ValueError("pass a created stream (torch.cuda.Stream), not the default stream")
        self.stream = stream if stream is not None else torch.cuda.Stream(device=device)
        h = _vp()
        _check(_lib.kfbi_ctx_create(device, _vp(self.stream.cuda_stream), ct.byref(h)))
        self._h = h
        self._tls = threading.local()     # per-thread events, made once and reused

    def _events(self):
        ev = getattr(self._tls, "ev", None)
        if ev is None:
            ev = self._tls.ev = (torch.cuda.Event(), torch.cuda.Event())
        return ev

    def __enter__(self):
        cur = torch.cuda.current_stream(self.device)
        if cur.cuda_stream != self.stream.cuda_stream:   # nothing to order on one stream
            ev = self._events()[0]
            ev.record(cur)
            self.stream.wait_event(ev)
        return self

    def __exit__(self, *exc):
        cur = torch.cuda.current_stream(self.device)
        if cur.cuda_stream != self.stream.cuda_stream:
            ev = self._events()[1]
            ev.record(self.stream)
            cur.wait_event(ev)
        return False

    def sync(self):
        _check(_lib.kfbi_ctx_sync(self._h))

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.kfbi_ctx_destroy(self._h)
        self._h = None

    def __del__(self):
        self.close()


class Problem:
    """One domain on one grid: the geometry plan and the device workspace."""

    def __init__(self, ctx: Context, xy, n: int, kappa: float, lo: float = -1.2, hi: float = 1.2,
                 tol: float = 1e-10, restart: int = 50, max_iter: int = 500, precision: str = "fp64",
                 refine_steps: int = 1):
        """``precision``: "fp64", or "fp32" (FP32 grid transforms with ``refine_steps``
        FP64 residual corrections) for the dense grid solves."""
        self.ctx = ctx
        xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1, 2)
        self._xy = xy
        if precision not in _PRECISION:
            raise ValueError(f"precision must be one of {sorted(_PRECISION)}")
        self.precision, self.refine_steps = precision, int(refine_steps)
        d = _Desc(lo, hi, int(n), float(kappa), xy.shape[0], xy.ctypes.data_as(ct.POINTER(ct.c_double)),
                  float(tol), int(restart), int(max_iter), _PRECISION[precision], int(refine_steps))
        h = _vp()
        _check(_lib.kfbi_prob_create(ctx._h, ct.byref(d), ct.byref(h)))
        self._h = h
        self.n, self.kappa, self.lo, self.hi = int(n), float(kappa), lo, hi
        m, q, ni, nb = ct.c_int(), ct.c_int(), ct.c_int(), ct.c_size_t()
        _check(_lib.kfbi_prob_info(h, ct.byref(m), ct.byref(q), ct.byref(ni), ct.byref(nb)))
        self.M, self.Q, self.I, self.device_bytes = m.value, q.value, ni.value, nb.value

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.kfbi_prob_destroy(self._h)
        self._h = None

    def __del__(self):
        self.close()

    @property
    def grid_numel(self):
        return (self.n + 1) ** 2

    # ---- plan export (host)
    def mask(self) -> np.ndarray:
        out = np.zeros((self.n + 1, self.n + 1), dtype=np.uint8)
        _check(_lib.kfbi_prob_mask(self._h, _vp(out.ctypes.data)))
        return out.astype(bool)

    def crossings(self):
        axis = np.zeros(self.Q, dtype=np.int32)
        nodes = np.zeros((self.Q, 4), dtype=np.int32)
        t = np.zeros(self.Q)
        xy = np.zeros((self.Q, 2))
        _check(_lib.kfbi_prob_crossings(self._h, _vp(axis.ctypes.data), _vp(nodes.ctypes.data),
                                        _vp(t.ctypes.data), _vp(xy.ctypes.data)))
        return axis, nodes, t, xy

    def irregular(self) -> np.ndarray:
        ij = np.zeros((self.I, 2), dtype=np.int32)
        _check(_lib.kfbi_prob_irregular(self._h, _vp(ij.ctypes.data)))
        return ij

    def points(self):
        """The control points (M x 2) and the spline's unit outward normals there (M x 2)."""
        xy = np.zeros((self.M, 2))
        nrm = np.zeros((self.M, 2))
        _check(_lib.kfbi_prob_points(self._h, _vp(xy.ctypes.data), _vp(nrm.ctypes.data)))
        return xy, nrm

    # ---- device work
    def apply(self, phi: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        if out is None:
            out = torch.empty_like(phi)
        with self.ctx:
            _check(_lib.kfbi_apply(self._h, _dptr(phi, "phi", self.M), _dptr(out, "out", self.M)))
        return out

    def apply_noalloc(self, phi: torch.Tensor, out: torch.Tensor) -> torch.Tensor:
        """``kfbi_apply_noalloc``: K_D phi into ``out`` with the library's static
        scratch (no device allocation, no wait)."""
        with self.ctx:
            _check(_lib.kfbi_apply_noalloc(self._h, _dptr(phi, "phi", self.M), _dptr(out, "out", self.M)))
        return out

    def correct(self, phi, f_gamma=None, out=None):
        if out is None:
            out = torch.empty(self.I, dtype=torch.float64, device=f"cuda:{self.ctx.device}")
        with self.ctx:
            _check(_lib.kfbi_correct(self._h, _dptr(phi, "phi", self.M), _dptr(f_gamma, "f_gamma", self.M),
                                     _dptr(out, "corr", self.I)))
        return out

    def fast_solve(self, rhs, out=None):
        if out is None:
            out = torch.empty_like(rhs)
        with self.ctx:
            _check(_lib.kfbi_fast_solve(self._h, _dptr(rhs, "rhs", self.grid_numel), _dptr(out, "v", self.grid_numel)))
        return out

    def interface_solve(self, phi, ftilde, f_gamma=None):
        dev = f"cuda:{self.ctx.device}"
        vg = torch.empty((self.n + 1, self.n + 1), dtype=torch.float64, device=dev)
        vz = torch.empty(self.M, dtype=torch.float64, device=dev)
        with self.ctx:
            _check(_lib.kfbi_interface_solve(self._h, _dptr(phi, "phi", self.M),
                                             _dptr(ftilde, "ftilde", self.grid_numel),
                                             _dptr(f_gamma, "f_gamma", self.M), _dptr(vg, "vgrid"), _dptr(vz, "vz")))
        return vg, vz

    def interface_solve_jumps(self, jq, jz, ftilde):
        dev = f"cuda:{self.ctx.device}"
        vg = torch.empty((self.n + 1, self.n + 1), dtype=torch.float64, device=dev)
        vz = torch.empty(self.M, dtype=torch.float64, device=dev)
        with self.ctx:
            _check(_lib.kfbi_interface_solve_jumps(self._h, _dptr(jq, "jq", 6 * self.Q), _dptr(jz, "jz", 6 * self.M),
                                                   _dptr(ftilde, "ftilde", self.grid_numel), _dptr(vg, "vgrid"),
                                                   _dptr(vz, "vz")))
        return vg, vz

    def solve(self, f_grid, f_gamma, g, phi0=None):
        """Dirichlet solve; returns ``(u_grid, u_gamma, phi, iters, relres, converged)``."""
        dev = f"cuda:{self.ctx.device}"
        u = torch.empty((self.n + 1, self.n + 1), dtype=torch.float64, device=dev)
        ug = torch.empty(self.M, dtype=torch.float64, device=dev)
        phi = torch.zeros(self.M, dtype=torch.float64, device=dev) if phi0 is None else phi0.clone()
        it, rel = ct.c_int(), ct.c_double()
        with self.ctx:
            st = _check(_lib.kfbi_solve(self._h, _dptr(f_grid, "f_grid", self.grid_numel),
                                        _dptr(f_gamma, "f_gamma", self.M), _dptr(g, "g", self.M), _dptr(u, "u_grid"),
                                        _dptr(ug, "u_gamma"), _dptr(phi, "phi"), ct.byref(it), ct.byref(rel)),
                        allow=(OK, NOT_CONVERGED))
        return u, ug, phi, it.value, rel.value, st == OK

    def gmres(self, rhs, phi0=None, tol=1e-10, max_iter=500, out=None):
        """GMRES on ``K_D phi = rhs``; returns ``(phi, iters, applies, relres, converged)``.
        ``out``: a device buffer holding the initial guess, overwritten with the
        iterate (no copy is made); else the guess is ``phi0`` (copied) or zero."""
        dev = f"cuda:{self.ctx.device}"
        if out is not None:
            phi = out
        else:
            phi = torch.zeros(self.M, dtype=torch.float64, device=dev) if phi0 is None else phi0.clone()
        it, ap, rel = ct.c_int(), ct.c_int(), ct.c_double()
        with self.ctx:
            st = _check(_lib.kfbi_gmres(self._h, _dptr(rhs, "rhs", self.M), _dptr(phi, "phi", self.M), float(tol),
                                        int(max_iter), ct.byref(it), ct.byref(ap), ct.byref(rel)),
                        allow=(OK, NOT_CONVERGED))
        return phi, it.value, ap.value, rel.value, st == OK

    def set_reorth(self, eta: float):
        """Threshold of the second Gram-Schmidt pass (``kfbi_prob_set_reorth``)."""
        _check(_lib.kfbi_prob_set_reorth(self._h, float(eta)))

    # ---- Table 2's other outer iterations
    def richardson(self, rhs, phi0=None, gamma=1.0, tol=1e-10, max_iter=500):
        """``x <- x + gamma (rhs - K_D x)``; returns ``(phi, iters, relres, converged)``."""
        dev = f"cuda:{self.ctx.device}"
        phi = torch.zeros(self.M, dtype=torch.float64, device=dev) if phi0 is None else phi0.clone()
        it, rel = ct.c_int(), ct.c_double()
        with self.ctx:
            st = _check(_lib.kfbi_richardson(self._h, _dptr(rhs, "rhs", self.M), _dptr(phi, "phi", self.M),
                                             float(gamma), float(tol), int(max_iter), ct.byref(it), ct.byref(rel)),
                        allow=(OK, NOT_CONVERGED))
        return phi, it.value, rel.value, st == OK

    def bicgstab(self, rhs, phi0=None, tol=1e-10, max_iter=500):
        """BiCGSTAB on ``K_D phi = rhs``; returns ``(phi, iters, applies, relres, converged)``."""
        dev = f"cuda:{self.ctx.device}"
        phi = torch.zeros(self.M, dtype=torch.float64, device=dev) if phi0 is None else phi0.clone()
        it, ap, rel = ct.c_int(), ct.c_int(), ct.c_double()
        with self.ctx:
            st = _check(_lib.kfbi_bicgstab(self._h, _dptr(rhs, "rhs", self.M), _dptr(phi, "phi", self.M),
                                           float(tol), int(max_iter), ct.byref(it), ct.byref(ap), ct.byref(rel)),
                        allow=(OK, NOT_CONVERGED))
        return phi, it.value, ap.value, rel.value, st == OK

    METHODS = {"gmres": 0, "bicgstab": 1, "richardson": 2}

    def solve_method(self, method, f_grid, f_gamma, g, phi0=None, relax=1.0):
        """Dirichlet solve with ``method`` in ``gmres``/``bicgstab``/``richardson``;
        returns ``(u_grid, u_gamma, phi, iters, relres, converged)``."""
        dev = f"cuda:{self.ctx.device}"
        u = torch.empty((self.n + 1, self.n + 1), dtype=torch.float64, device=dev)
        ug = torch.empty(self.M, dtype=torch.float64, device=dev)
        phi = torch.zeros(self.M, dtype=torch.float64, device=dev) if phi0 is None else phi0.clone()
        it, rel = ct.c_int(), ct.c_double()
        with self.ctx:
            st = _check(_lib.kfbi_solve_method(self._h, self.METHODS[method], float(relax),
                                               _dptr(f_grid, "f_grid", self.grid_numel),
                                               _dptr(f_gamma, "f_gamma", self.M), _dptr(g, "g", self.M),
                                               _dptr(u, "u_grid"), _dptr(ug, "u_gamma"), _dptr(phi, "phi"),
                                               ct.byref(it), ct.byref(rel)),
                        allow=(OK, NOT_CONVERGED))
        return u, ug, phi, it.value, rel.value, st == OK

    # ---- the Neumann problem
    def apply_neumann(self, psi: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """``K_N psi = d_n v+`` at the samples (``kfbi_apply_neumann``)."""
        if out is None:
            out = torch.empty_like(psi)
        with self.ctx:
            _check(_lib.kfbi_apply_neumann(self._h, _dptr(psi, "psi", self.M), _dptr(out, "out", self.M)))
        return out

    def interface_solve_neumann(self, psi=None, ftilde=None, f_gamma=None):
        """``[v] = 0``, ``[d_n v] = psi``, ``F = ftilde``: returns ``(v_grid, v+, d_n v+)``."""
        dev = f"cuda:{self.ctx.device}"
        vg = torch.empty((self.n + 1, self.n + 1), dtype=torch.float64, device=dev)
        vz = torch.empty(self.M, dtype=torch.float64, device=dev)
        dn = torch.empty(self.M, dtype=torch.float64, device=dev)
        with self.ctx:
            _check(_lib.kfbi_interface_solve_neumann(self._h, _dptr(psi, "psi", self.M),
                                                     _dptr(ftilde, "ftilde", self.grid_numel),
                                                     _dptr(f_gamma, "f_gamma", self.M), _dptr(vg, "vgrid"),
                                                     _dptr(vz, "vz"), _dptr(dn, "dnz")))
        return vg, vz, dn

    def gmres_neumann(self, rhs, psi0=None, tol=1e-10, max_iter=500):
        """GMRES on ``K_N psi = rhs``; returns ``(psi, iters, applies, relres, converged)``."""
        dev = f"cuda:{self.ctx.device}"
        psi = torch.zeros(self.M, dtype=torch.float64, device=dev) if psi0 is None else psi0.clone()
        it, ap, rel = ct.c_int(), ct.c_int(), ct.c_double()
        with self.ctx:
            st = _check(_lib.kfbi_gmres_neumann(self._h, _dptr(rhs, "rhs", self.M), _dptr(psi, "psi", self.M),
                                                float(tol), int(max_iter), ct.byref(it), ct.byref(ap),
                                                ct.byref(rel)),
                        allow=(OK, NOT_CONVERGED))
        return psi, it.value, ap.value, rel.value, st == OK

    def solve_neumann(self, f_grid, f_gamma, g_n, psi0=None):
        """Neumann solve; returns ``(u_grid, u_gamma, dn_gamma, psi, iters, relres, converged)``."""
        dev = f"cuda:{self.ctx.device}"
        u = torch.empty((self.n + 1, self.n + 1), dtype=torch.float64, device=dev)
        ug = torch.empty(self.M, dtype=torch.float64, device=dev)
        dn = torch.empty(self.M, dtype=torch.float64, device=dev)
        psi = torch.zeros(self.M, dtype=torch.float64, device=dev) if psi0 is None else psi0.clone()
        it, rel = ct.c_int(), ct.c_double()
        with self.ctx:
            st = _check(_lib.kfbi_solve_neumann(self._h, _dptr(f_grid, "f_grid", self.grid_numel),
                                                _dptr(f_gamma, "f_gamma", self.M), _dptr(g_n, "g_n", self.M),
                                                _dptr(u, "u_grid"), _dptr(ug, "u_gamma"), _dptr(dn, "dn_gamma"),
                                                _dptr(psi, "psi"), ct.byref(it), ct.byref(rel)),
                        allow=(OK, NOT_CONVERGED))
        return u, ug, dn, psi, it.value, rel.value, st == OK

    # ---- launch shapes
    def autotune(self, reps: int = 10) -> dict:
        """Time the candidate shapes on this problem and keep the fastest (``kfbi_prob_autotune``)."""
        t = Tiles()
        _check(_lib.kfbi_prob_autotune(self._h, int(reps), ct.byref(t)))
        return t.as_dict()

    def tiles(self) -> dict:
        t = Tiles()
        _check(_lib.kfbi_prob_get_tiles(self._h, ct.byref(t)))
        return t.as_dict()

    def set_tiles(self, modes_per_group: int, dst_cols: int):
        t = Tiles(int(modes_per_group), 0, int(dst_cols), 0.0, 0.0)
        _check(_lib.kfbi_prob_set_tiles(self._h, ct.byref(t)))

    # ---- timing of the three apply stages (HIP events on the context stream)
    def set_timing(self, on: bool):
        _check(_lib.kfbi_set_timing(self._h, 1 if on else 0))

    def apply_timing(self):
        a, b, c, n = ct.c_double(), ct.c_double(), ct.c_double(), ct.c_int()
        _check(_lib.kfbi_apply_timing(self._h, ct.byref(a), ct.byref(b), ct.byref(c), ct.byref(n)))
        return {"correct_us": a.value, "modes_us": b.value, "interp_us": c.value, "count": n.value}


class Problem3:
    """The ellipsoid problem on an ``n^3``-interval grid (``kfbi3_*``).

    The control points (the unknowns of the boundary equation) are the
    grid-edge / surface crossings; ``points()`` gives them, so that ``g`` and
    ``f`` on the surface can be sampled there.  3D grid arrays are indexed
    ``[k, j, i]`` with shape ``(n+1, n+1, n+1)``.
    """

    def __init__(self, ctx: Context, n: int, axes=(0.9, 0.7, 0.5), kappa: float = 0.0, lo: float = -1.2,
                 hi: float = 1.2, tol: float = 1e-10, restart: int = 50, max_iter: int = 500):
        self.ctx = ctx
        d = _Desc3(int(n), float(lo), float(hi), float(kappa), (ct.c_double * 3)(*[float(a) for a in axes]),
                   float(tol), int(restart), int(max_iter))
        h = _vp()
        _check(_lib.kfbi3_prob_create(ctx._h, ct.byref(d), ct.byref(h)))
        self._h = h
        self.n, self.kappa, self.lo, self.hi, self.axes = int(n), float(kappa), lo, hi, tuple(axes)
        m, ni, nb = ct.c_int(), ct.c_int(), ct.c_size_t()
        _check(_lib.kfbi3_prob_info(h, ct.byref(m), ct.byref(ni), ct.byref(nb)))
        self.M, self.I, self.device_bytes = m.value, ni.value, nb.value

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.kfbi3_prob_destroy(self._h)
        self._h = None

    def __del__(self):
        self.close()

    @property
    def grid_numel(self):
        return (self.n + 1) ** 3

    def points(self):
        """``(pts, axis)``: control point coordinates (M, 3) and the axis of each one's grid edge."""
        pts = np.zeros((self.M, 3))
        axis = np.zeros(self.M, dtype=np.int32)
        _check(_lib.kfbi3_prob_points(self._h, _vp(pts.ctypes.data), _vp(axis.ctypes.data)))
        return pts, axis

    def mask(self) -> np.ndarray:
        out = np.zeros((self.n + 1,) * 3, dtype=np.uint8)
        _check(_lib.kfbi3_prob_mask(self._h, _vp(out.ctypes.data)))
        return out.astype(bool)

    def irregular(self) -> np.ndarray:
        """Irregular nodes as ``(i, j, k)`` rows."""
        node = np.zeros(self.I, dtype=np.int32)
        _check(_lib.kfbi3_prob_irregular(self._h, _vp(node.ctypes.data)))
        n = self.n
        return np.stack([node % n + 1, (node // n) % n + 1, node // (n * n) + 1], axis=1)

    def jumps(self, phi, f_gamma=None):
        """Cartesian jumps, shape (10, M): [v], gradient, Hessian (xx, yy, zz, xy, xz, yz)."""
        J = torch.empty((10, self.M), dtype=torch.float64, device=f"cuda:{self.ctx.device}")
        with self.ctx:
            _check(_lib.kfbi3_jumps(self._h, _dptr(phi, "phi", self.M), _dptr(f_gamma, "f_gamma", self.M),
                                    _dptr(J, "J")))
        return J

    def apply(self, phi, out=None):
        if out is None:
            out = torch.empty_like(phi)
        with self.ctx:
            _check(_lib.kfbi3_apply(self._h, _dptr(phi, "phi", self.M), _dptr(out, "out", self.M)))
        return out

    def interface_solve(self, phi=None, f_grid=None, f_gamma=None):
        dev = f"cuda:{self.ctx.device}"
        vg = torch.empty((self.n + 1,) * 3, dtype=torch.float64, device=dev)
        vz = torch.empty(self.M, dtype=torch.float64, device=dev)
        with self.ctx:
            _check(_lib.kfbi3_interface_solve(self._h, _dptr(phi, "phi", self.M),
                                              _dptr(f_grid, "f_grid", self.grid_numel),
                                              _dptr(f_gamma, "f_gamma", self.M), _dptr(vg, "vgrid"), _dptr(vz, "vz")))
        return vg, vz

    def solve(self, f_grid, f_gamma, g, phi0=None):
        """Dirichlet solve; returns ``(u_grid, u_gamma, phi, iters, relres, converged)``."""
        dev = f"cuda:{self.ctx.device}"
        u = torch.empty((self.n + 1,) * 3, dtype=torch.float64, device=dev)
        ug = torch.empty(self.M, dtype=torch.float64, device=dev)
        phi = torch.zeros(self.M, dtype=torch.float64, device=dev) if phi0 is None else phi0.clone()
        it, rel = ct.c_int(), ct.c_double()
        with self.ctx:
            st = _check(_lib.kfbi3_solve(self._h, _dptr(f_grid, "f_grid", self.grid_numel),
                                         _dptr(f_gamma, "f_gamma", self.M), _dptr(g, "g", self.M),
                                         _dptr(u, "u_grid"), _dptr(ug, "u_gamma"), _dptr(phi, "phi"),
                                         ct.byref(it), ct.byref(rel)),
                        allow=(OK, NOT_CONVERGED))
        return u, ug, phi, it.value, rel.value, st == OK

    def gmres(self, rhs, phi0=None, tol=1e-10, max_iter=500):
        """GMRES on ``K_D phi = rhs``; returns ``(phi, iters, applies, relres, converged)``."""
        dev = f"cuda:{self.ctx.device}"
        phi = torch.zeros(self.M, dtype=torch.float64, device=dev) if phi0 is None else phi0.clone()
        it, ap, rel = ct.c_int(), ct.c_int(), ct.c_double()
        with self.ctx:
            st = _check(_lib.kfbi3_gmres(self._h, _dptr(rhs, "rhs", self.M), _dptr(phi, "phi", self.M), float(tol),
                                         int(max_iter), ct.byref(it), ct.byref(ap), ct.byref(rel)),
                        allow=(OK, NOT_CONVERGED))
        return phi, it.value, ap.value, rel.value, st == OK


class GrayScott:
    """Gray-Scott time stepping on a curved domain with zero Neumann data
    (``kfbi_gs_*``): the state lives on the device; ``step`` advances it by
    Strang splitting, two Neumann solves per step."""

    def __init__(self, ctx: Context, xy, n: int, dt: float, gamma=0.024, kill=0.06, eps0=0.01, eps1=0.008,
                 eps2=0.004, lo: float = -2.0, hi: float = 2.0, tol: float = 1e-8, restart: int = 50,
                 max_iter: int = 500):
        self.ctx = ctx
        xy = np.ascontiguousarray(xy, dtype=np.float64)
        d = _GsDesc(lo, hi, int(n), xy.shape[0], _vp(xy.ctypes.data), gamma, kill, eps0, eps1, eps2, dt, tol,
                    restart, max_iter)
        h = _vp()
        with ctx:
            _check(_lib.kfbi_gs_create(ctx._h, ct.byref(d), ct.byref(h)))
        self._h = h
        self.n = int(n)
        self.lo, self.hi = lo, hi
        m = ct.c_int()
        _check(_lib.kfbi_gs_info(self._h, ct.byref(m), None, None))
        self.M = m.value

    def close(self):
        if getattr(self, "_h", None):
            _lib.kfbi_gs_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def info(self):
        m, st, it = ct.c_int(), ct.c_int(), ct.c_longlong()
        _check(_lib.kfbi_gs_info(self._h, ct.byref(m), ct.byref(st), ct.byref(it)))
        return {"samples": m.value, "steps": st.value, "gmres_iters": it.value}

    def set_state(self, u_grid, v_grid, u_gamma, v_gamma):
        g = (self.n + 1) ** 2
        with self.ctx:
            _check(_lib.kfbi_gs_set_state(self._h, _dptr(u_grid, "u_grid", g), _dptr(v_grid, "v_grid", g),
                                          _dptr(u_gamma, "u_gamma", self.M), _dptr(v_gamma, "v_gamma", self.M)))

    def state(self):
        """``(u_grid, v_grid, u_gamma, v_gamma)`` as new device tensors."""
        dev = f"cuda:{self.ctx.device}"
        out = [torch.empty((self.n + 1, self.n + 1), dtype=torch.float64, device=dev) for _ in range(2)]
        out += [torch.empty(self.M, dtype=torch.float64, device=dev) for _ in range(2)]
        with self.ctx:
            _check(_lib.kfbi_gs_get_state(self._h, *[_dptr(t, "state") for t in out]))
        return tuple(out)

    def step(self, nsteps: int = 1):
        with self.ctx:
            _check(_lib.kfbi_gs_step(self._h, int(nsteps)))


class Batch:
    """Many problems advancing through one launch per GMRES stage (``kfbi_batch_*``).

    ``admit`` starts a problem (volume potential + GMRES state), ``step`` runs
    iterations of every live problem, ``poll`` reports convergence per slot and
    ``finish`` computes the final solution and frees the slot.  The tensors
    passed to ``admit`` are kept alive until ``finish``.
    """

    def __init__(self, ctx: Context, max_slots: int = 32, m_max: int = 8192, hbm_budget: int = 0):
        self.ctx = ctx
        self.max_slots = int(max_slots)
        h = _vp()
        _check(_lib.kfbi_batch_create(ctx._h, self.max_slots, int(m_max), int(hbm_budget), ct.byref(h)))
        self._h = h
        self._held = {}

    def close(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.kfbi_batch_destroy(self._h)
        self._h = None

    def __del__(self):
        self.close()

    @staticmethod
    def estimate_bytes(n: int, m: int, restart: int = 50) -> int:
        out = ct.c_size_t()
        _check(_lib.kfbi_batch_estimate_bytes(int(n), int(m), int(restart), ct.byref(out)))
        return out.value

    def admit(self, prob: Problem, f_grid, f_gamma, g):
        """Returns the slot id, or None when no slot or memory is free right now."""
        slot = ct.c_int(-1)
        with self.ctx:
            st = _check(_lib.kfbi_batch_admit(self._h, prob._h, _dptr(f_grid, "f_grid", prob.grid_numel),
                                              _dptr(f_gamma, "f_gamma", prob.M), _dptr(g, "g", prob.M),
                                              ct.byref(slot)), allow=(OK, ERR_BUDGET))
        if st == ERR_BUDGET:
            return None
        self._held[slot.value] = (prob, f_grid, f_gamma, g)
        return slot.value

    def step(self, nsteps: int):
        with self.ctx:
            _check(_lib.kfbi_batch_step(self._h, int(nsteps)))

    def poll(self):
        """``(state, iters, relres)`` per slot: state 1 converged, -1 cap, 0 running, -2 empty,
        -3 stopped on a NaN or Inf in the request's data."""
        state = np.zeros(self.max_slots, dtype=np.int32)
        iters = np.zeros(self.max_slots, dtype=np.int32)
        rel = np.zeros(self.max_slots)
        _check(_lib.kfbi_batch_poll(self._h, _vp(state.ctypes.data), _vp(iters.ctypes.data), _vp(rel.ctypes.data)))
        return state, iters, rel

    def finish(self, slot: int):
        """Final solve of a slot; returns ``(u_grid, u_gamma, phi, prob)`` and frees the slot."""
        prob = self._held[slot][0]
        dev = f"cuda:{self.ctx.device}"
        u = torch.empty((prob.n + 1, prob.n + 1), dtype=torch.float64, device=dev)
        ug = torch.empty(prob.M, dtype=torch.float64, device=dev)
        phi = torch.empty(prob.M, dtype=torch.float64, device=dev)
        with self.ctx:
            st = _lib.kfbi_batch_finish(self._h, int(slot), _dptr(u, "u_grid"), _dptr(ug, "u_gamma"),
                                        _dptr(phi, "phi"))
        if st in (OK, ERR_NONFINITE):            # the slot is released either way
            del self._held[slot]
        _check(st)
        return u, ug, phi, prob

    def info(self):
        live, nb = ct.c_int(), ct.c_size_t()
        _check(_lib.kfbi_batch_info(self._h, ct.byref(live), ct.byref(nb)))
        return live.value, nb.value
