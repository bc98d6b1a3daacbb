"""Python binding of libwwbi (ctypes).  Argument marshalling only: every step of
the solve runs in the HIP library; torch supplies device memory and the stream.

The library must be built first (``python -m paper_2108_01786_amd.build``);
importing this module on a machine without the built library raises.
"""
from __future__ import annotations

import ctypes as C
import os
import warnings
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwwbi.so")

# status codes and option values (mirror include/wwbi.h)
OK, EINVAL_NULL, EINVAL_SIZE, EINVAL_NONFINITE, EINVAL_ORIENTATION = 0, -1, -2, -3, -4
ECAPACITY, EHIP, EINVAL_OPTS, EINVAL_RANGE, ESCRATCH = -5, -6, -7, -8, -9
NOT_CONVERGED, STAGNATED, REFINE_STALLED, WARN_UNDERRESOLVED = 1, 2, 3, 4
FP64, FP32_REFINED = 0, 1
SURF_GRAPH, SURF_HLS = 0, 1
MATVEC_AUTO, MATVEC_STORED, MATVEC_ON_THE_FLY = 0, 1, 2
FLAG_PROFILE, FLAG_NO_CORRECTION, FLAG_NO_RECYCLE = 1, 2, 4
OP_D, OP_D2, OP_H, OP_ABSD = 0, 1, 2, 3
MAT_A, MAT_WALL, MAT_T = 0, 1, 2


class _Geom(C.Structure):
    _fields_ = [("nb", C.c_int32), ("M", C.POINTER(C.c_int32)),
                ("x", C.c_void_p), ("y", C.c_void_p), ("dx", C.c_void_p), ("dy", C.c_void_p),
                ("ddx", C.c_void_p), ("ddy", C.c_void_p),
                ("zc", C.POINTER(C.c_double)), ("a", C.POINTER(C.c_double)),
                ("V1", C.c_double), ("psi_wall", C.c_void_p)]


class _Opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("inner_tol", C.c_double), ("restart", C.c_int32),
                ("max_iter", C.c_int32), ("precision", C.c_int32), ("matvec", C.c_int32),
                ("poll_every", C.c_int32), ("max_refine", C.c_int32), ("band", C.c_int32),
                ("flags", C.c_int32), ("x0", C.c_void_p)]


class Report(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("restarts", C.c_int32),
                ("refine_steps", C.c_int32), ("rel_resid", C.c_double),
                ("ms_prep", C.c_double), ("ms_assemble", C.c_double), ("ms_solve", C.c_double),
                ("ms_U", C.c_double), ("ms_total", C.c_double), ("n_matvec", C.c_int32),
                ("pad0", C.c_int32), ("ms_matvec", C.c_double), ("bytes_matvec", C.c_double),
                ("tail_ratio", C.c_double), ("n_hist", C.c_int32), ("pad1", C.c_int32),
                ("resid_hist", C.c_double * 32)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_
             if k not in ("pad0", "pad1", "resid_hist")}
        d["resid_hist"] = self.history()
        return d

    def history(self):
        """The relative residuals the solve measured (cycle starts of an FP64
        solve, refinement steps of a refined one), in order."""
        return [self.resid_hist[i] for i in range(max(0, min(self.n_hist, 32)))]


_SIGS = {
    "wwbi_default_opts": (None, [C.POINTER(_Opts)]),
    "wwbi_status_str": (C.c_char_p, [C.c_int]),
    "wwbi_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int32, C.c_void_p]),
    "wwbi_set_stream": (C.c_int, [C.c_void_p, C.c_void_p]),
    "wwbi_destroy": (C.c_int, [C.c_void_p]),
    "wwbi_reserve": (C.c_int, [C.c_void_p, C.c_int64, C.c_int32, C.c_int32]),
    "wwbi_solve_phi": (C.c_int, [C.c_void_p, C.POINTER(_Geom), C.c_void_p, C.POINTER(_Opts),
                                 C.c_void_p, C.c_void_p, C.POINTER(C.c_double),
                                 C.POINTER(Report)]),
    "wwbi_solve_phi_noalloc": (C.c_int, [C.c_void_p, C.POINTER(_Geom), C.c_void_p,
                                         C.POINTER(_Opts), C.c_void_p, C.c_void_p,
                                         C.POINTER(C.c_double), C.POINTER(Report)]),
    "wwbi_solve_gamma": (C.c_int, [C.c_void_p, C.POINTER(_Geom), C.c_void_p, C.POINTER(_Opts),
                                   C.c_void_p, C.c_void_p, C.POINTER(Report)]),
    "wwbi_tangential_energy": (C.c_int, [C.c_void_p, C.POINTER(_Geom), C.c_void_p, C.c_void_p,
                                         C.c_double, C.c_double, C.c_void_p,
                                         C.POINTER(C.c_double), C.POINTER(Report)]),
    "wwbi_solve_gamma_t": (C.c_int, [C.c_void_p, C.POINTER(_Geom), C.c_void_p, C.c_void_p,
                                     C.c_double, C.c_double, C.POINTER(_Opts), C.c_void_p,
                                     C.c_void_p, C.POINTER(Report), C.POINTER(Report)]),
    "wwbi_stage_rhs": (C.c_int, [C.c_void_p, C.POINTER(_Geom), C.c_int32, C.c_void_p, C.c_void_p,
                                 C.c_double, C.c_double, C.POINTER(_Opts), C.c_void_p,
                                 C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(Report)]),
    "wwbi_rk_step": (C.c_int, [C.c_void_p, C.POINTER(_Geom), C.c_int32, C.c_int32,
                               C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_double,
                               C.c_void_p, C.c_void_p, C.c_double, C.c_double, C.c_int32,
                               C.POINTER(_Opts), C.POINTER(Report)]),
    "wwbi_boundary_velocity": (C.c_int, [C.c_void_p, C.POINTER(_Geom), C.c_void_p, C.c_void_p,
                                         C.c_void_p]),
    "wwbi_interior_eval": (C.c_int, [C.c_void_p, C.POINTER(_Geom), C.c_void_p, C.c_void_p,
                                     C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_void_p]),
    "wwbi_interior_velocity": (C.c_int, [C.c_void_p, C.POINTER(_Geom), C.c_void_p, C.c_int32,
                                         C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "wwbi_pressure": (C.c_int, [C.c_void_p, C.POINTER(_Geom), C.c_void_p, C.c_double, C.c_double,
                                C.POINTER(_Opts), C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p,
                                C.POINTER(Report)]),
    "wwbi_adjoint_phi": (C.c_int, [C.c_void_p, C.POINTER(_Geom), C.c_void_p, C.c_void_p,
                                   C.POINTER(_Opts)] + [C.c_void_p] * 7 + [C.POINTER(Report)]),
    "wwbi_solve_phi_multi": (C.c_int, [C.c_void_p, C.POINTER(_Geom), C.c_void_p, C.c_int32,
                                       C.POINTER(_Opts), C.c_void_p, C.POINTER(Report)]),
    "wwbi_tangent_phi": (C.c_int, [C.c_void_p, C.POINTER(_Geom), C.c_void_p, C.c_int32,
                                   C.c_void_p, C.POINTER(_Opts), C.c_void_p, C.c_void_p,
                                   C.POINTER(Report)]),
    "wwbi_spectral": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int32, C.c_double,
                                C.c_double, C.c_void_p]),
    "wwbi_surface_fill": (C.c_int, [C.c_void_p, C.c_int32] + [C.c_void_p] * 8),
    "wwbi_surface_fill_adjoint": (C.c_int, [C.c_void_p, C.c_int32] + [C.c_void_p] * 8),
    "wwbi_debug_matrix": (C.c_int, [C.c_void_p, C.POINTER(_Geom), C.c_int32, C.c_int32,
                                    C.c_int32, C.c_void_p]),
    "wwbi_matvec": (C.c_int, [C.c_void_p, C.POINTER(_Geom), C.c_void_p, C.c_void_p, C.c_int32,
                              C.c_int32, C.c_int32, C.c_int32, C.POINTER(Report)]),
}

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libwwbi.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: build it with "
                               "`python -m paper_2108_01786_amd.build`")
        lib = C.CDLL(path)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name, None)
            if fn is None:
                continue
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class WWBIError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = load_library().wwbi_status_str(status).decode()
        super().__init__(f"{where}: {msg} ({status})")


def status_str(status: int) -> str:
    return load_library().wwbi_status_str(status).decode()


def _check(rc: int, check: bool, name: str):
    """Raise for an error (rc < 0), and with check for a numerical warning;
    an under-resolved grid (WARN_UNDERRESOLVED) only emits a RuntimeWarning,
    as the solve itself succeeded."""
    if rc == WARN_UNDERRESOLVED:
        if check:
            warnings.warn(f"{name}: omega is not resolved by the grid (Fourier tail above "
                          "max(1e-12, 10 tol))", RuntimeWarning, stacklevel=3)
        return
    if rc < 0 or (check and rc != OK):
        raise WWBIError(rc, name)


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return C.c_void_p(t.data_ptr())


def _f64(t: torch.Tensor, device) -> torch.Tensor:
    t = torch.as_tensor(t, dtype=torch.float64, device=device)
    return t.contiguous()


class DeviceGeometry:
    """Boundary samples on the device, concatenated boundary by boundary
    (surface, bottom, obstacles), plus the multi-valued flow data."""

    def __init__(self, M: Sequence[int], x, y, dx, dy, ddx, ddy, zc, a, V1: float,
                 psi_wall=None, device="cuda"):
        self.M = [int(m) for m in M]
        dev = torch.device(device)
        self.x, self.y = _f64(x, dev), _f64(y, dev)
        self.dx, self.dy = _f64(dx, dev), _f64(dy, dev)
        self.ddx, self.ddy = _f64(ddx, dev), _f64(ddy, dev)
        zc = np.asarray(zc, dtype=np.complex128).reshape(-1)
        self.zc = np.ascontiguousarray(np.stack([zc.real, zc.imag], 1).reshape(-1), dtype=np.float64)
        self.a = np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(-1))
        self.V1 = float(V1)
        self.psi_wall = None if psi_wall is None else _f64(psi_wall, dev)
        self._M = (C.c_int32 * len(self.M))(*self.M)

    @classmethod
    def from_synth(cls, geom, device="cuda") -> "DeviceGeometry":
        arr = geom.arrays()
        return cls(geom.M, arr["x"], arr["y"], arr["dx"], arr["dy"], arr["ddx"], arr["ddy"],
                   geom.zc, geom.a, geom.V1, geom.psi_wall, device)

    @property
    def n(self) -> int:
        return sum(self.M)

    @property
    def nb(self) -> int:
        return len(self.M)

    def _fields(self):
        return (self.x, self.y, self.dx, self.dy, self.ddx, self.ddy, self.psi_wall, self.zc,
                self.a)

    def _key(self):
        # the cache holds the field objects, so equal ids mean the same objects
        return (tuple(self.M), self.V1) + tuple(map(id, self._fields()))

    def c_struct(self) -> _Geom:
        """The C view of the geometry; rebuilt only when a field was replaced
        (building it costs tens of microseconds of Python per call)."""
        key = self._key()
        if getattr(self, "_cache", None) is not None and self._cache[0] == key:
            return self._cache[1]
        if tuple(self.M) != tuple(self._M):
            self._M = (C.c_int32 * len(self.M))(*self.M)
        g = _Geom()
        g.nb = len(self.M)
        g.M = C.cast(self._M, C.POINTER(C.c_int32))
        g.x, g.y, g.dx, g.dy = _ptr(self.x), _ptr(self.y), _ptr(self.dx), _ptr(self.dy)
        g.ddx, g.ddy = _ptr(self.ddx), _ptr(self.ddy)
        g.zc = self.zc.ctypes.data_as(C.POINTER(C.c_double))
        g.a = self.a.ctypes.data_as(C.POINTER(C.c_double))
        g.V1 = self.V1
        g.psi_wall = _ptr(self.psi_wall)
        self._cache = (key, g, self._fields())
        return g


def make_opts(tol=1e-13, inner_tol=1e-7, restart=100, max_iter=2000, precision=FP64,
              matvec=MATVEC_AUTO, poll_every=2, max_refine=8, band=16, flags=0,
              x0: Optional[torch.Tensor] = None) -> _Opts:
    o = _Opts()
    load_library().wwbi_default_opts(C.byref(o))
    o.tol, o.inner_tol, o.restart, o.max_iter = tol, inner_tol, restart, max_iter
    o.precision, o.matvec, o.poll_every, o.max_refine = precision, matvec, poll_every, max_refine
    o.band, o.flags = band, flags
    o.x0 = _ptr(x0)
    return o


class Context:
    """A libwwbi context on one device; every call runs on torch's current stream."""

    def __init__(self, device: int = 0):
        self.lib = load_library()
        self.device = device
        h = C.c_void_p()
        with torch.cuda.device(device):
            rc = self.lib.wwbi_create(C.byref(h), device, C.c_void_p(torch.cuda.current_stream().cuda_stream))
        if rc != OK:
            raise WWBIError(rc, "wwbi_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.wwbi_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _stream(self):
        self.lib.wwbi_set_stream(self.h, C.c_void_p(torch.cuda.current_stream().cuda_stream))

    def _dev(self):
        return torch.device("cuda", self.device)

    def reserve(self, max_unknowns: int, max_restart: int = 100, precision: int = -1):
        rc = self.lib.wwbi_reserve(self.h, max_unknowns, max_restart, precision)
        if rc != OK:
            raise WWBIError(rc, "wwbi_reserve")

    def solve_phi(self, geom: DeviceGeometry, phi: torch.Tensor, check: bool = True,
                  want_omega: bool = True, U: Optional[torch.Tensor] = None,
                  omega: Optional[torch.Tensor] = None, **kw):
        self._stream()
        dev = self._dev()
        phi = _f64(phi, dev)
        if U is None:
            U = torch.empty(geom.M[0], dtype=torch.float64, device=dev)
        if omega is None and want_omega:
            omega = torch.empty(geom.n, dtype=torch.float64, device=dev)
        psi = (C.c_double * max(1, geom.nb - 2))()
        rep = Report()
        g = geom.c_struct()
        o = make_opts(**kw)
        rc = self.lib.wwbi_solve_phi(self.h, C.byref(g), _ptr(phi), C.byref(o), _ptr(U),
                                     _ptr(omega), psi, C.byref(rep))
        _check(rc, check, "wwbi_solve_phi")
        psi_k = np.array(psi[: max(0, geom.nb - 2)], dtype=np.float64)
        return U, omega, psi_k, rep

    def solve_phi_noalloc(self, geom: DeviceGeometry, phi: torch.Tensor, check: bool = True,
                          U: Optional[torch.Tensor] = None, omega: Optional[torch.Tensor] = None,
                          **kw):
        """wwbi_solve_phi_noalloc: the on-the-fly solve with its workspace in the
        library's static scratch array (no device allocation inside the call).
        U and omega may be passed in; they are allocated here otherwise."""
        self._stream()
        dev = self._dev()
        phi = _f64(phi, dev)
        if U is None:
            U = torch.empty(geom.M[0], dtype=torch.float64, device=dev)
        if omega is None:
            omega = torch.empty(geom.n, dtype=torch.float64, device=dev)
        psi = (C.c_double * max(1, geom.nb - 2))()
        rep = Report()
        g = geom.c_struct()
        kw.setdefault("matvec", MATVEC_ON_THE_FLY)
        o = make_opts(**kw)
        rc = self.lib.wwbi_solve_phi_noalloc(self.h, C.byref(g), _ptr(phi), C.byref(o), _ptr(U),
                                             _ptr(omega), psi, C.byref(rep))
        _check(rc, check, "wwbi_solve_phi_noalloc")
        psi_k = np.array(psi[: max(0, geom.nb - 2)], dtype=np.float64)
        return U, omega, psi_k, rep

    def solve_gamma(self, geom: DeviceGeometry, gamma0: torch.Tensor, check: bool = True, **kw):
        self._stream()
        dev = self._dev()
        gamma0 = _f64(gamma0, dev)
        U = torch.empty(geom.M[0], dtype=torch.float64, device=dev)
        gw = torch.empty(geom.n - geom.M[0], dtype=torch.float64, device=dev)
        rep = Report()
        g = geom.c_struct()
        o = make_opts(**kw)
        rc = self.lib.wwbi_solve_gamma(self.h, C.byref(g), _ptr(gamma0), C.byref(o), _ptr(U),
                                       _ptr(gw), C.byref(rep))
        _check(rc, check, "wwbi_solve_gamma")
        return U, gw, rep

    def tangential_energy(self, geom: DeviceGeometry, omega: torch.Tensor,
                          phi: Optional[torch.Tensor] = None, tau: float = 0.0, grav: float = 1.0,
                          want_dphids: bool = True, want_energy: bool = True):
        """dphi/ds on every node (device, sum(M)) and the energy E (float), from
        the densities omega of a velocity-potential solve; either may be None."""
        self._stream()
        dev = self._dev()
        omega = _f64(omega, dev)
        phi = _f64(phi, dev) if phi is not None else None
        dphids = torch.empty(geom.n, dtype=torch.float64, device=dev) if want_dphids else None
        E = C.c_double(0.0)
        rep = Report()
        g = geom.c_struct()
        rc = self.lib.wwbi_tangential_energy(self.h, C.byref(g), _ptr(phi), _ptr(omega), tau, grav,
                                             _ptr(dphids), C.byref(E) if want_energy else None,
                                             C.byref(rep))
        if rc != OK:
            raise WWBIError(rc, "wwbi_tangential_energy")
        return dphids, (E.value if want_energy else None), rep

    def solve_gamma_t(self, geom: DeviceGeometry, phi: torch.Tensor, V: torch.Tensor,
                      tau: float = 0.0, grav: float = 1.0, check: bool = True, **kw):
        """gamma_t (device, sum(M)) of the Sec. 4.2 system at the state (geometry, phi~)
        with surface tangential velocity V; also U and both reports."""
        self._stream()
        dev = self._dev()
        phi, V = _f64(phi, dev), _f64(V, dev)
        gt = torch.empty(geom.n, dtype=torch.float64, device=dev)
        U = torch.empty(geom.M[0], dtype=torch.float64, device=dev)
        r1, r2 = Report(), Report()
        g = geom.c_struct()
        o = make_opts(**kw)
        rc = self.lib.wwbi_solve_gamma_t(self.h, C.byref(g), _ptr(phi), _ptr(V), tau, grav,
                                         C.byref(o), _ptr(gt), _ptr(U), C.byref(r1), C.byref(r2))
        _check(rc, check, "wwbi_solve_gamma_t")
        return gt, U, r1, r2

    def stage_rhs(self, geom: DeviceGeometry, mode: int, q: torch.Tensor, phi: torch.Tensor,
                  tau: float = 0.0, grav: float = 1.0, check: bool = True, **kw):
        """(q_t, phi_t, U, V, report) of one evolution stage; the stage's surface
        is written into the first M_0 entries of the geometry arrays."""
        self._stream()
        dev = self._dev()
        q, phi = _f64(q, dev), _f64(phi, dev)
        out = [torch.empty(geom.M[0], dtype=torch.float64, device=dev) for _ in range(4)]
        rep = Report()
        g = geom.c_struct()
        o = make_opts(**kw)
        rc = self.lib.wwbi_stage_rhs(self.h, C.byref(g), mode, _ptr(q), _ptr(phi), tau, grav,
                                     C.byref(o), *[_ptr(t) for t in out], C.byref(rep))
        _check(rc, check, "wwbi_stage_rhs")
        return out[0], out[1], out[2], out[3], rep

    def rk_step(self, geom: DeviceGeometry, mode: int, A, b, h: float, q: torch.Tensor,
                phi: torch.Tensor, tau: float = 0.0, grav: float = 1.0, filt: bool = True,
                check: bool = True, **kw):
        """One explicit Runge-Kutta step with tableau (A, b); q and phi (device,
        contiguous FP64) are updated in place.  Returns the report."""
        self._stream()
        A = np.ascontiguousarray(np.asarray(A, dtype=np.float64))
        b = np.ascontiguousarray(np.asarray(b, dtype=np.float64))
        ns = int(b.shape[0])
        if A.shape != (ns, ns):
            raise ValueError("A must be nstage x nstage")
        for t in (q, phi):
            if t.dtype != torch.float64 or not t.is_contiguous() or not t.is_cuda:
                raise ValueError("q and phi must be contiguous FP64 device tensors")
        rep = Report()
        g = geom.c_struct()
        o = make_opts(**kw)
        Ac = A.ctypes.data_as(C.POINTER(C.c_double))
        bc = b.ctypes.data_as(C.POINTER(C.c_double))
        rc = self.lib.wwbi_rk_step(self.h, C.byref(g), mode, ns, Ac, bc, h, _ptr(q), _ptr(phi),
                                   tau, grav, 1 if filt else 0, C.byref(o), C.byref(rep))
        _check(rc, check, "wwbi_rk_step")
        return rep

    def boundary_velocity(self, geom: DeviceGeometry, omega: torch.Tensor):
        """(u, v) on every boundary node (device, sum(M) each)."""
        self._stream()
        dev = self._dev()
        omega = _f64(omega, dev)
        u = torch.empty(geom.n, dtype=torch.float64, device=dev)
        v = torch.empty_like(u)
        g = geom.c_struct()
        rc = self.lib.wwbi_boundary_velocity(self.h, C.byref(g), _ptr(omega), _ptr(u), _ptr(v))
        if rc != OK:
            raise WWBIError(rc, "wwbi_boundary_velocity")
        return u, v

    def interior_eval(self, geom: DeviceGeometry, f: torch.Tensor, z: torch.Tensor):
        """f (complex, sum(M)) on the boundary nodes -> f at the complex points z."""
        self._stream()
        dev = self._dev()
        fr, fi = _f64(f.real, dev), _f64(f.imag, dev)
        zx, zy = _f64(z.real, dev), _f64(z.imag, dev)
        outr, outi = torch.empty_like(zx), torch.empty_like(zx)
        g = geom.c_struct()
        rc = self.lib.wwbi_interior_eval(self.h, C.byref(g), _ptr(fr), _ptr(fi), int(zx.numel()),
                                         _ptr(zx), _ptr(zy), _ptr(outr), _ptr(outi))
        if rc != OK:
            raise WWBIError(rc, "wwbi_interior_eval")
        return torch.complex(outr, outi)

    def interior_velocity(self, geom: DeviceGeometry, omega: torch.Tensor, z: torch.Tensor):
        """(u, v) at the complex points z inside the fluid."""
        self._stream()
        dev = self._dev()
        omega = _f64(omega, dev)
        zx, zy = _f64(z.real, dev), _f64(z.imag, dev)
        u, v = torch.empty_like(zx), torch.empty_like(zx)
        g = geom.c_struct()
        rc = self.lib.wwbi_interior_velocity(self.h, C.byref(g), _ptr(omega), int(zx.numel()),
                                             _ptr(zx), _ptr(zy), _ptr(u), _ptr(v))
        if rc != OK:
            raise WWBIError(rc, "wwbi_interior_velocity")
        return u, v

    def pressure(self, geom: DeviceGeometry, phi: torch.Tensor, z: torch.Tensor, tau: float = 0.0,
                 grav: float = 1.0, check: bool = True, **kw):
        """p / rho at the complex points z inside the fluid, and the report."""
        self._stream()
        dev = self._dev()
        phi = _f64(phi, dev)
        zx, zy = _f64(z.real, dev), _f64(z.imag, dev)
        p = torch.empty_like(zx)
        rep = Report()
        g = geom.c_struct()
        o = make_opts(**kw)
        rc = self.lib.wwbi_pressure(self.h, C.byref(g), _ptr(phi), tau, grav, C.byref(o),
                                    int(zx.numel()), _ptr(zx), _ptr(zy), _ptr(p), C.byref(rep))
        _check(rc, check, "wwbi_pressure")
        return p, rep

    def adjoint_phi(self, geom: DeviceGeometry, omega: torch.Tensor, dJdU: torch.Tensor,
                    check: bool = True, **kw):
        self._stream()
        dev = self._dev()
        omega, dJdU = _f64(omega, dev), _f64(dJdU, dev)
        outs = [torch.empty(geom.M[0], dtype=torch.float64, device=dev) for _ in range(7)]
        rep = Report()
        g = geom.c_struct()
        o = make_opts(**kw)
        rc = self.lib.wwbi_adjoint_phi(self.h, C.byref(g), _ptr(omega), _ptr(dJdU), C.byref(o),
                                       *[_ptr(t) for t in outs], C.byref(rep))
        _check(rc, check, "wwbi_adjoint_phi")
        names = ["phi", "x", "y", "dx", "dy", "ddx", "ddy"]
        return dict(zip(names, outs)), rep

    def solve_phi_multi(self, geom: DeviceGeometry, rhs: torch.Tensor, check: bool = True, **kw):
        """rhs: (n_rhs, sum(M)) device tensor; returns omega of the same shape."""
        self._stream()
        dev = self._dev()
        rhs = _f64(rhs, dev)
        nr = rhs.shape[0]
        out = torch.empty_like(rhs)
        rep = Report()
        g = geom.c_struct()
        o = make_opts(**kw)
        rc = self.lib.wwbi_solve_phi_multi(self.h, C.byref(g), _ptr(rhs), nr, C.byref(o),
                                           _ptr(out), C.byref(rep))
        _check(rc, check, "wwbi_solve_phi_multi")
        return out, rep

    def tangent_phi(self, geom: DeviceGeometry, omega: torch.Tensor, dirs: torch.Tensor,
                    want_omega: bool = False, check: bool = True, **kw):
        """wwbi_tangent_phi: dirs is a (7, nd, M_0) device tensor (x, y, x', y',
        x'', y'', phi~ of the surface nodes for each direction); returns dU
        (nd, M_0), d omega (nd, sum(M)) or None, and the report."""
        self._stream()
        dev = self._dev()
        omega = _f64(omega, dev)
        dirs = _f64(dirs, dev)
        nd = dirs.shape[1]
        dU = torch.empty((nd, geom.M[0]), dtype=torch.float64, device=dev)
        dom = torch.empty((nd, geom.n), dtype=torch.float64, device=dev) if want_omega else None
        rep = Report()
        g = geom.c_struct()
        o = make_opts(**kw)
        rc = self.lib.wwbi_tangent_phi(self.h, C.byref(g), _ptr(omega), nd, _ptr(dirs),
                                       C.byref(o), _ptr(dU), _ptr(dom), C.byref(rep))
        _check(rc, check, "wwbi_tangent_phi")
        return dU, dom, rep

    def spectral(self, f: torch.Tensor, op: int, alpha: float = 1.0, beta: float = 0.0,
                 out: Optional[torch.Tensor] = None) -> torch.Tensor:
        self._stream()
        f = _f64(f, self._dev())
        if out is None:
            out = torch.zeros_like(f)
        rc = self.lib.wwbi_spectral(self.h, f.shape[0], _ptr(f), op, alpha, beta, _ptr(out))
        if rc != OK:
            raise WWBIError(rc, "wwbi_spectral")
        return out

    def surface_fill(self, xt: torch.Tensor, yt: torch.Tensor, outs=None):
        self._stream()
        dev = self._dev()
        xt, yt = _f64(xt, dev), _f64(yt, dev)
        n = xt.shape[0]
        if outs is None:
            outs = [torch.empty(n, dtype=torch.float64, device=dev) for _ in range(6)]
        rc = self.lib.wwbi_surface_fill(self.h, n, _ptr(xt), _ptr(yt), *[_ptr(t) for t in outs])
        if rc != OK:
            raise WWBIError(rc, "wwbi_surface_fill")
        return outs

    def surface_fill_adjoint(self, grads):
        self._stream()
        dev = self._dev()
        grads = [_f64(t, dev) for t in grads]
        n = grads[0].shape[0]
        gxt = torch.empty(n, dtype=torch.float64, device=dev)
        gyt = torch.empty(n, dtype=torch.float64, device=dev)
        rc = self.lib.wwbi_surface_fill_adjoint(self.h, n, *[_ptr(t) for t in grads], _ptr(gxt),
                                                _ptr(gyt))
        if rc != OK:
            raise WWBIError(rc, "wwbi_surface_fill_adjoint")
        return gxt, gyt

    def debug_matrix(self, geom: DeviceGeometry, which: int = MAT_A, precision: int = FP64,
                     band: int = 16) -> torch.Tensor:
        self._stream()
        if which == MAT_T:
            shape = (geom.M[0], geom.n)
        else:
            n = geom.n if which == MAT_A else geom.n - geom.M[0]
            shape = (n, n)
        dt = torch.float64 if precision == FP64 else torch.float32
        out = torch.empty(shape, dtype=dt, device=self._dev())
        g = geom.c_struct()
        rc = self.lib.wwbi_debug_matrix(self.h, C.byref(g), which, precision, band, _ptr(out))
        if rc != OK:
            raise WWBIError(rc, "wwbi_debug_matrix")
        return out

    def matvec(self, geom: DeviceGeometry, x: torch.Tensor, precision: int = FP64,
               mode: int = MATVEC_STORED, transpose: bool = False, band: int = 16):
        self._stream()
        x = _f64(x, self._dev())
        y = torch.empty_like(x)
        rep = Report()
        g = geom.c_struct()
        rc = self.lib.wwbi_matvec(self.h, C.byref(g), _ptr(x), _ptr(y), precision, mode,
                                  int(transpose), band, C.byref(rep))
        if rc != OK:
            raise WWBIError(rc, "wwbi_matvec")
        return y, rep
