"""ctypes binding of libfr (include/fr.h): argument marshalling only.

Device arrays are torch tensors on the handle's GPU (their data_ptr() is passed through);
host arrays are numpy arrays. Every computation runs in libfr's HIP kernels; if the library is
missing this module raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfr.so")

FR_OK = 0
ERRORS = {-1: "FR_ERR_ARG", -2: "FR_ERR_MESH", -3: "FR_ERR_HIP", -4: "FR_ERR_OOM",
          -5: "FR_ERR_UNSUPPORTED", -6: "FR_ERR_NONFINITE"}
FLUX = {"rusanov": 0, "roe": 1}
PREC = {"fp64": 0, "fp32": 1}
SCHEME = {"rk4": 0, "lsrk45": 1}


class FRError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code
        self.name = ERRORS.get(code, str(code))


class fr_mesh_desc(ctypes.Structure):
    _fields_ = [
        ("p", ctypes.c_int32), ("q", ctypes.c_int32), ("n_elem", ctypes.c_int64),
        ("elem_vert", ctypes.c_void_p), ("elem_nodes", ctypes.c_void_p),
        ("gamma", ctypes.c_double), ("prandtl", ctypes.c_double), ("mu", ctypes.c_double),
        ("br2_eta", ctypes.c_double), ("flux", ctypes.c_int32), ("prec", ctypes.c_int32),
        ("check_finite", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("ref_rho", ctypes.c_double), ("ref_p", ctypes.c_double),
    ]


_lib = None


def load():
    """Load libfr.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2308_06605_amd.build`"
                           " (or __graft_entry__.build()); there is no fallback path")
    L = ctypes.CDLL(LIB_PATH)
    P, i32, i64, f64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
    L.fr_last_error.restype = ctypes.c_char_p
    L.fr_mesh_create.argtypes = [ctypes.POINTER(fr_mesh_desc), P, ctypes.POINTER(P)]
    L.fr_mesh_destroy.argtypes = [P]
    L.fr_set_stream.argtypes = [P, P]
    L.fr_sol_coords.argtypes = [P, P]
    L.fr_set_state.argtypes = [P, P, i32]
    L.fr_get_state.argtypes = [P, P, i32]
    L.fr_residual.argtypes = [P, P, i32]
    L.fr_rk_step.argtypes = [P, f64, i32, i32]
    L.fr_mesh_info.argtypes = [P, ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(i64)]
    L.fr_profile_stages.argtypes = [P, f64, i32, i32, P]
    L.fr_mesh_geometry_host.argtypes = [ctypes.POINTER(fr_mesh_desc), P, P, P, P, P]
    L.fr_basis_host.argtypes = [i32, P, P, P, P, P]
    L.fr_kinetic_energy.argtypes = [P, P]
    for name in ("fr_mesh_create", "fr_mesh_destroy", "fr_set_stream", "fr_sol_coords", "fr_set_state",
                 "fr_get_state", "fr_residual", "fr_rk_step", "fr_mesh_info", "fr_profile_stages",
                 "fr_mesh_geometry_host", "fr_basis_host", "fr_kinetic_energy"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(rc: int):
    if rc != FR_OK:
        raise FRError(rc, load().fr_last_error().decode())


def _current_stream():
    import torch

    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _desc(mesh, p, mu, gamma, prandtl, eta, flux, prec, check_finite, keep, ref=(1.0, 0.0)):
    ev = np.ascontiguousarray(mesh.elem_vert, dtype=np.int64)
    nodes = np.ascontiguousarray(mesh.elem_nodes, dtype=np.float64)
    keep.extend([ev, nodes])
    return fr_mesh_desc(p=int(p), q=int(mesh.q), n_elem=int(ev.shape[0]), elem_vert=ev.ctypes.data,
                        elem_nodes=nodes.ctypes.data, gamma=gamma, prandtl=prandtl, mu=mu,
                        br2_eta=eta, flux=FLUX[flux], prec=PREC[prec],
                        check_finite=int(bool(check_finite)), reserved=0,
                        ref_rho=float(ref[0]), ref_p=float(ref[1]))


def geometry_host(mesh, p: int, eta: float = 6.0):
    """Host-only mesh setup (fr_mesh_geometry_host): geo, fgeo, ftab, conn, xyz as numpy arrays."""
    keep = []
    d = _desc(mesh, p, 0.0, 1.4, 0.72, eta, "rusanov", "fp64", False, keep)
    E, Ns, Nfp = d.n_elem, (p + 1) ** 3, (p + 1) ** 2
    geo = np.empty((E, 10, Ns))
    fgeo = np.empty((3 * E, 4, Nfp))
    ftab = np.empty((3 * E, 4), dtype=np.int32)
    conn = np.empty((E, 6, 2), dtype=np.int32)
    xyz = np.empty((E, 3, Ns))
    _check(load().fr_mesh_geometry_host(ctypes.byref(d), geo.ctypes.data, fgeo.ctypes.data,
                                        ftab.ctypes.data, conn.ctypes.data, xyz.ctypes.data))
    return geo, fgeo, ftab, conn, xyz


def basis_host(p: int) -> dict:
    """The library's 1-D operator tables of degree p (fr_basis_host)."""
    n = p + 1
    out = {"D": np.empty((n, n)), "lm": np.empty(n), "lp": np.empty(n), "gcL": np.empty(n), "gcR": np.empty(n)}
    _check(load().fr_basis_host(int(p), *(out[k].ctypes.data for k in ("D", "lm", "lp", "gcL", "gcR"))))
    return out


class FRMesh:
    """One mesh on the current GPU (see fr_mesh_create)."""

    def __init__(self, mesh, p: int, *, mu: float = 0.0, gamma: float = 1.4, prandtl: float = 0.72,
                 eta: float = 6.0, flux: str = "rusanov", prec: str = "fp64", check_finite: bool = False,
                 stream=None, ref_rho: float = 1.0, ref_p: float = 0.0):
        L = load()
        self.p = int(p)
        self.Ns = (self.p + 1) ** 3
        self.E = int(mesh.elem_vert.shape[0])
        keep = []
        d = _desc(mesh, p, mu, gamma, prandtl, eta, flux, prec, check_finite, keep, (ref_rho, ref_p))
        self._stream = _current_stream() if stream is None else ctypes.c_void_p(stream)
        h = ctypes.c_void_p()
        _check(L.fr_mesh_create(ctypes.byref(d), self._stream, ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            load().fr_mesh_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream):
        self._stream = ctypes.c_void_p(stream)
        _check(load().fr_set_stream(self.h, self._stream))

    @property
    def shape(self):
        return (self.E, 5, self.Ns)

    def sol_coords(self) -> np.ndarray:
        X = np.empty((self.E, 3, self.Ns))
        _check(load().fr_sol_coords(self.h, X.ctypes.data))
        return X

    def set_state(self, U):
        if hasattr(U, "data_ptr"):  # torch tensor on the device
            assert U.is_cuda and U.dtype.is_floating_point and U.is_contiguous() and tuple(U.shape) == self.shape
            _check(load().fr_set_state(self.h, ctypes.c_void_p(U.data_ptr()), 1))
        else:
            U = np.ascontiguousarray(U, dtype=np.float64)
            assert U.shape == self.shape
            _check(load().fr_set_state(self.h, U.ctypes.data, 0))

    def get_state(self, out=None):
        if out is not None and hasattr(out, "data_ptr"):
            _check(load().fr_get_state(self.h, ctypes.c_void_p(out.data_ptr()), 1))
            return out
        U = np.empty(self.shape)
        _check(load().fr_get_state(self.h, U.ctypes.data, 0))
        return U

    def residual(self, out=None):
        """dU/dt of the current state: into a device tensor `out`, else returned as numpy."""
        if out is not None:
            assert out.is_cuda and tuple(out.shape) == self.shape and out.is_contiguous()
            _check(load().fr_residual(self.h, ctypes.c_void_p(out.data_ptr()), 1))
            return out
        R = np.empty(self.shape)
        _check(load().fr_residual(self.h, R.ctypes.data, 0))
        return R

    def rk_step(self, dt: float, scheme: str = "lsrk45", n_steps: int = 1):
        _check(load().fr_rk_step(self.h, float(dt), SCHEME[scheme], int(n_steps)))

    def profile_stages(self, dt: float, scheme: str = "lsrk45", n_steps: int = 1):
        """Mean ms per stage of (pre-pass, face, volume) kernels, from HIP events."""
        ms = np.zeros(3)
        _check(load().fr_profile_stages(self.h, float(dt), SCHEME[scheme], int(n_steps), ms.ctypes.data))
        return tuple(float(x) for x in ms)

    def kinetic_energy(self):
        """(E_k, dE_k/dt) of the current state, volume averaged (fr_kinetic_energy)."""
        out = np.zeros(2)
        _check(load().fr_kinetic_energy(self.h, out.ctypes.data))
        return float(out[0]), float(out[1])

    def info(self):
        E, ns, b = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int64()
        _check(load().fr_mesh_info(self.h, ctypes.byref(E), ctypes.byref(ns), ctypes.byref(b)))
        return {"n_elem": E.value, "n_sol": ns.value, "device_bytes": b.value}
