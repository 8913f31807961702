"""CPU oracle for the flux-reconstruction residual and Runge-Kutta update.

TEST INFRASTRUCTURE ONLY: a plain, slow, obviously-correct C++ implementation written from the
paper's statement of the method (section "FR Algorithm", Eqs. (1)-(3)). Only tests/, the smoke
check in __graft_entry__ and the bench's CPU-baseline leg may import this package. It shares no
code with the HIP library under paper_2308_06605_amd/.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# FR_ORACLE_LIB_PATH selects another build of the same source (the sanitizer builds below)
LIB_PATH = os.environ.get("FR_ORACLE_LIB_PATH") or os.path.join(_HERE, "liboracle.so")
SRC = os.path.join(_HERE, "fr_oracle.cpp")
SANITIZERS = {"address,undefined", "thread"}

PREC = {"f64": 0, "ld": 1, "f32": 2}
FLUX = {"rusanov": 0, "roe": 1}
SCHEME = {"rk4": 0, "lsrk45": 1, "ssprk104": 2}

_lib = None


def build(force: bool = True, sanitize: str = "") -> str:
    """Compile liboracle.so with g++ (OpenMP, no fast-math, no FMA contraction).

    sanitize = "address,undefined" or "thread": an instrumented build, liboracle_<name>.so, with
    the ROCm clang++ and its OpenMP runtime (whose sanitizer runtimes the process preloads; the
    thread sanitizer runs with the runtime's OMPT race-detection tool). Load it with
    FR_ORACLE_LIB_PATH."""
    if sanitize:
        if sanitize not in SANITIZERS:
            raise ValueError(f"sanitize must be one of {sorted(SANITIZERS)}")
        out = os.path.join(_HERE, "liboracle_" + sanitize.replace(",", "_") + ".so")
        cmd = ["/opt/rocm/llvm/bin/clang++", "-std=c++17", "-O1", "-g", "-fopenmp", "-fPIC", "-shared",
               "-ffp-contract=off", "-fno-omit-frame-pointer", "-fsanitize=" + sanitize, "-o", out + ".tmp", SRC]
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)
        return out
    if force or not os.path.exists(LIB_PATH):
        cmd = ["g++", "-std=c++17", "-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
               "-o", LIB_PATH + ".tmp", SRC]
        subprocess.run(cmd, check=True)
        os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        build()
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i64, i32, f64 = ctypes.c_int64, ctypes.c_int, ctypes.c_double
    L.ora_last_error.restype = ctypes.c_char_p
    L.ora_create.restype = P
    L.ora_create.argtypes = [i32, i32, i64, P, i32, P, f64, f64, f64, f64, i32, i32, i64, P, i32,
                             ctypes.c_uint64, P, f64]
    L.ora_destroy.argtypes = [P]
    for name in ("ora_residual", "ora_sol_coords"):
        getattr(L, name).argtypes = [P, P] if name == "ora_sol_coords" else [P, P, P]
    L.ora_rk_step.argtypes = [P, P, f64, i32, i32]
    L.ora_geometry.argtypes = [P, P, P, P, P]
    L.ora_connectivity.argtypes = [P, P, P, P, P]
    L.ora_basis.argtypes = [i32, i32] + [P] * 9
    L.ora_riemann.argtypes = [i32, f64, P, P, P, P]
    L.ora_inviscid_flux.argtypes = [f64, P, P, P]
    L.ora_viscous_flux.argtypes = [f64, f64, f64, P, P, P]
    L.ora_rk_scalar.argtypes = [i32, i32, f64, f64, f64, i32, P]
    L.ora_rk_upwind.argtypes = [i32, i32, f64, i32, P]
    L.ora_lsrk45_tables.argtypes = [P, P]
    L.ora_n_features.argtypes = [P]
    L.ora_sgs_features.argtypes = [P, P, P]
    L.ora_set_eddy_viscosity.argtypes = [P, P, f64]
    L.ora_set_body_force.argtypes = [P, P]
    L.ora_set_viscous_scheme.argtypes = [P, i32, f64]
    _lib = L
    return L


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class Oracle:
    """Residual / RK on one mesh.

    mesh       : paper_2308_06605_amd.inputs.Mesh (or any object with elem_vert, elem_nodes, q)
    p          : polynomial degree (0..15)
    precision  : "f64", "ld" (long double) or "f32"
    active     : optional element subset whose residual is returned (all by default)
    metric     : "curl" (conservative curl form) or "cross" (cross-product form, a negative
                 control for the freestream test)
    metric_jitter : non-zero seed: each rounded metric term moves by -1, 0 or +1 unit in the
                 last place. A test knob that measures how much two implementations which round
                 the same long-double metric terms independently may differ; 0 = exact rounding.
    """

    def __init__(self, mesh, p: int, *, mu: float = 0.0, gamma: float = 1.4,
                 prandtl: float = 0.72, eta: float = 6.0, flux: str = "rusanov",
                 precision: str = "f64", active=None, metric: str = "curl", nthreads: int = 0,
                 metric_jitter: int = 0, bc_tag=None, wall_T: float = 1.0):
        L = _load()
        self.p = p
        self.n = p + 1
        self.Ns = self.n ** 3
        self.Nfp = self.n ** 2
        self.E = int(mesh.elem_vert.shape[0])
        self._ev = np.ascontiguousarray(mesh.elem_vert, dtype=np.int64)
        self._nodes = np.ascontiguousarray(mesh.elem_nodes, dtype=np.float64)
        if active is None:
            self.active = None
            nact, act_ptr = 0, None
            self.NA = self.E
        else:
            self.active = np.ascontiguousarray(active, dtype=np.int64)
            nact, act_ptr = len(self.active), _ptr(self.active)
            self.NA = nact
        self.nthreads = int(nthreads)
        tags = None
        if bc_tag is not None:
            tags = np.ascontiguousarray(bc_tag, dtype=np.int32)
            assert tags.shape == (self.E, 6)
        self.h = L.ora_create(PREC[precision], p, self.E, _ptr(self._ev), int(mesh.q),
                              _ptr(self._nodes), gamma, prandtl, mu, eta, FLUX[flux],
                              {"curl": 0, "cross": 1}[metric], nact, act_ptr, self.nthreads,
                              int(metric_jitter), _ptr(tags) if tags is not None else None, float(wall_T))
        if not self.h:
            raise RuntimeError("oracle: " + L.ora_last_error().decode())

    def __del__(self):
        if getattr(self, "h", None):
            _load().ora_destroy(self.h)
            self.h = None

    def residual(self, U: np.ndarray) -> np.ndarray:
        U = np.ascontiguousarray(U, dtype=np.float64)
        assert U.shape == (self.E, 5, self.Ns)
        R = np.empty((self.NA, 5, self.Ns))
        rc = _load().ora_residual(self.h, _ptr(U), _ptr(R))
        if rc:
            raise RuntimeError("oracle residual failed")
        return R

    def rk_step(self, U: np.ndarray, dt: float, scheme: str = "rk4", nsteps: int = 1) -> np.ndarray:
        U = np.array(U, dtype=np.float64, order="C", copy=True)
        rc = _load().ora_rk_step(self.h, _ptr(U), dt, SCHEME[scheme], nsteps)
        if rc:
            raise RuntimeError("oracle rk_step failed: " + _load().ora_last_error().decode())
        return U

    def set_eddy_viscosity(self, nu_t, prandtl_t: float = 0.9):
        """Per-element eddy kinematic viscosity [E] (>= 0) for every later residual, or None."""
        if nu_t is None:
            self._nut = None
            rc = _load().ora_set_eddy_viscosity(self.h, None, prandtl_t)
        else:
            self._nut = np.ascontiguousarray(nu_t, dtype=np.float64)
            assert self._nut.shape == (self.E,)
            rc = _load().ora_set_eddy_viscosity(self.h, _ptr(self._nut), prandtl_t)
        if rc:
            raise RuntimeError("oracle: " + _load().ora_last_error().decode())

    def set_viscous_scheme(self, scheme: str = "br2", tau: float = 0.1):
        """"br2" (default) or "ldg" with penalty tau (LDG needs the full mesh)."""
        rc = _load().ora_set_viscous_scheme(self.h, {"br2": 0, "ldg": 1}[scheme], tau)
        if rc:
            raise RuntimeError("oracle: " + _load().ora_last_error().decode())

    def set_body_force(self, g):
        """Constant body force per unit mass (3 values) for every later residual."""
        self._g = np.ascontiguousarray(g, dtype=np.float64)
        assert self._g.shape == (3,)
        _load().ora_set_body_force(self.h, _ptr(self._g))

    def sgs_features(self, U: np.ndarray) -> np.ndarray:
        """Inputs of the learned closure per (active) element: [NA][(p+1)^3 + 4]."""
        U = np.ascontiguousarray(U, dtype=np.float64)
        assert U.shape == (self.E, 5, self.Ns)
        nf = _load().ora_n_features(self.h)
        out = np.empty((self.NA, nf))
        _load().ora_sgs_features(self.h, _ptr(U), _ptr(out))
        return out

    def sol_coords(self) -> np.ndarray:
        X = np.empty((self.NA, 3, self.Ns))
        _load().ora_sol_coords(self.h, _ptr(X))
        return X

    def geometry(self):
        """(Ja [NA,Ns,3,3] with Ja[n,i] = |J| dxi_n/dx_i, detJ [NA,Ns], Nf [NA,6,Nfp,3], Jf [NA,6,Nfp])"""
        Ja = np.empty((self.NA, self.Ns, 3, 3))
        dJ = np.empty((self.NA, self.Ns))
        Nf = np.empty((self.NA, 6, self.Nfp, 3))
        Jf = np.empty((self.NA, 6, self.Nfp))
        _load().ora_geometry(self.h, _ptr(Ja), _ptr(dJ), _ptr(Nf), _ptr(Jf))
        return Ja, dJ, Nf, Jf

    def connectivity(self):
        nbr = np.empty((self.E, 6), dtype=np.int64)
        nface = np.empty((self.E, 6), dtype=np.int32)
        owner = np.empty((self.E, 6), dtype=np.int32)
        perm = np.empty((self.E, 6, self.Nfp), dtype=np.int32)
        _load().ora_connectivity(self.h, _ptr(nbr), _ptr(nface), _ptr(owner), _ptr(perm))
        return nbr, nface, owner, perm


def basis(p: int, precision: str = "f64") -> dict:
    n = p + 1
    g = max(p, 1) + 1
    out = {k: np.empty(n) for k in ("xs", "ws", "lm", "lp", "gcR", "gcL")}
    out["D"] = np.empty((n, n))
    out["xg"] = np.empty(g)
    out["wg"] = np.empty(g)
    _load().ora_basis(PREC[precision], p, _ptr(out["xs"]), _ptr(out["ws"]), _ptr(out["D"]),
                      _ptr(out["lm"]), _ptr(out["lp"]), _ptr(out["gcR"]), _ptr(out["gcL"]),
                      _ptr(out["xg"]), _ptr(out["wg"]))
    return out


def riemann(flux: str, UL, UR, n, gamma: float = 1.4) -> np.ndarray:
    UL = np.ascontiguousarray(UL, dtype=np.float64)
    UR = np.ascontiguousarray(UR, dtype=np.float64)
    n = np.ascontiguousarray(n, dtype=np.float64)
    F = np.empty(5)
    _load().ora_riemann(FLUX[flux], gamma, _ptr(UL), _ptr(UR), _ptr(n), _ptr(F))
    return F


def inviscid_flux(U, n, gamma: float = 1.4) -> np.ndarray:
    U = np.ascontiguousarray(U, dtype=np.float64)
    n = np.ascontiguousarray(n, dtype=np.float64)
    F = np.empty(5)
    _load().ora_inviscid_flux(gamma, _ptr(U), _ptr(n), _ptr(F))
    return F


def viscous_flux(U, G, mu: float, gamma: float = 1.4, prandtl: float = 0.72) -> np.ndarray:
    U = np.ascontiguousarray(U, dtype=np.float64)
    G = np.ascontiguousarray(G, dtype=np.float64).reshape(3, 5)
    Fv = np.empty((3, 5))
    _load().ora_viscous_flux(gamma, prandtl, mu, _ptr(U), _ptr(G), _ptr(Fv))
    return Fv


def rk_scalar(scheme: str, ode: int, lam: float, y0: float, dt: float, nsteps: int) -> np.ndarray:
    out = np.empty(nsteps + 1)
    _load().ora_rk_scalar(SCHEME[scheme], ode, lam, y0, dt, nsteps, _ptr(out))
    return out


def lsrk45_tables():
    """(A[5], B[5]): the 2N-storage coefficients the oracle's LSRK45 driver uses."""
    A, B = np.empty(5), np.empty(5)
    _load().ora_lsrk45_tables(_ptr(A), _ptr(B))
    return A, B


def rk_upwind(scheme: str, u0, dt: float, nsteps: int) -> np.ndarray:
    """The RK driver on periodic first-order upwind advection with unit spacing."""
    u = np.array(u0, dtype=np.float64, order="C", copy=True)
    rc = _load().ora_rk_upwind(SCHEME[scheme], u.size, dt, nsteps, _ptr(u))
    if rc:
        raise RuntimeError("oracle rk_upwind failed")
    return u
