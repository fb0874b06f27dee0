"""ctypes binding of the plain FP64 CPU oracle (``cosenu_oracle.c``).

TEST INFRASTRUCTURE ONLY.  The product library never imports this module;
only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark do.  The oracle shares no code with the GPU path.

State arrays are numpy float64 of shape (8, nz, nv), C-contiguous, with the
component order (rho_ee, rho_xx, Re rho_ex, Im rho_ex, rhobar_ee, rhobar_xx,
Re rhobar_ex, Im rhobar_ex).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cosenu_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

FD_KO = 0
FV_WENO7 = 1

# velocity grid and quadrature rule (Sec. 3.1)
QUAD_MIDPOINT = 0
QUAD_TRAPEZOID = 1
QUAD_SIMPSON = 2

# index names of oracle_diagnostics' output
DIAG_NAMES = ("M0_trace", "M0_x", "M0_y", "M0_z", "N_nu", "N_nubar", "dP_max", "dP_mean",
              "ee_nu", "ee_nubar", "B_dot_M0", "nonfinite")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no fused multiply-add contraction)."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
           SRC, "-o", tmp, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


class _Params(ctypes.Structure):
    _fields_ = [
        ("nz", ctypes.c_int32), ("nv", ctypes.c_int32),
        ("L", ctypes.c_double), ("dt", ctypes.c_double),
        ("mu", ctypes.c_double), ("omega", ctypes.c_double), ("theta", ctypes.c_double),
        ("lam", ctypes.c_double), ("alpha", ctypes.c_double),
        ("scheme", ctypes.c_int32), ("ko_r", ctypes.c_int32),
        ("ko_eps", ctypes.c_double), ("weno_eps", ctypes.c_double),
        ("g_nu", ctypes.POINTER(ctypes.c_double)), ("g_nubar", ctypes.POINTER(ctypes.c_double)),
        ("quad", ctypes.c_int32),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build(force=True)
        L = ctypes.CDLL(LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        L.oracle_velocity.restype = ctypes.c_double
        L.oracle_velocity.argtypes = [ctypes.c_int32, ctypes.c_int32]
        L.oracle_velocity_q.restype = ctypes.c_double
        L.oracle_velocity_q.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
        L.oracle_vweight.restype = ctypes.c_double
        L.oracle_vweight.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
        L.oracle_dt_q.restype = ctypes.c_double
        L.oracle_dt_q.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                  ctypes.c_double]
        L.oracle_angular_dist_q.restype = None
        L.oracle_angular_dist_q.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double, dp]
        L.oracle_position.restype = ctypes.c_double
        L.oracle_position.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_int32]
        L.oracle_dt.restype = ctypes.c_double
        L.oracle_dt.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double]
        L.oracle_angular_dist.restype = None
        L.oracle_angular_dist.argtypes = [ctypes.c_int32, ctypes.c_double, dp]
        L.oracle_initial_state.restype = None
        L.oracle_initial_state.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_double, ctypes.c_double, dp]
        L.oracle_weno7_parts.restype = None
        L.oracle_weno7_parts.argtypes = [dp, ctypes.c_double, dp, dp, dp]
        L.oracle_weno7_minus.restype = ctypes.c_double
        L.oracle_weno7_minus.argtypes = [dp, ctypes.c_double]
        L.oracle_rhs.restype = None
        L.oracle_rhs.argtypes = [ctypes.POINTER(_Params), dp, dp]
        L.oracle_rk4.restype = ctypes.c_int
        L.oracle_rk4.argtypes = [ctypes.POINTER(_Params), dp, ctypes.c_int64]
        L.oracle_moments.restype = None
        L.oracle_moments.argtypes = [ctypes.POINTER(_Params), dp, dp]
        L.oracle_diagnostics.restype = None
        L.oracle_diagnostics.argtypes = [ctypes.POINTER(_Params), dp, dp]
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_num_threads.argtypes = []
        L.oracle_set_num_threads.restype = ctypes.c_int
        L.oracle_set_num_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check_quad(nv: int, quad: int):
    if quad not in (QUAD_MIDPOINT, QUAD_TRAPEZOID, QUAD_SIMPSON):
        raise ValueError(f"unknown quadrature {quad}")
    if quad != QUAD_MIDPOINT and nv < 2:
        raise ValueError("a vertex grid needs nv >= 2")
    if quad == QUAD_SIMPSON and nv % 2 == 0:
        raise ValueError("Simpson's rule needs an odd number of velocity points")


def velocities(nv: int, quad: int = QUAD_MIDPOINT) -> np.ndarray:
    _check_quad(nv, quad)
    return np.array([lib().oracle_velocity_q(nv, quad, j) for j in range(nv)])


def vweights(nv: int, quad: int = QUAD_MIDPOINT) -> np.ndarray:
    """Quadrature weights w_j of the velocity integral."""
    _check_quad(nv, quad)
    return np.array([lib().oracle_vweight(nv, quad, j) for j in range(nv)])


def positions(nz: int, L: float) -> np.ndarray:
    return np.array([lib().oracle_position(nz, L, i) for i in range(nz)])


def dt_from_cfl(nz: int, nv: int, L: float, cfl: float, quad: int = QUAD_MIDPOINT) -> float:
    _check_quad(nv, quad)
    return lib().oracle_dt_q(nz, nv, quad, L, cfl)


def angular_dist(nv: int, sigma: float, quad: int = QUAD_MIDPOINT) -> np.ndarray:
    _check_quad(nv, quad)
    g = np.zeros(nv)
    lib().oracle_angular_dist_q(nv, quad, sigma, _ptr(g))
    return g


def initial_state(nz: int, nv: int, L: float, amp: float, width: float, phi: float) -> np.ndarray:
    y = np.zeros((8, nz, nv))
    lib().oracle_initial_state(nz, nv, L, amp, width, phi, _ptr(y))
    return y


def weno7_minus(a, eps: float = 1e-6) -> float:
    arr = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    assert arr.shape == (7,)
    return lib().oracle_weno7_minus(_ptr(arr), eps)


def weno7_parts(a, eps: float = 1e-6):
    """(q_r, SI_r, unnormalised w_r) of the reconstruction at i+1/2, r = 0..3."""
    arr = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    assert arr.shape == (7,)
    q, si, w = np.zeros(4), np.zeros(4), np.zeros(4)
    lib().oracle_weno7_parts(_ptr(arr), eps, _ptr(q), _ptr(si), _ptr(w))
    return q, si, w


@dataclass
class Problem:
    """Everything the oracle needs besides the state."""
    nz: int
    nv: int
    L: float
    dt: float
    mu: float = 1.0
    omega: float = 0.0
    theta: float = 0.0
    lam: float = 0.0
    alpha: float = 0.9
    scheme: int = FD_KO
    ko_eps: float = 0.1
    ko_r: int = 2
    weno_eps: float = 1e-6
    g_nu: np.ndarray = field(default=None)
    g_nubar: np.ndarray = field(default=None)
    quad: int = QUAD_MIDPOINT

    def _c(self):
        _check_quad(self.nv, self.quad)
        self.g_nu = np.ascontiguousarray(self.g_nu, dtype=np.float64)
        self.g_nubar = np.ascontiguousarray(self.g_nubar, dtype=np.float64)
        assert self.g_nu.shape == (self.nv,) and self.g_nubar.shape == (self.nv,)
        return _Params(self.nz, self.nv, self.L, self.dt, self.mu, self.omega, self.theta, self.lam,
                       self.alpha, self.scheme, self.ko_r, self.ko_eps, self.weno_eps,
                       _ptr(self.g_nu), _ptr(self.g_nubar), self.quad)


def _check_state(p: Problem, y: np.ndarray):
    assert y.shape == (8, p.nz, p.nv) and y.dtype == np.float64 and y.flags["C_CONTIGUOUS"], y.shape


def rhs(p: Problem, y: np.ndarray) -> np.ndarray:
    _check_state(p, y)
    k = np.zeros_like(y)
    cp = p._c()
    lib().oracle_rhs(ctypes.byref(cp), _ptr(y), _ptr(k))
    return k


def rk4(p: Problem, y: np.ndarray, nsteps: int) -> np.ndarray:
    """Advance a copy of y by nsteps classic RK4 steps and return it."""
    _check_state(p, y)
    out = np.array(y, dtype=np.float64, order="C", copy=True)
    cp = p._c()
    rc = lib().oracle_rk4(ctypes.byref(cp), _ptr(out), int(nsteps))
    if rc != 0:
        raise MemoryError("oracle_rk4 could not allocate its stage arrays")
    return out


def moments(p: Problem, y: np.ndarray) -> np.ndarray:
    _check_state(p, y)
    out = np.zeros((p.nz, 2, 4))
    cp = p._c()
    lib().oracle_moments(ctypes.byref(cp), _ptr(y), _ptr(out))
    return out


def diagnostics(p: Problem, y: np.ndarray) -> dict:
    _check_state(p, y)
    out = np.zeros(len(DIAG_NAMES))
    cp = p._c()
    lib().oracle_diagnostics(ctypes.byref(cp), _ptr(y), _ptr(out))
    return dict(zip(DIAG_NAMES, out.tolist()))


def num_threads() -> int:
    return lib().oracle_num_threads()


def set_num_threads(n: int) -> int:
    """Thread count of later oracle calls; returns the count in force."""
    return lib().oracle_set_num_threads(int(n))


def problem_from_workload(w: dict) -> Problem:
    """Build a Problem from a workload dict (see paper_2203_12866_amd.workloads)."""
    quad = w.get("quadrature", QUAD_MIDPOINT)
    dt = dt_from_cfl(w["nz"], w["nv"], w["L"], w["cfl"], quad)
    return Problem(nz=w["nz"], nv=w["nv"], L=w["L"], dt=dt, mu=w["mu"], omega=w["omega"],
                   theta=w["theta"], lam=w["lam"], alpha=w["alpha"], scheme=w["scheme"],
                   ko_eps=w["ko_eps"], ko_r=w.get("ko_order", 2), weno_eps=w["weno_eps"],
                   g_nu=angular_dist(w["nv"], w["sigma_nu"], quad),
                   g_nubar=angular_dist(w["nv"], w["sigma_nubar"], quad), quad=quad)


def initial_state_for(w: dict) -> np.ndarray:
    return initial_state(w["nz"], w["nv"], w["L"], w["pert_amp"], w["pert_width"], w["phase"])
