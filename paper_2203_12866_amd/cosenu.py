"""Thin ctypes binding of the C ABI in include/cosenu.h (libcosenu.so).

Argument marshalling only: every step of the hot path runs in the HIP
kernels of the shared library.  There is no CPU fallback; if the library has
not been built, loading fails with an error that says so.

PyTorch is used, optionally, for streams only (``Sim.bind_torch_stream``).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcosenu.so")

FD_KO = 0
FV_WENO7 = 1
FP64 = 0
FP32_ACC64 = 1
QUAD_MIDPOINT = 0
QUAD_TRAPEZOID = 1
QUAD_SIMPSON = 2

OK, EINVAL, ENOMEM, EDEVICE, ENONFINITE, ESTATE = 0, -1, -2, -3, -4, -5


class CosenuError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str = ""):
        self.code = code
        msg = f"{where}: {_lib().cosenu_strerror(code).decode()} ({code})"
        if detail:
            msg += f": {detail}"
        super().__init__(msg)


class Params(ctypes.Structure):
    _fields_ = [
        ("nz", ctypes.c_int32), ("nv", ctypes.c_int32),
        ("scheme", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("L", ctypes.c_double), ("cfl", ctypes.c_double),
        ("mu", ctypes.c_double), ("omega", ctypes.c_double), ("theta", ctypes.c_double), ("lam", ctypes.c_double),
        ("alpha", ctypes.c_double), ("sigma_nu", ctypes.c_double), ("sigma_nubar", ctypes.c_double),
        ("pert_amp", ctypes.c_double), ("pert_width", ctypes.c_double), ("phase", ctypes.c_double),
        ("ko_eps", ctypes.c_double), ("weno_eps", ctypes.c_double),
        ("ko_order", ctypes.c_int32), ("quadrature", ctypes.c_int32),
    ]


class Conserved(ctypes.Structure):
    _fields_ = [
        ("t", ctypes.c_double), ("step", ctypes.c_int64),
        ("M0", ctypes.c_double * 4),
        ("N_nu", ctypes.c_double), ("N_nubar", ctypes.c_double),
        ("dP_max", ctypes.c_double), ("dP_mean", ctypes.c_double),
        ("ee_nu", ctypes.c_double), ("ee_nubar", ctypes.c_double),
        ("Pee_nu", ctypes.c_double), ("Pee_nubar", ctypes.c_double),
        ("B_dot_M0", ctypes.c_double),
        ("nonfinite", ctypes.c_int64),
    ]

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "M0"}
        d["M0"] = list(self.M0)
        return d


class Info(ctypes.Structure):
    _fields_ = [
        ("dt", ctypes.c_double), ("dz", ctypes.c_double), ("dv", ctypes.c_double), ("t", ctypes.c_double),
        ("step", ctypes.c_int64), ("device_bytes", ctypes.c_size_t),
        ("seg_rows", ctypes.c_int32), ("lanes_per_row", ctypes.c_int32), ("v_chunks", ctypes.c_int32),
        ("blocks_per_stage", ctypes.c_int32), ("bytes_per_step", ctypes.c_double),
        ("launches_per_step", ctypes.c_int32), ("waves_per_workgroup", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it first (python -c 'import __graft_entry__ as g; g.build()')")
        # torch ships its own copy of the HIP runtime under the same soname; load
        # it first so that this library binds to that copy and one process never
        # holds two HIP runtimes (the second cannot open the device).
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        vp, dp, i32, i64, sz = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
        PP = ctypes.POINTER(Params)
        sigs = {
            "cosenu_params_default": (ctypes.c_int, [PP]),
            "cosenu_create": (ctypes.c_int, [PP, ctypes.POINTER(vp)]),
            "cosenu_destroy": (None, [vp]),
            "cosenu_step": (ctypes.c_int, [vp, i64]),
            "cosenu_sync": (ctypes.c_int, [vp]),
            "cosenu_get_state": (ctypes.c_int, [vp, dp, sz]),
            "cosenu_set_state": (ctypes.c_int, [vp, dp, sz]),
            "cosenu_get_rows": (ctypes.c_int, [vp, ctypes.c_int64, ctypes.c_int32, dp, sz]),
            "cosenu_set_clock": (ctypes.c_int, [vp, ctypes.c_double, i64]),
            "cosenu_moments": (ctypes.c_int, [vp, dp, sz]),
            "cosenu_conserved": (ctypes.c_int, [vp, ctypes.POINTER(Conserved)]),
            "cosenu_info": (ctypes.c_int, [vp, ctypes.POINTER(Info)]),
            "cosenu_set_stream": (ctypes.c_int, [vp, vp]),
            "cosenu_set_seg_rows": (ctypes.c_int, [vp, i32]),
            "cosenu_time_steps": (ctypes.c_int, [vp, i64, dp]),
            "cosenu_time_stages": (ctypes.c_int, [vp, i64, dp]),
            "cosenu_autotune": (ctypes.c_int, [vp, ctypes.POINTER(i32)]),
            "cosenu_set_fusion": (ctypes.c_int, [vp, i32]),
            "cosenu_strerror": (ctypes.c_char_p, [ctypes.c_int]),
            "cosenu_last_error": (ctypes.c_char_p, [vp]),
            "cosenu_batch_create": (ctypes.c_int, [PP, i32, ctypes.POINTER(vp)]),
            "cosenu_batch_destroy": (None, [vp]),
            "cosenu_batch_step": (ctypes.c_int, [vp, i64]),
            "cosenu_batch_sync": (ctypes.c_int, [vp]),
            "cosenu_batch_get_state": (ctypes.c_int, [vp, i32, dp, sz]),
            "cosenu_batch_set_state": (ctypes.c_int, [vp, i32, dp, sz]),
            "cosenu_batch_conserved": (ctypes.c_int, [vp, i32, ctypes.POINTER(Conserved)]),
            "cosenu_batch_moments": (ctypes.c_int, [vp, i32, dp, sz]),
            "cosenu_batch_set_clock": (ctypes.c_int, [vp, i32, ctypes.c_double, i64]),
            "cosenu_batch_get_rows": (ctypes.c_int, [vp, i32, ctypes.c_int64, ctypes.c_int32, dp, sz]),
            "cosenu_batch_info": (ctypes.c_int, [vp, i32, ctypes.POINTER(Info)]),
            "cosenu_batch_time_steps": (ctypes.c_int, [vp, i64, dp]),
            "cosenu_batch_autotune": (ctypes.c_int, [vp, ctypes.POINTER(i32)]),
            "cosenu_batch_last_error": (ctypes.c_char_p, [vp]),
            "cosenu_test_inject_failure": (ctypes.c_int, [i32, i32]),
            "cosenu_step_noalloc": (ctypes.c_int, [PP, vp, i64, vp]),
        }
        for name, (res, args) in sigs.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _LIB = L
    return _LIB


def lib():
    """The loaded shared library (raises ImportError if it was not built)."""
    return _lib()


def default_params() -> Params:
    p = Params()
    rc = _lib().cosenu_params_default(ctypes.byref(p))
    if rc:
        raise CosenuError(rc, "cosenu_params_default")
    return p


_KEYMAP = {"lambda": "lam", "lam": "lam"}


def params_from(w: dict | None = None, **kw) -> Params:
    """Params from a workload dict (paper_2203_12866_amd.workloads) and/or keywords."""
    p = default_params()
    src = dict(w or {})
    src.update(kw)
    names = {f for f, _ in Params._fields_}
    for k, v in src.items():
        k2 = _KEYMAP.get(k, k)
        if k2 in names:
            setattr(p, k2, v)
    return p


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Sim:
    """One simulation (cosenu_sim handle)."""

    def __init__(self, params: Params | dict | None = None, **kw):
        if not isinstance(params, Params):
            params = params_from(params, **kw)
        self.params = params
        h = ctypes.c_void_p()
        rc = _lib().cosenu_create(ctypes.byref(params), ctypes.byref(h))
        if rc:
            raise CosenuError(rc, "cosenu_create")
        self._h = h
        self.nz, self.nv = params.nz, params.nv

    def _check(self, rc: int, where: str):
        if rc:
            raise CosenuError(rc, where, _lib().cosenu_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            _lib().cosenu_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def step(self, n: int = 1):
        self._check(_lib().cosenu_step(self._h, int(n)), "cosenu_step")

    def sync(self):
        self._check(_lib().cosenu_sync(self._h), "cosenu_sync")

    def get_state(self) -> np.ndarray:
        out = np.empty((8, self.nz, self.nv))
        self._check(_lib().cosenu_get_state(self._h, _dptr(out), out.size), "cosenu_get_state")
        return out

    def get_rows(self, z0: int, nrows: int) -> np.ndarray:
        """State of rows z0 .. z0+nrows-1 (periodic), shape (8, nrows, nv)."""
        out = np.empty((8, int(nrows), self.nv))
        self._check(_lib().cosenu_get_rows(self._h, int(z0), int(nrows), _dptr(out), out.size), "cosenu_get_rows")
        return out

    def set_state(self, y: np.ndarray):
        a = np.ascontiguousarray(y, dtype=np.float64)
        if a.shape != (8, self.nz, self.nv):
            raise ValueError(f"state must have shape (8, {self.nz}, {self.nv}), got {a.shape}")
        self._check(_lib().cosenu_set_state(self._h, _dptr(a), a.size), "cosenu_set_state")

    def set_clock(self, t: float, step: int):
        self._check(_lib().cosenu_set_clock(self._h, float(t), int(step)), "cosenu_set_clock")

    def moments(self) -> np.ndarray:
        out = np.empty((self.nz, 2, 4))
        self._check(_lib().cosenu_moments(self._h, _dptr(out), out.size), "cosenu_moments")
        return out

    def conserved(self, allow_nonfinite: bool = False) -> dict:
        c = Conserved()
        rc = _lib().cosenu_conserved(self._h, ctypes.byref(c))
        if rc and not (allow_nonfinite and rc == ENONFINITE):
            self._check(rc, "cosenu_conserved")
        return c.as_dict()

    def info(self) -> dict:
        i = Info()
        self._check(_lib().cosenu_info(self._h, ctypes.byref(i)), "cosenu_info")
        return i.as_dict()

    def set_stream(self, hip_stream: int | None):
        self._check(_lib().cosenu_set_stream(self._h, ctypes.c_void_p(hip_stream or 0)), "cosenu_set_stream")

    def bind_torch_stream(self, stream=None):
        """Enqueue on a torch HIP stream (default: torch's current stream)."""
        import torch
        s = stream if stream is not None else torch.cuda.current_stream()
        self.set_stream(int(s.cuda_stream))

    def set_seg_rows(self, seg: int):
        self._check(_lib().cosenu_set_seg_rows(self._h, int(seg)), "cosenu_set_seg_rows")

    def time_steps(self, n: int) -> float:
        ms = ctypes.c_double()
        self._check(_lib().cosenu_time_steps(self._h, int(n), ctypes.byref(ms)), "cosenu_time_steps")
        return ms.value

    def time_stages(self, n: int) -> list:
        ms = (ctypes.c_double * 4)()
        self._check(_lib().cosenu_time_stages(self._h, int(n), ms), "cosenu_time_stages")
        return list(ms)

    def set_fusion(self, on):
        """0 / False: four single stages; 1 / True: fused (stage pairs, or the
        path the autotuner chose); 2: the whole RK4 step in one launch where the
        shape allows it.  Results are bitwise the same on every path."""
        self._check(_lib().cosenu_set_fusion(self._h, int(on)), "cosenu_set_fusion")

    def autotune(self) -> int:
        seg = ctypes.c_int32()
        self._check(_lib().cosenu_autotune(self._h, ctypes.byref(seg)), "cosenu_autotune")
        return seg.value


def step_noalloc(params: Params | dict, state_ptr: int, nsteps: int, hip_stream: int | None = None):
    """cosenu_step_noalloc: nsteps RK4 steps of a caller-owned FP64 device state
    [8][nz][nv] at address state_ptr (for example a torch tensor's data_ptr()),
    with the library's static scratch array instead of allocations; enqueued on
    hip_stream (None: the default stream), asynchronous."""
    p = params if isinstance(params, Params) else params_from(params)
    rc = _lib().cosenu_step_noalloc(ctypes.byref(p), ctypes.c_void_p(int(state_ptr)), int(nsteps),
                                    ctypes.c_void_p(hip_stream or 0))
    if rc:
        raise CosenuError(rc, "cosenu_step_noalloc")


class Batch:
    """Many independent simulations advanced by one graph (cosenu_batch handle)."""

    def __init__(self, params_list):
        ps = [p if isinstance(p, Params) else params_from(p) for p in params_list]
        arr = (Params * len(ps))(*ps)
        h = ctypes.c_void_p()
        rc = _lib().cosenu_batch_create(arr, len(ps), ctypes.byref(h))
        if rc:
            raise CosenuError(rc, "cosenu_batch_create")
        self._h = h
        self.params = ps
        self.shapes = [(p.nz, p.nv) for p in ps]

    def _check(self, rc, where):
        if rc:
            raise CosenuError(rc, where, _lib().cosenu_batch_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            _lib().cosenu_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __len__(self):
        return len(self.shapes)

    def step(self, n: int = 1):
        self._check(_lib().cosenu_batch_step(self._h, int(n)), "cosenu_batch_step")

    def sync(self):
        self._check(_lib().cosenu_batch_sync(self._h), "cosenu_batch_sync")

    def get_state(self, i: int) -> np.ndarray:
        nz, nv = self.shapes[i]
        out = np.empty((8, nz, nv))
        self._check(_lib().cosenu_batch_get_state(self._h, i, _dptr(out), out.size), "cosenu_batch_get_state")
        return out

    def set_state(self, i: int, y: np.ndarray):
        nz, nv = self.shapes[i]
        a = np.ascontiguousarray(y, dtype=np.float64)
        if a.shape != (8, nz, nv):
            raise ValueError("bad state shape")
        self._check(_lib().cosenu_batch_set_state(self._h, i, _dptr(a), a.size), "cosenu_batch_set_state")

    def set_clock(self, i: int, t: float, step: int):
        self._check(_lib().cosenu_batch_set_clock(self._h, int(i), float(t), int(step)), "cosenu_batch_set_clock")

    def moments(self, i: int) -> np.ndarray:
        """Instance i's per-row angular moments, shape (nz, 2, 4) (as Sim.moments)."""
        out = np.empty((self.shapes[i][0], 2, 4))
        self._check(_lib().cosenu_batch_moments(self._h, i, _dptr(out), out.size), "cosenu_batch_moments")
        return out

    def get_rows(self, i: int, z0: int, nrows: int) -> np.ndarray:
        """Rows z0 .. z0+nrows-1 (periodic) of instance i, shape (8, nrows, nv)."""
        out = np.empty((8, int(nrows), self.shapes[i][1]))
        self._check(_lib().cosenu_batch_get_rows(self._h, i, int(z0), int(nrows), _dptr(out), out.size),
                    "cosenu_batch_get_rows")
        return out

    def conserved(self, i: int) -> dict:
        c = Conserved()
        rc = _lib().cosenu_batch_conserved(self._h, i, ctypes.byref(c))
        if rc and rc != ENONFINITE:
            self._check(rc, "cosenu_batch_conserved")
        return c.as_dict()

    def info(self, i: int) -> dict:
        inf = Info()
        self._check(_lib().cosenu_batch_info(self._h, i, ctypes.byref(inf)), "cosenu_batch_info")
        return inf.as_dict()

    def time_steps(self, n: int) -> float:
        ms = ctypes.c_double()
        self._check(_lib().cosenu_batch_time_steps(self._h, int(n), ctypes.byref(ms)), "cosenu_batch_time_steps")
        return ms.value

    def autotune(self) -> list:
        """Segment length per kernel variant: 2*k + (nv > 32) for single stages,
        k = 0 FD (KO r <= 2), 1 WENO7, 2 FD (KO r = 3); 6 + vchunks - 1 for
        fused stage pairs; 10 + vchunks - 1 for whole steps; 0 where absent."""
        segs = (ctypes.c_int32 * 14)()
        self._check(_lib().cosenu_batch_autotune(self._h, segs), "cosenu_batch_autotune")
        return list(segs)
