"""Seeded synthetic workloads: parameter sets and random input states.

This module only draws numbers.  It holds none of the method's arithmetic
(no angular distributions, no initial-data formula, no Hamiltonian): both the
GPU library and the CPU oracle compute those themselves from the parameters
returned here.  Random quantities the method would otherwise draw (the seed
phase of the off-diagonal perturbation, alpha, sigma ...) are drawn here and
passed in as plain parameters.

The workload family is the paper's collective-oscillation setup (Sec. 5):
Gaussian angular distributions g ~ exp(-(v-1)^2 / 2 sigma^2) for neutrinos
and antineutrinos, asymmetry alpha = n_nubar / n_nu, mu = 1, and an
off-diagonal seed eps(z) = amp exp(-z^2 / width) at the centre of a periodic
box.  No public dataset is involved.
"""
from __future__ import annotations

import math

import numpy as np

FD_KO = 0
FV_WENO7 = 1
FP64 = 0
FP32_ACC64 = 1

THETA_37 = 37.0 * math.pi / 180.0


def _base(**kw) -> dict:
    w = dict(nz=512, nv=32, L=400.0, cfl=0.4, mu=1.0, omega=0.0, theta=THETA_37, lam=0.0,
             alpha=0.9, sigma_nu=0.6, sigma_nubar=0.5, pert_amp=1e-6, pert_width=50.0,
             phase=0.0, scheme=FD_KO, precision=FP64, ko_eps=0.1, weno_eps=1e-6, steps=100,
             ko_order=2, quadrature=0)
    w.update(kw)
    return w


def _phase(rng: np.random.Generator) -> float:
    return float(rng.uniform(0.0, 2.0 * math.pi))


def small_fd(seed: int = 1) -> dict:
    """FD + Kreiss-Oliger, 512 x 32 cells, L = 400, 100 steps, FP64 (the oracle-sized case)."""
    rng = np.random.default_rng(seed)
    return _base(name="fd_ko_512x32", phase=_phase(rng))


def small_fv(seed: int = 1) -> dict:
    """The finite-volume WENO7 twin of the small FD case."""
    w = small_fd(seed)
    w.update(name="fv_weno7_512x32", scheme=FV_WENO7)
    return w


def small_full_h(seed: int = 1, scheme: int = FD_KO) -> dict:
    """Small case with vacuum and matter terms switched on."""
    w = small_fd(seed)
    w.update(name="full_h_512x32", omega=0.05, lam=0.3, scheme=scheme)
    return w


def fd_16384x128(seed: int = 2, precision: int = FP64) -> dict:
    """FD + KO, 16384 x 128 cells, L = 1600, 2000 steps; alpha drawn in [0.8, 1.0]."""
    rng = np.random.default_rng(seed)
    phase = _phase(rng)
    alpha = float(rng.uniform(0.8, 1.0))
    return _base(name="fd_ko_16384x128", nz=16384, nv=128, L=1600.0, steps=2000, alpha=alpha,
                 phase=phase, precision=precision)


def fv_65536x256(seed: int = 3, precision: int = FP64) -> dict:
    """FV WENO7, 65536 x 256 cells, L = 6400, omega = 1e-3, lambda = 0, 5000 steps."""
    rng = np.random.default_rng(seed)
    phase = _phase(rng)
    alpha = float(rng.uniform(0.8, 1.0))
    return _base(name="fv_weno7_65536x256", nz=65536, nv=256, L=6400.0, steps=5000, alpha=alpha,
                 omega=1e-3, phase=phase, scheme=FV_WENO7, precision=precision)


def fv_1m_x512(seed: int = 5, precision: int = FP32_ACC64) -> dict:
    """FV WENO7, 2^20 x 512 cells, L = 1e5, omega = 1e-3, lambda = 10, 1000 steps."""
    rng = np.random.default_rng(seed)
    phase = _phase(rng)
    alpha = float(rng.uniform(0.8, 1.0))
    return _base(name="fv_weno7_1048576x512", nz=1 << 20, nv=512, L=1e5, steps=1000, alpha=alpha,
                 omega=1e-3, lam=10.0, phase=phase, scheme=FV_WENO7, precision=precision)


def batch_64(seed: int = 4, n: int = 64, nz_min: int = 2048, nz_max: int = 32768,
             nvs=(32, 64, 128, 256), dz: float = 0.09765625) -> list:
    """64 independent uneven instances: Nz log-uniform, Nv from a set, scheme,
    alpha, sigmas, omega and lambda drawn per instance; same dz for all."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        nz = int(round(math.exp(rng.uniform(math.log(nz_min), math.log(nz_max)))))
        nv = int(rng.choice(nvs))
        scheme = int(rng.integers(0, 2))
        alpha = float(rng.uniform(0.8, 1.0))
        s_nu = float(rng.uniform(0.4, 0.8))
        s_nb = float(rng.uniform(0.3, s_nu))
        omega = 0.0 if rng.uniform() < 0.5 else float(math.exp(rng.uniform(math.log(1e-4), math.log(1e-2))))
        lam = 0.0 if rng.uniform() < 0.5 else float(rng.uniform(0.0, 10.0))
        out.append(_base(name=f"batch[{i}]", nz=nz, nv=nv, L=nz * dz, scheme=scheme, alpha=alpha,
                         sigma_nu=s_nu, sigma_nubar=s_nb, omega=omega, lam=lam, phase=_phase(rng),
                         precision=FP32_ACC64, steps=1000))
    return out


# ---------------------------------------------------------------------------
# random states for property and parity tests
# ---------------------------------------------------------------------------
def random_state(nz: int, nv: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """Arbitrary real planes (8, nz, nv), uniform in [-scale, scale]."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.uniform(-scale, scale, size=(8, nz, nv)))


def random_unit_state(nz: int, nv: int, seed: int) -> np.ndarray:
    """Planes of density matrices with unit trace and a unit-length random
    polarisation vector in every cell, for neutrinos and antineutrinos."""
    rng = np.random.default_rng(seed)
    y = np.empty((8, nz, nv))
    for base in (0, 4):
        p = rng.normal(size=(3, nz, nv))
        p /= np.sqrt((p * p).sum(axis=0))
        # rho = (1 + P.sigma)/2 : ee = (1+P3)/2, xx = (1-P3)/2, ex = (P1 - i P2)/2
        y[base + 0] = 0.5 * (1.0 + p[2])
        y[base + 1] = 0.5 * (1.0 - p[2])
        y[base + 2] = 0.5 * p[0]
        y[base + 3] = -0.5 * p[1]
    return np.ascontiguousarray(y)


def smooth_offdiag_state(nz: int, nv: int, seed: int, amp: float, modes: int = 3) -> np.ndarray:
    """rho = rhobar = diag(1, 0) plus a small smooth periodic off-diagonal made
    of a few random Fourier modes per velocity bin; rhobar_ex = conj(rho_ex)."""
    rng = np.random.default_rng(seed)
    z = np.arange(nz) / nz
    s = np.zeros((nz, nv), dtype=complex)
    for m in range(1, modes + 1):
        c = (rng.normal(size=nv) + 1j * rng.normal(size=nv)) / m
        s += np.exp(2j * math.pi * m * z)[:, None] * c[None, :]
        c2 = (rng.normal(size=nv) + 1j * rng.normal(size=nv)) / m
        s += np.exp(-2j * math.pi * m * z)[:, None] * c2[None, :]
    s *= amp / np.abs(s).max()
    y = np.zeros((8, nz, nv))
    y[0] = 1.0
    y[4] = 1.0
    y[2] = s.real
    y[3] = s.imag
    y[6] = s.real
    y[7] = -s.imag
    return np.ascontiguousarray(y)
