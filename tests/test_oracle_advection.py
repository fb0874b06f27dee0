"""Pins of the oracle's advection operators and RK4 integrator (mu = omega =
lambda = 0, so H = 0 and every component is advected independently).

* FD4 + Kreiss-Oliger is a linear, shift-invariant scheme: one RK4 step
  multiplies Fourier mode theta = k dz by G = sum_{n<=4} (dt L)^n / n! with
  L = -i v (8 sin th - sin 2th)/(6 dz) - (eps/dz) sin^(2r)(th/2).  The oracle
  must reproduce FFT^-1[G^n FFT(u0)] to rounding (any data, any r).
* In the linear-weight limit (amplitude so small that every smoothness
  indicator is far below epsilon) the WENO7 scheme is linear too, with the
  interface weights of eq:f7 (golden fixture) on the upwind side.
* On smooth profiles the measured orders are the ones the paper states
  (Sec. 4.1): 7 for FV WENO7, 4 for central FD without dissipation; adding
  Kreiss-Oliger (eps = 0.1) lowers FD to third order.
"""
import math

import numpy as np
import pytest

from oracle import oracle as o
from tests.golden.fixtures import key_values, weno7_linear_coefficients


def advect_problem(nz, nv, L, dt, scheme, ko_eps=0.1, ko_r=2):
    return o.Problem(nz=nz, nv=nv, L=L, dt=dt, mu=0.0, omega=0.0, theta=0.3, lam=0.0, alpha=0.9,
                     scheme=scheme, ko_eps=ko_eps, ko_r=ko_r, weno_eps=1e-6,
                     g_nu=np.ones(nv), g_nubar=np.ones(nv))


def spectral_evolve(u0, symbol, dt, nsteps):
    """u0: (nz,) real; symbol(theta) -> complex semi-discrete eigenvalue."""
    nz = u0.shape[0]
    theta = 2.0 * math.pi * np.fft.fftfreq(nz)
    z = dt * symbol(theta)
    G = 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24
    return np.fft.ifft(G ** nsteps * np.fft.fft(u0)).real


@pytest.mark.parametrize("ko_eps,ko_r", [(0.0, 2), (0.1, 2), (0.3, 1), (0.2, 3)])
def test_fd_ko_matches_fourier_propagator(ko_eps, ko_r):
    nz, nv, L = 48, 4, 30.0
    dz = L / nz
    dt = 0.37 * dz
    steps = 25
    y0 = np.random.default_rng(3).uniform(-1, 1, size=(8, nz, nv))
    p = advect_problem(nz, nv, L, dt, o.FD_KO, ko_eps, ko_r)
    y = o.rk4(p, y0, steps)
    v = o.velocities(nv)
    for c in range(8):
        for j in range(nv):
            sym = lambda th: (-1j * v[j] * (8 * np.sin(th) - np.sin(2 * th)) / (6 * dz)
                              - (ko_eps / dz) * np.sin(th / 2) ** (2 * ko_r))
            expect = spectral_evolve(y0[c, :, j], sym, dt, steps)
            np.testing.assert_allclose(y[c, :, j], expect, rtol=0, atol=2e-13)


def test_fv_weno7_linear_limit_matches_fourier_propagator():
    cf = weno7_linear_coefficients()
    nz, nv, L = 40, 4, 20.0
    dz = L / nz
    dt = 0.3 * dz
    steps = 20
    amp = 1e-12
    y0 = amp * np.random.default_rng(4).uniform(-1, 1, size=(8, nz, nv))
    p = advect_problem(nz, nv, L, dt, o.FV_WENO7)
    y = o.rk4(p, y0, steps)
    v = o.velocities(nv)
    for c in range(8):
        for j in range(nv):
            if v[j] > 0:
                sym = lambda th: -(v[j] / dz) * (1 - np.exp(-1j * th)) * sum(
                    float(cf[m]) * np.exp(1j * m * th) for m in range(-3, 4))
            else:
                sym = lambda th: -(v[j] / dz) * (np.exp(1j * th) - 1) * sum(
                    float(cf[m]) * np.exp(-1j * m * th) for m in range(-3, 4))
            expect = spectral_evolve(y0[c, :, j], sym, dt, steps)
            np.testing.assert_allclose(y[c, :, j], expect, rtol=0, atol=1e-10 * amp)


def _advection_error(nz, scheme, ko_eps, dt, T, amp=1.0):
    L, nv = 1.0, 2  # v = -0.5, +0.5
    p = advect_problem(nz, nv, L, dt, scheme, ko_eps)
    z = o.positions(nz, L)
    prof = lambda x: amp * np.exp(np.sin(2 * math.pi * x / L))
    y0 = np.zeros((8, nz, nv))
    y0[0, :, 1] = prof(z)
    y0[0, :, 0] = prof(z)
    nsteps = int(round(T / dt))
    y = o.rk4(p, y0, nsteps)
    t = nsteps * dt
    errs = []
    for j, v in ((0, -0.5), (1, 0.5)):
        exact = prof(z - v * t)
        errs.append(math.sqrt(np.mean((y[0, :, j] - exact) ** 2)))  # E_2 of eq:E2
    return max(errs)


def test_convergence_orders_match_paper():
    orders = key_values("advection_orders.txt")
    T = 0.5
    # FV WENO7 at a time step small enough that the RK4 error stays below the
    # spatial one.  The asymptotic regime of WENO is the one where every
    # smoothness indicator has fallen below epsilon (SI ~ dz^2 -> 0); a small
    # amplitude reaches it at sizes the oracle finishes quickly.  At O(1)
    # amplitude the same grids are pre-asymptotic (nonlinear weights active
    # near the critical points of the profile) and show order ~6.
    dt = 0.05 * (1.0 / 64) / 0.5
    e = [_advection_error(n, o.FV_WENO7, 0.0, dt, T, amp=1e-4) for n in (16, 32, 64)]
    fv_order = math.log2(e[1] / e[2])
    assert abs(fv_order - orders["fv_weno7"]) < 0.4, (e, fv_order)
    e1 = [_advection_error(n, o.FV_WENO7, 0.0, dt, T) for n in (32, 64)]
    assert 5.0 < math.log2(e1[0] / e1[1]) < 7.5
    # central FD without dissipation: fourth order
    dt = 0.1 * (1.0 / 128) / 0.5
    e = [_advection_error(n, o.FD_KO, 0.0, dt, T) for n in (32, 64, 128)]
    fd_order = math.log2(e[1] / e[2])
    assert abs(fd_order - orders["fd_central"]) < 0.3, (e, fd_order)
    # Kreiss-Oliger with eps = 0.1 adds an O(dz^3) term: larger errors, third order
    e_ko = [_advection_error(n, o.FD_KO, 0.1, dt, T) for n in (64, 128)]
    assert e_ko[1] > e[2]
    assert abs(math.log2(e_ko[0] / e_ko[1]) - 3.0) < 0.3, e_ko
