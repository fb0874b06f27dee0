"""Pins of the oracle's alternative velocity grids (Sec. 3.1): nv vertices
v_j = -1 + j dv spanning [-1, 1] with the composite trapezoid rule, or with
the composite Simpson rule (nv odd), in place of the midpoint bins.

* The weights are those of scipy's own trapezoid and Simpson routines (the
  oracle's sums against scipy on random integrands).
* Exactness and order: the trapezoid rule integrates linear functions
  exactly and converges as dv^2, Simpson's rule integrates cubics exactly and
  converges as dv^4; the angular distributions are normalised by the rule, so
  their normalisation constant converges to the Gaussian's exact integral at
  those rates.
* The rule reaches every velocity sum: moments and diagnostics are the stated
  weighted sums, the exact discrete invariants still hold, and the
  linear-regime evolution matches an eigen prediction whose coupling matrix
  is built from scipy's weights.
"""
import math

import numpy as np
import pytest
from scipy.integrate import simpson, trapezoid
from scipy.special import erf

from oracle import oracle as o
from paper_2203_12866_amd import workloads as wl
from tests.test_oracle_collective import _linear_prediction_general


def scipy_weights(nv, quad):
    v = np.linspace(-1.0, 1.0, nv)
    rule = trapezoid if quad == o.QUAD_TRAPEZOID else simpson
    return np.array([rule(np.eye(nv)[l], x=v) for l in range(nv)])


@pytest.mark.parametrize("quad,nv", [(o.QUAD_TRAPEZOID, 2), (o.QUAD_TRAPEZOID, 8), (o.QUAD_TRAPEZOID, 33),
                                     (o.QUAD_SIMPSON, 3), (o.QUAD_SIMPSON, 9), (o.QUAD_SIMPSON, 65)])
def test_vertex_grid_and_weights_match_scipy(quad, nv):
    v = o.velocities(nv, quad)
    np.testing.assert_allclose(v, np.linspace(-1.0, 1.0, nv), rtol=0, atol=1e-15)
    assert v[0] == -1.0 and v[-1] == 1.0
    w = o.vweights(nv, quad)
    np.testing.assert_allclose(w, scipy_weights(nv, quad), rtol=1e-14, atol=0)
    rng = np.random.default_rng(nv)
    f = rng.normal(size=nv)
    rule = trapezoid if quad == o.QUAD_TRAPEZOID else simpson
    assert abs(np.dot(w, f) - rule(f, x=v)) < 1e-14 * np.abs(f).sum()
    # dt = CFL dz / max|v| with max|v| = 1 on the vertex grid
    assert abs(o.dt_from_cfl(64, nv, 32.0, 0.4, quad) - 0.4 * 0.5) < 1e-15


def test_midpoint_weights_are_dv():
    for nv in (1, 6, 32):
        np.testing.assert_allclose(o.vweights(nv), np.full(nv, 2.0 / nv), rtol=0, atol=0)


def test_exactness_degrees():
    for nv in (3, 7, 21):
        v, wt, ws = o.velocities(nv, o.QUAD_TRAPEZOID), o.vweights(nv, o.QUAD_TRAPEZOID), o.vweights(nv, o.QUAD_SIMPSON)
        for k in range(6):
            exact = (1.0 - (-1.0) ** (k + 1)) / (k + 1)
            if k <= 1:
                assert abs(np.dot(wt, v ** k) - exact) < 1e-14
            if k <= 3:
                assert abs(np.dot(ws, v ** k) - exact) < 1e-14
        # and not beyond: v^2 under the trapezoid rule, v^4 under Simpson's
        assert abs(np.dot(wt, v ** 2) - 2.0 / 3.0) > 1e-3 / nv ** 2
        assert abs(np.dot(ws, v ** 4) - 2.0 / 5.0) > 1e-3 / nv ** 4


def test_normalisation_converges_at_the_rules_orders():
    """g_j = f_j / Q[f]: the recovered Q[f] tends to the Gaussian's integral
    sigma sqrt(pi/2) erf(sqrt(2)/sigma) as dv^2 (trapezoid) and dv^4 (Simpson)."""
    sigma = 0.6
    exact = sigma * math.sqrt(math.pi / 2) * erf(math.sqrt(2.0) / sigma)
    for quad, order in ((o.QUAD_TRAPEZOID, 2), (o.QUAD_SIMPSON, 4), (o.QUAD_MIDPOINT, 2)):
        errs = []
        for n in (8, 16, 32, 64):
            nv = n + 1 if quad != o.QUAD_MIDPOINT else n
            g = o.angular_dist(nv, sigma, quad)
            v = o.velocities(nv, quad)
            f = np.exp(-(v - 1.0) ** 2 / (2 * sigma ** 2))
            assert abs(np.dot(o.vweights(nv, quad), g) - 1.0) < 1e-14
            errs.append(abs(f[-1] / g[-1] - exact))
        rates = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
        assert all(abs(r - order) < 0.15 for r in rates[1:]), (quad, rates)


@pytest.mark.parametrize("quad,nv", [(o.QUAD_TRAPEZOID, 6), (o.QUAD_SIMPSON, 7)])
def test_moments_and_diagnostics_carry_the_weights(quad, nv):
    nz, L, alpha, theta = 7, 3.5, 0.83, 0.4
    y = wl.random_state(nz, nv, seed=9)
    g, gb = o.angular_dist(nv, 0.6, quad), o.angular_dist(nv, 0.45, quad)
    p = o.Problem(nz=nz, nv=nv, L=L, dt=0.1, alpha=alpha, theta=theta, g_nu=g, g_nubar=gb, quad=quad)
    v, w, dz = np.linspace(-1, 1, nv), scipy_weights(nv, quad), L / nz
    D = {0: g * y[0] - alpha * gb * y[4], 1: g * y[1] - alpha * gb * y[5]}
    Dex = g * (y[2] + 1j * y[3]) - alpha * gb * np.conj(y[6] + 1j * y[7])
    m = o.moments(p, y)
    for q, arr in ((0, D[0]), (1, D[1]), (2, Dex.real), (3, Dex.imag)):
        np.testing.assert_allclose(m[:, 0, q], (w * arr).sum(axis=1), rtol=1e-13, atol=1e-14)
        np.testing.assert_allclose(m[:, 1, q], (w * v * arr).sum(axis=1), rtol=1e-13, atol=1e-14)
    d = o.diagnostics(p, y)
    assert abs(d["M0_trace"] - dz * (w * (D[0] + D[1])).sum()) < 1e-13
    assert abs(d["M0_z"] - dz * (w * (D[0] - D[1])).sum()) < 1e-13
    assert abs(d["M0_x"] - dz * (w * 2 * Dex.real).sum()) < 1e-13
    assert abs(d["N_nubar"] - dz * (w * gb * (y[4] + y[5])).sum()) < 1e-13
    assert abs(d["ee_nu"] - dz * (w * g * y[0]).sum()) < 1e-13
    P = np.sqrt((2 * y[2]) ** 2 + (2 * y[3]) ** 2 + (y[0] - y[1]) ** 2)
    dPm = (w * g * np.abs(P - 1)).sum() / (nz * (w * g).sum())
    assert abs(d["dP_mean"] - dPm) < 1e-13


@pytest.mark.parametrize("quad,nv", [(o.QUAD_TRAPEZOID, 8), (o.QUAD_SIMPSON, 9)])
@pytest.mark.parametrize("scheme", [o.FD_KO, o.FV_WENO7])
def test_invariants_with_vertex_grid(quad, nv, scheme):
    nz, L = 20, 14.0
    p = o.Problem(nz=nz, nv=nv, L=L, dt=0.35 * (L / nz), mu=1.0, alpha=0.87, scheme=scheme,
                  g_nu=o.angular_dist(nv, 0.6, quad), g_nubar=o.angular_dist(nv, 0.5, quad), quad=quad)
    y0 = wl.random_unit_state(nz, nv, seed=17)
    d0 = o.diagnostics(p, y0)
    y = o.rk4(p, y0, 12)
    d1 = o.diagnostics(p, y)
    tol = 1e-13 * L * 2
    for k in ("N_nu", "N_nubar", "M0_trace", "M0_x", "M0_y", "M0_z"):
        assert abs(d1[k] - d0[k]) < tol, k


@pytest.mark.parametrize("quad,nv", [(o.QUAD_TRAPEZOID, 16), (o.QUAD_SIMPSON, 17)])
@pytest.mark.parametrize("scheme", [o.FD_KO, o.FV_WENO7])
def test_linear_regime_with_vertex_grid(quad, nv, scheme):
    nz, L, mu, alpha, steps = 32, 2 * math.pi / 0.16, 1.0, 0.9, 250
    g, gb = o.angular_dist(nv, 0.6, quad), o.angular_dist(nv, 0.5, quad)
    dt = 0.4 * (L / nz)
    y0 = wl.smooth_offdiag_state(nz, nv, seed=3, amp=1e-9, modes=4)
    p = o.Problem(nz=nz, nv=nv, L=L, dt=dt, mu=mu, alpha=alpha, scheme=scheme, ko_eps=0.1,
                  g_nu=g, g_nubar=gb, quad=quad)
    y = o.rk4(p, y0, steps)
    S0 = y0[2] + 1j * y0[3]
    v = np.linspace(-1.0, 1.0, nv)
    pred = _linear_prediction_general(S0, v, scipy_weights(nv, quad), L, dt, steps, mu, alpha, g, gb, scheme, 0.1)
    got = y[2] + 1j * y[3]
    assert np.abs(pred).max() / np.abs(S0).max() > 10.0
    err = np.abs(got - pred).max() / np.abs(pred).max()
    assert err < 1e-11, err
