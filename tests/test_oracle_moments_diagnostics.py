"""Pins of the oracle's angular moments and of its error measures, against
things other than the oracle's own sums:

* eq:ham has the separable kernel (1 - v v'), so the self-interaction
  Hamiltonian of bin j is mu (M0 - v_j M1) with M0, M1 the weighted velocity
  moments of D = g rho - alpha gbar rhobar^* (and Hbar_nunu = -mu (M0 - v_j M1)^*).
  The moments that oracle_moments returns, assembled that way with numpy's
  complex 2x2 matrices, must give the commutator that oracle_rhs forms from its
  literal O(nv) quadrature of eq:ham for every (z, v).  oracle_rhs itself is
  pinned by an independent numpy transcription (test_oracle_hamiltonian), so a
  wrong sign or conjugation in the moments fails here.
* dP = |P| - 1 (Sec. 5): states built from polarisation vectors of known
  length s (axis-aligned, dyadic s, so |P| = s exactly) give
  dP_max = max |s - 1| exactly, with the maximum placed in a neutrino or an
  antineutrino cell, above or below one.
* Homogeneous precession at mu = 0: one RK4 step of dP/dt = B x P is the
  degree-4 Taylor polynomial R of exp(dt [B x]) (a closed form built here in
  numpy), so after n steps every bin's vector is R^n P_j.  The g-weighted mean
  <dP>, dP_max and the flavour contents ee_nu, ee_nubar of the oracle's
  diagnostics must equal the same measures of those closed-form vectors.
"""
import math

import numpy as np
import pytest

from oracle import oracle as o
from paper_2203_12866_amd import workloads as wl


def _velocities(nv, quad):
    if quad == o.QUAD_MIDPOINT:
        return -1.0 + (np.arange(nv) + 0.5) * (2.0 / nv)
    return np.linspace(-1.0, 1.0, nv)


def _to_matrices(y, base):
    """(nz, nv, 2, 2) complex density matrices from the real planes."""
    m = np.zeros(y.shape[1:] + (2, 2), dtype=complex)
    m[..., 0, 0] = y[base]
    m[..., 1, 1] = y[base + 1]
    m[..., 0, 1] = y[base + 2] + 1j * y[base + 3]
    m[..., 1, 0] = y[base + 2] - 1j * y[base + 3]
    return m


def _commutator_from_moments(mom, y, v, mu, flip_im=False):
    """-i [H, rho] and -i [Hbar, rhobar] per cell with H = mu (M0 - v M1) built
    from the moment array [nz][2][4] (q = ee, xx, Re ex, Im ex)."""
    nz, nv = y.shape[1:]
    rho, rhob = _to_matrices(y, 0), _to_matrices(y, 4)
    out = np.zeros((8, nz, nv))
    sgn = -1.0 if flip_im else 1.0
    for z in range(nz):
        for j in range(nv):
            q = mom[z, 0] - v[j] * mom[z, 1]
            H = mu * np.array([[q[0], q[2] + 1j * sgn * q[3]], [q[2] - 1j * sgn * q[3], q[1]]])
            Hb = -np.conj(H)
            for base, r, HH in ((0, rho[z, j], H), (4, rhob[z, j], Hb)):
                c = -1j * (HH @ r - r @ HH)
                out[base:base + 4, z, j] = (c[0, 0].real, c[1, 1].real, c[0, 1].real, c[0, 1].imag)
    return out


@pytest.mark.parametrize("quad,nv", [(o.QUAD_MIDPOINT, 6), (o.QUAD_TRAPEZOID, 6), (o.QUAD_SIMPSON, 7)])
@pytest.mark.parametrize("scheme", [o.FD_KO, o.FV_WENO7])
def test_moments_reproduce_direct_integral(quad, nv, scheme):
    rng = np.random.default_rng(101 + nv + 7 * quad + 3 * scheme)
    nz, mu, alpha = 11, 1.3, 0.83
    # z-dependent random Hermitian states with rhobar unrelated to rho^*, so
    # that every part of D (and the conjugation of rhobar) matters
    y = wl.random_state(nz, nv, seed=int(rng.integers(1 << 30)), scale=0.7)
    g, gb = rng.uniform(0.1, 1.0, nv), rng.uniform(0.1, 1.0, nv)
    # a large dz keeps the advection part of the right-hand side small; it is
    # removed by subtracting the right-hand side at mu = 0 (where H = 0 and
    # the commutator vanishes exactly)
    p1 = o.Problem(nz=nz, nv=nv, L=50.0 * nz, dt=0.1, mu=mu, omega=0.0, theta=0.3, lam=0.0, alpha=alpha,
                   scheme=scheme, g_nu=g, g_nubar=gb, quad=quad)
    p0 = o.Problem(nz=nz, nv=nv, L=50.0 * nz, dt=0.1, mu=0.0, omega=0.0, theta=0.3, lam=0.0, alpha=alpha,
                   scheme=scheme, g_nu=g, g_nubar=gb, quad=quad)
    direct = o.rhs(p1, y) - o.rhs(p0, y)
    mom = o.moments(p1, y)
    v = _velocities(nv, quad)
    via_moments = _commutator_from_moments(mom, y, v, mu)
    np.testing.assert_allclose(via_moments, direct, rtol=0, atol=2e-14)
    # the check is sensitive: a sign error on Im D_ex in the moments would fail it
    wrong = _commutator_from_moments(mom, y, v, mu, flip_im=True)
    assert np.abs(wrong - direct).max() > 1e-2


def _axis_state(nz, nv, s, axis, sign):
    """Planes with unit trace and P = sign * s * e_axis in every cell
    (s, axis, sign of shape (2, nz, nv): species 0 the neutrino's own vector,
    species 1 the antineutrino's)."""
    y = np.zeros((8, nz, nv))
    for sp, base in ((0, 0), (1, 4)):
        P = np.zeros((3, nz, nv))
        for a in range(3):
            P[a] = np.where(axis[sp] == a, sign[sp] * s[sp], 0.0)
        y[base + 0] = 0.5 * (1.0 + P[2])
        y[base + 1] = 0.5 * (1.0 - P[2])
        y[base + 2] = 0.5 * P[0]
        y[base + 3] = -0.5 * P[1]
    return y


@pytest.mark.parametrize("where", ["nubar_below_one", "nu_above_one", "nu_below_one", "nubar_above_one"])
def test_dP_max_is_exact_on_vectors_of_known_length(where):
    nz, nv = 13, 5
    rng = np.random.default_rng(7)
    # lengths 1 + k/64 with |k| <= 3: exact in binary, and so are their squares
    s = 1.0 + rng.integers(-3, 4, size=(2, nz, nv)) / 64.0
    axis = rng.integers(0, 3, size=(2, nz, nv))
    sign = rng.choice([-1.0, 1.0], size=(2, nz, nv))
    sp = 1 if where.startswith("nubar") else 0
    big = 1.0 - 5.0 / 64.0 if where.endswith("below_one") else 1.0 + 5.0 / 64.0
    s[sp, 8, 3] = big  # the one cell of largest deviation
    y = _axis_state(nz, nv, s, axis, sign)
    p = o.Problem(nz=nz, nv=nv, L=3.0, dt=0.1, alpha=0.8, g_nu=o.angular_dist(nv, 0.6),
                  g_nubar=o.angular_dist(nv, 0.5))
    d = o.diagnostics(p, y)
    assert d["dP_max"] == 5.0 / 64.0
    # <dP> covers the neutrinos only: sum_j w g_j | s - 1 | / sum_j w g_j
    g = o.angular_dist(nv, 0.6)
    want = (g[None, :] * np.abs(s[0] - 1.0)).sum() / (nz * g.sum())
    assert abs(d["dP_mean"] - want) < 1e-15
    assert d["nonfinite"] == 0


def _rk4_propagator(B, dt):
    X = np.array([[0, -B[2], B[1]], [B[2], 0, -B[0]], [-B[1], B[0], 0]])
    hA = dt * X
    R, term = np.eye(3), np.eye(3)
    for n in range(1, 5):
        term = term @ hA / n
        R = R + term
    return R


@pytest.mark.parametrize("quad,nv", [(o.QUAD_MIDPOINT, 6), (o.QUAD_TRAPEZOID, 7)])
def test_diagnostics_follow_homogeneous_precession(quad, nv):
    nz, L, omega, theta, lam, dt, steps = 5, 4.0, 0.9, 0.61, 0.35, 0.4, 30
    rng = np.random.default_rng(17 + nv)
    # per bin and species: a random direction of length s_j (not one, so that
    # dP is not zero), the same in every z row
    y0 = np.zeros((8, nz, nv))
    P0 = {}
    for base in (0, 4):
        n = rng.normal(size=(3, nv))
        n /= np.sqrt((n * n).sum(axis=0))
        s = rng.uniform(0.9, 1.1, nv)
        P = n * s
        P0[base] = P
        y0[base + 0] = 0.5 * (1.0 + P[2])[None, :]
        y0[base + 1] = 0.5 * (1.0 - P[2])[None, :]
        y0[base + 2] = 0.5 * P[0][None, :]
        y0[base + 3] = -0.5 * P[1][None, :]
    y0 = np.ascontiguousarray(y0)
    g, gb = o.angular_dist(nv, 0.6, quad), o.angular_dist(nv, 0.45, quad)
    p = o.Problem(nz=nz, nv=nv, L=L, dt=dt, mu=0.0, omega=omega, theta=theta, lam=lam, alpha=0.8,
                  scheme=o.FD_KO, g_nu=g, g_nubar=gb, quad=quad)
    y = o.rk4(p, y0, steps)
    d = o.diagnostics(p, y)
    Bvac = omega * np.array([math.sin(2 * theta), 0.0, -math.cos(2 * theta)])
    ez = np.array([0.0, 0.0, 1.0])
    Pn = {0: np.linalg.matrix_power(_rk4_propagator(Bvac + lam * ez, dt), steps) @ P0[0],
          4: np.linalg.matrix_power(_rk4_propagator(Bvac - lam * ez, dt), steps) @ P0[4]}
    w = o.vweights(nv, quad)
    dPn = np.abs(np.sqrt((Pn[0] ** 2).sum(axis=0)) - 1.0)
    dPb = np.abs(np.sqrt((Pn[4] ** 2).sum(axis=0)) - 1.0)
    assert abs(d["dP_max"] - max(dPn.max(), dPb.max())) < 1e-14
    assert abs(d["dP_mean"] - (w * g * dPn).sum() / (w * g).sum()) < 1e-14
    # ee = dz sum w g rho_ee over the whole box = L sum_j w_j g_j (1 + P3_j)/2
    assert abs(d["ee_nu"] - L * (w * g * 0.5 * (1.0 + Pn[0][2])).sum()) < 1e-13
    assert abs(d["ee_nubar"] - L * (w * gb * 0.5 * (1.0 + Pn[4][2])).sum()) < 1e-13
    # the traces are untouched by the precession
    assert abs(d["N_nu"] - L * (w * g).sum()) < 1e-13
    assert abs(d["N_nubar"] - L * (w * gb).sum()) < 1e-13
