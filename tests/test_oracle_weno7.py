"""Pins of the oracle's WENO7 reconstruction (Appendix A) against facts fixed
by the paper and by the mathematics, not by the oracle's own formulas:

* the printed linear seventh-order reconstruction eq:f7 (golden fixture) is
  what the nonlinear scheme reduces to when every smoothness indicator is far
  below the regulator epsilon;
* each candidate is the exact interface value of the cubic with the given
  cell averages, and eq:f7 is exact for polynomials up to degree six;
* each smoothness indicator is 240 times the Jiang-Shu indicator (sum over
  derivatives 1..3 of the squared derivative integrated over the target cell,
  in cell units), computed here from a polynomial fit;
* the ENO property near a jump, and homogeneity / odd symmetry.
"""
import numpy as np
import pytest
from numpy.polynomial import polynomial as Pn

from oracle import oracle as o
from tests.golden.fixtures import weno7_linear_coefficients

OFFS = list(range(-3, 4))
SUBSTENCILS = [(0, 1, 2, 3), (-1, 0, 1, 2), (-2, -1, 0, 1), (-3, -2, -1, 0)]


def cell_averages(coeffs, offsets):
    """Exact averages of the polynomial sum_n c_n xi^n over [k-1/2, k+1/2]."""
    I = Pn.polyint(coeffs)
    return np.array([Pn.polyval(k + 0.5, I) - Pn.polyval(k - 0.5, I) for k in offsets])


def fit_cubic(offsets, values):
    A = np.zeros((4, 4))
    for r, k in enumerate(offsets):
        for n in range(4):
            A[r, n] = ((k + 0.5) ** (n + 1) - (k - 0.5) ** (n + 1)) / (n + 1)
    return np.linalg.solve(A, values)


def jiang_shu_beta(c):
    b = 0.0
    for l in range(1, 4):
        d = Pn.polyder(c, l)
        I = Pn.polyint(Pn.polymul(d, d))
        b += Pn.polyval(0.5, I) - Pn.polyval(-0.5, I)
    return b


def test_linear_limit_is_eq_f7():
    """Tiny amplitude: SI << eps, the weights are the linear ones and the
    result must be the printed seventh-order combination eq:f7."""
    cf = weno7_linear_coefficients()
    rng = np.random.default_rng(11)
    for _ in range(20):
        a = rng.normal(size=7) * 1e-14  # SI ~ 1e-24: relative weight change ~ 1e-18
        expect = sum(float(cf[m]) * a[m + 3] for m in OFFS)
        got = o.weno7_minus(a, 1e-6)
        assert abs(got - expect) <= 1e-13 * np.abs(a).max(), (got, expect)


def test_eq_f7_fixture_is_consistent():
    """The golden coefficients themselves: they sum to one and reproduce the
    interface value of every polynomial of degree <= 6 (exact arithmetic)."""
    from fractions import Fraction
    cf = weno7_linear_coefficients()
    assert sum(cf.values()) == 1
    for n in range(7):
        # average of xi^n over [k-1/2, k+1/2] in exact fractions
        avg = {k: (Fraction(2 * k + 1, 2) ** (n + 1) - Fraction(2 * k - 1, 2) ** (n + 1)) / (n + 1) for k in OFFS}
        assert sum(cf[k] * avg[k] for k in OFFS) == Fraction(1, 2) ** n


@pytest.mark.parametrize("deg", [0, 1, 2, 3])
def test_candidates_exact_for_cubics(deg):
    """Every candidate reconstructs a cubic exactly; so does the nonlinear
    combination, whatever the weights (O(1) amplitude)."""
    rng = np.random.default_rng(deg)
    c = rng.normal(size=deg + 1)
    a = cell_averages(c, OFFS)
    exact = Pn.polyval(0.5, c)
    q, si, w = o.weno7_parts(a, 1e-6)
    np.testing.assert_allclose(q, exact, rtol=0, atol=1e-12)
    assert abs(o.weno7_minus(a, 1e-6) - exact) < 1e-12


@pytest.mark.parametrize("deg", [4, 5, 6])
def test_seventh_order_exact_in_linear_limit(deg):
    rng = np.random.default_rng(100 + deg)
    c = rng.normal(size=deg + 1) * 1e-16  # values <= 1e-13: SI << eps
    a = cell_averages(c, OFFS)
    exact = Pn.polyval(0.5, c)
    assert abs(o.weno7_minus(a, 1e-6) - exact) < 1e-12 * np.abs(a).max()


def test_smoothness_indicators_are_240_jiang_shu():
    rng = np.random.default_rng(7)
    for _ in range(50):
        a = rng.normal(size=7)
        q, si, w = o.weno7_parts(a, 1e-6)
        for r, st in enumerate(SUBSTENCILS):
            c = fit_cubic(st, np.array([a[k + 3] for k in st]))
            beta = jiang_shu_beta(c)
            assert abs(si[r] - 240.0 * beta) <= 1e-9 * max(1.0, abs(si[r])), (r, si[r], 240 * beta)
            # candidate = interface value of the same cubic
            assert abs(q[r] - Pn.polyval(0.5, c)) <= 1e-12 * max(1.0, np.abs(a).max())


def test_weights_use_regulated_inverse_square():
    """w_r proportional to d_r / (SI_r + eps)^2 with d from eq:f7: checked by
    the ratio of weights for data whose SI are known (constant data: SI = 0,
    w_r = d_r / eps^2, and d_r are the unique weights giving eq:f7)."""
    cf = weno7_linear_coefficients()
    # d_r from the two end coefficients and the two-stencil equations
    d0 = float(cf[3]) / (1.0 / 12.0)
    d3 = float(cf[-3]) / (-3.0 / 12.0)
    q, si, w = o.weno7_parts(np.full(7, 2.5), 1e-6)
    assert np.all(si == 0.0)
    np.testing.assert_allclose(w[0] * 1e-12, d0, rtol=1e-14)
    np.testing.assert_allclose(w[3] * 1e-12, d3, rtol=1e-14)
    np.testing.assert_allclose(w.sum() * 1e-12, 1.0, rtol=1e-14)
    # a linear profile: all SI equal 240 slope^2, weights stay proportional to d
    a = 0.3 * np.arange(-3, 4)
    q, si, w = o.weno7_parts(a, 1e-6)
    np.testing.assert_allclose(si, 240.0 * 0.09, rtol=1e-13)
    np.testing.assert_allclose(w * (240 * 0.09 + 1e-6) ** 2, [d0, w[1] * (240 * 0.09 + 1e-6) ** 2, w[2] * (240 * 0.09 + 1e-6) ** 2, d3], rtol=1e-13)


def test_eno_property_at_jump():
    """A jump between i+1 and i+2: only S_2 and S_3 avoid it; their weights
    must dominate and the result must be close to their candidates."""
    a = np.array([0, 0, 0, 0, 0, 1, 1], dtype=float)
    q, si, w = o.weno7_parts(a, 1e-6)
    wn = w / w.sum()
    assert wn[0] + wn[1] < 1e-10
    assert abs(o.weno7_minus(a) - 0.0) < 1e-10


def test_symmetries():
    rng = np.random.default_rng(5)
    a = rng.normal(size=7)
    f = o.weno7_minus(a, 1e-6)
    assert o.weno7_minus(-a, 1e-6) == -f
    s = 7.0
    assert abs(o.weno7_minus(s * a, s * s * 1e-6) - s * f) < 1e-13 * s
    assert o.weno7_minus(a + 0.0, 1e-6) == f
