"""FD without Kreiss-Oliger dissipation on the collective setup of Sec. 5
(Fig. collosc_noko_Pi_comparison_cmap): without dissipation the central
differences carry grid-scale modes backwards and faster than light, so
flavour structure appears where causality forbids it and |P| leaves 1; with
KO (eps = 0.1), and with WENO7, nothing propagates outside the light cone.

Measure: the largest |rho_ex| (neutrinos and antineutrinos) at |z| > t + 5
sqrt(W), outside the light cone of the seed eps(z) = 1e-2 exp(-z^2 / W),
W = 50, where the exact solution keeps the seed's Gaussian tail (below 5e-14
from t = 0).  Setup: alpha = 0.9, sigma = 0.6 / 0.5, Nv = 100, C = 0.2 (Sec.
5); the paper gives no L, here L = 2400 so that the cone does not wrap before
t = 1100; Nz = 4000 (dz = 0.6) and 8000 (dz = 0.3).  Measured: without KO the
value grows from ~1e-15 at t = 300 at the same rate at both resolutions
(about e^0.04 t: ~1e-6 at t = 800, ~0.5 at t = 1100, with |P| up to 1.8);
with KO and with WENO7 it stays below 1e-14 throughout."""
import math

import numpy as np
import pytest

from oracle import oracle as o
from paper_2203_12866_amd import cosenu
from paper_2203_12866_amd import workloads as wl

pytestmark = pytest.mark.gpu

W = 50.0
MARGIN = 5.0 * math.sqrt(W)
TIMES = (600.0, 800.0, 1000.0, 1100.0)


def _outside_cone(nz, L, scheme, ko_eps):
    w = dict(wl.small_fd(1), nz=nz, nv=100, L=L, cfl=0.2, pert_amp=1e-2, pert_width=W, phase=0.0, alpha=0.9,
             scheme=scheme, ko_eps=ko_eps)
    z = o.positions(nz, L)
    out, plen = [], []
    with cosenu.Sim(w) as s:
        dt = s.info()["dt"]
        done = 0
        for t in TIMES:
            n = int(round(t / dt))
            s.step(n - done)
            done = n
            y = s.get_state()
            far = np.abs(z) > n * dt + MARGIN
            assert far.any()
            ex = np.maximum(np.hypot(y[2], y[3]), np.hypot(y[6], y[7]))
            out.append(float(ex[far].max()))
            plen.append(float(np.sqrt((y[0] - y[1]) ** 2 + 4 * (y[2] ** 2 + y[3] ** 2)).max()))
    return out, plen


@pytest.mark.parametrize("nz", [4000, 8000])
def test_fd_without_ko_violates_causality(nz):
    L = 2400.0
    noko, p_noko = _outside_cone(nz, L, wl.FD_KO, 0.0)
    ko, p_ko = _outside_cone(nz, L, wl.FD_KO, 0.1)
    weno, p_weno = _outside_cone(nz, L, wl.FV_WENO7, 0.1)
    print(f"dz = {L / nz}: outside the light cone at t = {TIMES}:\n  FD no KO {['%.1e' % x for x in noko]}"
          f" |P|max {['%.3f' % x for x in p_noko]}\n  FD + KO  {['%.1e' % x for x in ko]} "
          f"|P|max {['%.3f' % x for x in p_ko]}\n  WENO7    {['%.1e' % x for x in weno]} "
          f"|P|max {['%.3f' % x for x in p_weno]}")
    # with dissipation (KO) or upwinding (WENO7): nothing outside the cone beyond the seed's tail
    assert max(ko) < 1e-13 and max(weno) < 1e-13
    # without it: growing by orders of magnitude every 200 time units, visible by t = 1000
    assert noko[1] > 100 * noko[0] and noko[2] > 100 * noko[1]
    assert noko[2] > 1e-4 and noko[3] > 1e-2
    # and |P| = 1 is lost far more than with KO (unphysical P beyond unit length)
    assert p_noko[3] > 1.5 and p_noko[3] > p_ko[3] + 0.3
