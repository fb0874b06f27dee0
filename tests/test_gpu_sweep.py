"""A seeded sweep over the options that combine: scheme, form, Kreiss-Oliger
order, velocity grid, shape (ragged rows and bins, tiny grids), launch shape
and path (single stages, fused stage pairs, the whole step in one launch,
where the shape allows them), each case against the FP64 oracle from a
random nonlinear state.
Bars as everywhere: FP64 form within 1e-12 max-abs, FP32 form within 1e-5
max-abs (the state is O(1) and a few steps are taken)."""
import numpy as np
import pytest

from oracle import oracle as o
from paper_2203_12866_amd import cosenu
from paper_2203_12866_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _cases(n=96, seed=2026):
    rng = np.random.default_rng(seed)
    rng_path = np.random.default_rng(seed + 1)  # the path: 0 single stages, 1 fused pairs, 2 whole step
    out = []
    for i in range(n):
        scheme = int(rng.integers(0, 2))
        quad = int(rng.integers(0, 3))
        nv = int(rng.choice([2, 3, 5, 8, 17, 31, 32, 33, 47, 64, 65, 100, 128, 129, 140, 192, 256]))
        if quad == o.QUAD_SIMPSON and nv % 2 == 0:
            nv += 1
        r = int(rng.integers(1, 4))
        nzmin = 9 if scheme == wl.FV_WENO7 else max(5, 2 * r + 1)
        nz = int(rng.integers(nzmin, 160))
        precision = int(rng.integers(0, 2))
        seg = int(rng.choice([0, 1, 2, 5, 13, 64]))
        rng.integers(0, 2)  # a draw the earlier two-path version took here; kept so the other draws stay put
        fusion = int(rng_path.integers(0, 3))
        out.append(dict(i=i, scheme=scheme, quad=quad, nv=nv, nz=nz, ko_order=r, precision=precision, seg=seg,
                        fusion=fusion, steps=int(rng.integers(1, 6)),
                        omega=float(rng.uniform(0, 0.5)), lam=float(rng.uniform(0, 1.0)),
                        alpha=float(rng.uniform(0.5, 1.1)), ko_eps=float(rng.choice([0.0, 0.1, 0.3])),
                        cfl=float(rng.uniform(0.1, 0.6))))
    return out


@pytest.mark.parametrize("case", _cases(), ids=lambda c: f"case{c['i']}")
def test_option_sweep_against_oracle(case):
    c = case
    w = wl.small_fd(100 + c["i"])
    w.update(nz=c["nz"], nv=c["nv"], L=0.7 * c["nz"], scheme=c["scheme"], precision=c["precision"],
             ko_order=c["ko_order"], quadrature=c["quad"], omega=c["omega"], lam=c["lam"], alpha=c["alpha"],
             ko_eps=c["ko_eps"], cfl=c["cfl"])
    print(f"case {c}", flush=True)
    y0 = wl.random_unit_state(c["nz"], c["nv"], seed=1000 + c["i"])
    with cosenu.Sim(w) as s:
        s.set_fusion(c["fusion"])
        if c["seg"]:
            s.set_seg_rows(c["seg"])
        s.set_state(y0)
        s.step(c["steps"])
        got = s.get_state()
        info = s.info()
    p = o.problem_from_workload(w)
    assert abs(info["dt"] - p.dt) <= 1e-15 * p.dt
    ref = o.rk4(p, y0, c["steps"])
    err = float(np.abs(got - ref).max())
    tol = 1e-12 if c["precision"] == wl.FP64 else 1e-5
    assert err <= tol, (err, c)
