"""Parity at the full sizes of the benchmark workloads, in the launch
configuration bench.py times (autotuned segment length).

* FD + KO, 16384 x 128: after 150 GPU steps from the initial data, one more
  GPU step is compared with one oracle step from the same (downloaded)
  state, over the whole grid.
* Over the workloads' full lengths (FD 2000 steps, WENO7 5000 steps, into
  flavour conversion), the FP32 form against the FP64 form: off-diagonals
  within 1e-5 relative while the FD run stays linear, angle-averaged survival
  probabilities within 1e-6 once WENO7 is nonlinear, and the drift of every
  conserved quantity within 10x the FP64 form's (with a floor of a few
  hundred FP64 ulps).
* FV WENO7, 65536 x 256 (omega = 1e-3): one step of the oracle on periodic
  z-slabs cut from the GPU state with a 16-row margin (4 stages x 4 rows of
  WENO7 halo) is compared with the GPU step on the slab interiors, at the
  perturbation, at the periodic seam and at a random place.
"""
import numpy as np
import pytest

from oracle import oracle as o
from paper_2203_12866_amd import cosenu
from paper_2203_12866_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _one_step_pair(w, warm_steps):
    with cosenu.Sim(w) as s:
        s.autotune()
        s.step(warm_steps)
        y0 = s.get_state()
        s.step(1)
        y1 = s.get_state()
        dt = s.info()["dt"]
    return y0, y1, dt


@pytest.mark.parametrize("prec", [wl.FP64, wl.FP32_ACC64])
def test_fd_16384x128_one_step_full_grid(prec):
    w = wl.fd_16384x128(2, prec)
    y0, y1, dt = _one_step_pair(w, 150)
    p = o.problem_from_workload(w)
    assert abs(p.dt - dt) < 1e-15
    ref = o.rk4(p, y0, 1)
    err = np.abs(y1 - ref)
    print(f"precision {prec}: max abs {err.max():.3e}")
    if prec == wl.FP64:
        assert err.max() <= 1e-12
    else:
        # FP32 stencils on FP32-rounded stage values: one step moves every value by
        # at most ~dt * |k| with k rounded at ~6e-8 relative
        assert err.max() <= 1e-7
    assert np.abs(ref[2:4] - y0[2:4]).max() > 0  # the perturbation moved


@pytest.mark.parametrize("prec", [wl.FP64, wl.FP32_ACC64])
def test_fv_65536x256_windows(prec):
    w = wl.fv_65536x256(3, prec)
    nz, nv = w["nz"], w["nv"]
    y0, y1, dt = _one_step_pair(w, 40)
    margin, width = 16, 48
    rng = np.random.default_rng(0)
    starts = [nz // 2 - width // 2, 0, int(rng.integers(0, nz))]
    for a in starts:
        rows = np.arange(a - margin, a + width + margin) % nz
        slab = np.ascontiguousarray(y0[:, rows, :])
        p = o.problem_from_workload(dict(w, nz=len(rows), L=len(rows) * (w["L"] / nz)))
        p.dt = dt
        ref = o.rk4(p, slab, 1)[:, margin:margin + width, :]
        got = y1[:, rows[margin:margin + width], :]
        err = np.abs(got - ref).max()
        print(f"precision {prec}, window at {a}: max abs {err:.3e}")
        assert err <= (1e-12 if prec == wl.FP64 else 1e-7), (a, err)


def test_fv_1048576x512_windows_fp32acc():
    """The 2^20 x 512 WENO7 case (omega = 1e-3, lambda = 10) in its FP32 form,
    checked on periodic slabs fetched with get_rows: one oracle step on the
    slab against the GPU step on the slab interior, at the perturbation, at the
    periodic seam and at a random place."""
    w = wl.fv_1m_x512(5, wl.FP32_ACC64)
    nz = w["nz"]
    margin, width = 16, 32
    rng = np.random.default_rng(1)
    starts = [nz // 2 - width // 2, nz - width // 2, int(rng.integers(0, nz))]
    with cosenu.Sim(w) as s:
        s.autotune()
        s.step(10)
        slabs = [s.get_rows(a - margin, width + 2 * margin) for a in starts]
        s.step(1)
        outs = [s.get_rows(a, width) for a in starts]
        dt = s.info()["dt"]
    for a, slab, got in zip(starts, slabs, outs):
        p = o.problem_from_workload(dict(w, nz=width + 2 * margin, L=(width + 2 * margin) * (w["L"] / nz)))
        assert abs(p.dt - dt) < 1e-15
        ref = o.rk4(p, slab, 1)[:, margin:margin + width, :]
        err = np.abs(got - ref).max()
        print(f"window at {a}: max abs {err:.3e}")
        assert err <= 1e-7, (a, err)
        assert np.isfinite(got).all()


def _full_run(w):
    with cosenu.Sim(w) as s:
        s.autotune()
        c0 = s.conserved()
        s.step(w["steps"])
        c1 = s.conserved()
        y = s.get_state()
    scale = abs(c0["N_nu"]) + abs(c0["N_nubar"])
    keys = ["N_nu", "N_nubar"]
    d = [abs(c1[k] - c0[k]) for k in keys] + [abs(c1["M0"][0] - c0["M0"][0])]
    if w["omega"] == 0.0:
        d.append(abs(c1["M0"][3] - c0["M0"][3]))
    if w["lam"] == 0.0:
        d.append(abs(c1["B_dot_M0"] - c0["B_dot_M0"]))
    return y, c1, max(d) / scale


@pytest.mark.parametrize("which", ["fd_16384x128", "fv_65536x256"])
def test_fp32_form_tracks_fp64_over_full_run(which):
    mk = wl.fd_16384x128 if which == "fd_16384x128" else wl.fv_65536x256
    y64, c64, d64 = _full_run(mk(precision=wl.FP64))
    y32, c32, d32 = _full_run(mk(precision=wl.FP32_ACC64))
    rel_off = float(np.abs(y32[2:4] - y64[2:4]).max() / np.abs(y64[2:4]).max())
    print(f"{which}: steps {c64['step']}, Pee {c64['Pee_nu']:.10f} / {c32['Pee_nu']:.10f}, "
          f"offdiag rel {rel_off:.2e}, drift FP64 {d64:.2e} FP32 {d32:.2e}")
    assert c32["nonfinite"] == 0 and c64["nonfinite"] == 0
    if which == "fd_16384x128":
        assert c64["Pee_nu"] > 1 - 1e-9              # still linear
        assert rel_off <= 1e-5
    else:
        assert c64["Pee_nu"] < 0.9                     # flavour conversion has set in
    assert abs(c32["Pee_nu"] - c64["Pee_nu"]) < 1e-6 and abs(c32["Pee_nubar"] - c64["Pee_nubar"]) < 1e-6
    assert d64 < 1e-12
    assert d32 <= max(10 * d64, 500 * 2.2e-16)
