"""The whole RK4 step in one launch (FD + KO, 32 < nv <= 256, nz >= 16): the
four stages march each segment together, with Y2, Y3, Y4 and acc kept on chip.
It must reproduce four single stages (and the fused pairs) bit for bit, for
both forms, ragged segments, a segment covering the whole periodic grid, the
minimum nz, both directions of march, odd step counts, switches between paths
and checkpoints; moments and diagnostics included."""
import numpy as np
import pytest

from oracle import oracle as o
from paper_2203_12866_amd import cosenu
from paper_2203_12866_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _run(w, y0, steps, fusion, seg=None):
    with cosenu.Sim(w) as s:
        s.set_fusion(fusion)
        if seg is not None:
            s.set_seg_rows(seg)
        s.set_state(y0)
        s.step(steps)
        return s.get_state(), s.moments(), s.conserved(), s.info()


@pytest.mark.parametrize("precision", [wl.FP64, wl.FP32_ACC64])
@pytest.mark.parametrize("nz,nv,seg", [(512, 128, 16), (300, 100, 7), (77, 65, 13), (16, 64, 16), (40, 33, 40),
                                       (130, 128, 64), (130, 256, 32)])
def test_whole_step_equals_single_stages_bitwise(precision, nz, nv, seg):
    w = dict(wl.small_fd(7), nz=nz, nv=nv, L=nz * 0.78125, omega=0.05, lam=0.3, precision=precision)
    y0 = wl.random_unit_state(nz, nv, seed=nz + nv + 1)
    a, ma, ca, ia = _run(w, y0, 9, 2, seg)
    b, mb, cb, ib = _run(w, y0, 9, 0, seg)
    c, mc, cc, ic = _run(w, y0, 9, 1, seg)
    print(f"nz={nz} nv={nv} seg={seg}: launches per step {ia['launches_per_step']}, bytes/step {ia['bytes_per_step']:.3e}")
    if nv <= 128:
        assert ia["launches_per_step"] == 1
        assert ia["bytes_per_step"] == 128.0 * nz * nv
    assert ib["launches_per_step"] == 4 and ic["launches_per_step"] == 2
    assert np.array_equal(a, b) and np.array_equal(a, c)
    assert np.array_equal(ma, mb) and np.array_equal(ma, mc)
    assert ca == cb == cc


@pytest.mark.parametrize("precision", [wl.FP64, wl.FP32_ACC64])
def test_whole_step_independent_of_segment_length(precision):
    nz, nv = 256, 128
    w = dict(wl.small_fd(8), nz=nz, nv=nv, L=200.0, precision=precision)
    y0 = wl.random_unit_state(nz, nv, seed=3)
    ref = _run(w, y0, 6, 0)[0]
    for seg in (1, 3, 8, 33, 100, 256):
        got, _, _, info = _run(w, y0, 6, 2, seg)
        assert info["launches_per_step"] == 1
        assert np.array_equal(got, ref), seg


def test_whole_step_matches_oracle_fp64():
    nz, nv = 96, 128
    w = dict(wl.small_fd(9), nz=nz, nv=nv, L=75.0, omega=0.05, lam=0.3)
    y0 = wl.random_unit_state(nz, nv, seed=11)
    y, _, _, info = _run(w, y0, 20, 2)
    assert info["launches_per_step"] == 1
    ref = o.rk4(o.problem_from_workload(w), y0, 20)
    err = float(np.abs(y - ref).max())
    print(f"max |gpu - oracle| after 20 whole steps: {err:.2e}")
    assert err <= 1e-12


def test_whole_step_fiducial_linear_run_fp32_form():
    """The 512 x 128 linear run from the paper's initial data (A = 1e-6) in the
    FP32 form: the whole-step path against the single stages, bitwise, and
    against the FP64 oracle within the form's 1e-5 per component group."""
    w = dict(wl.small_fd(4), nz=512, nv=128, L=400.0, precision=wl.FP32_ACC64)
    with cosenu.Sim(w) as s:
        y0 = s.get_state()
    y, _, _, info = _run(w, y0, 100, 2)
    assert info["launches_per_step"] == 1
    assert np.array_equal(y, _run(w, y0, 100, 0)[0])
    ref = o.rk4(o.problem_from_workload(dict(w, precision=wl.FP64)), y0, 100)
    for grp in ([0, 1, 4, 5], [2, 3, 6, 7]):
        rel = float(np.abs(y[grp] - ref[grp]).max() / np.abs(ref[grp]).max())
        print(f"component group {grp}: relative error {rel:.2e}")
        assert rel <= 1e-5


def test_switching_paths_mid_run_and_checkpoint():
    nz, nv = 200, 128
    w = dict(wl.small_fd(5), nz=nz, nv=nv, L=156.25, omega=0.05, lam=0.3, precision=wl.FP32_ACC64)
    y0 = wl.random_unit_state(nz, nv, seed=21)
    ref, mref, _, _ = _run(w, y0, 14, 0)
    with cosenu.Sim(w) as s:
        s.set_state(y0)
        s.set_fusion(2)
        s.step(3)            # odd: the state and its moments sit in the second buffers
        s.set_fusion(1)
        s.step(1)
        s.set_fusion(2)
        s.step(5)
        s.set_fusion(0)
        s.step(2)
        s.set_fusion(2)
        s.step(1)
        mid = s.get_state()
        assert np.array_equal(s.get_rows(nz - 3, 7), mid[:, np.arange(nz - 3, nz + 4) % nz, :])
        s.step(2)
        assert np.array_equal(s.get_state(), ref)
        assert np.array_equal(s.moments(), mref)
    with cosenu.Sim(w) as s:
        s.set_fusion(2)
        s.set_state(mid)
        s.step(2)
        assert np.array_equal(s.get_state(), ref)


def test_time_stages_and_autotune_keep_results():
    nz, nv = 700, 128
    w = dict(wl.small_fd(8), nz=nz, nv=nv, L=500.0, omega=0.05, lam=0.2, precision=wl.FP64)
    y0 = wl.random_unit_state(nz, nv, seed=21)
    ref, mref, cref, _ = _run(w, y0, 10, 0)
    with cosenu.Sim(w) as s:
        s.set_fusion(2)
        s.set_state(y0)
        s.step(3)
        ms = s.time_stages(2)     # eager, one launch per step: the state moves twice
        assert ms[0] > 0 and ms[1] == 0
        before, m_before = s.get_state(), s.moments()
        seg = s.autotune()        # may pick any path
        print(f"autotune chose seg {seg}, {s.info()['launches_per_step']} launch(es) per step")
        assert np.array_equal(s.get_state(), before)
        assert np.array_equal(s.moments(), m_before)
        s.step(5)
        assert np.array_equal(s.get_state(), ref)
        assert np.array_equal(s.moments(), mref)
        assert s.conserved() == cref


@pytest.mark.parametrize("shape", [dict(nz=15, nv=64), dict(nz=64, nv=32), dict(nz=64, nv=128, ko_order=3),
                                   dict(nz=64, nv=128, scheme=wl.FV_WENO7)])
def test_unsupported_shapes_fall_back(shape):
    w = dict(wl.small_fd(1), L=50.0, **shape)
    with cosenu.Sim(w) as s:
        s.set_fusion(2)
        launches = s.info()["launches_per_step"]
    expect = 2 if shape.get("nz") == 15 else 4
    assert launches == expect
