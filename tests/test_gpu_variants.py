"""Parity of the discretisation variants (Sec. 3.1) with the FP64 CPU oracle,
through the C ABI: the Kreiss-Oliger order r = 1, 2, 3 (and no dissipation)
of the FD scheme, and the vertex grid with the trapezoid or Simpson rule for
both schemes.

Bars as for the fiducial variant: FP64 form within 1e-12 max-abs of the
oracle, FP32 form within 1e-5 relative in the linear regime.  Every variant
also runs through the fused stage pairs (where they apply: FD with r <= 2),
several launch shapes and the batch, each bit for bit equal to the plain
single-stage path.
"""
import numpy as np
import pytest

from oracle import oracle as o
from paper_2203_12866_amd import cosenu
from paper_2203_12866_amd import workloads as wl

pytestmark = pytest.mark.gpu


def run_gpu(w, steps, state=None, seg=None, fusion=None):
    with cosenu.Sim(w) as s:
        if fusion is not None:
            s.set_fusion(fusion)
        if seg:
            s.set_seg_rows(seg)
        if state is not None:
            s.set_state(state)
        s.step(steps)
        return s.get_state(), s.info()


def run_oracle(w, steps, state=None):
    p = o.problem_from_workload(w)
    y0 = o.initial_state_for(w) if state is None else state
    return o.rk4(p, y0, steps)


def maxabs(a, b):
    return float(np.abs(a - b).max())


@pytest.mark.parametrize("r,ko_eps", [(1, 0.1), (3, 0.1), (2, 0.0), (1, 0.4), (3, 0.3)])
def test_ko_order_fp64_matches_oracle_after_100_steps(r, ko_eps):
    w = wl.small_full_h(1, wl.FD_KO)
    w.update(ko_order=r, ko_eps=ko_eps)
    got, _ = run_gpu(w, 100)
    ref = run_oracle(w, 100)
    err = maxabs(got, ref)
    print(f"KO r={r} eps={ko_eps}: max|gpu-oracle| = {err:.3e}")
    assert err <= 1e-12, err


KO3_SHAPES = [(7, 2), (7, 65), (77, 5), (61, 100), (130, 129), (333, 32), (200, 256)]


@pytest.mark.parametrize("nz,nv", KO3_SHAPES)
def test_ko3_ragged_shapes_nonlinear_state(nz, nv):
    w = wl.small_fd(7)
    w.update(nz=nz, nv=nv, L=0.8 * nz, omega=0.3, lam=0.7, alpha=0.85, ko_order=3, ko_eps=0.3)
    y0 = wl.random_unit_state(nz, nv, seed=nz + nv)
    got, _ = run_gpu(w, 12, state=y0)
    ref = run_oracle(w, 12, state=y0)
    err = maxabs(got, ref)
    print(f"KO3 {nz}x{nv}: {err:.3e}")
    assert err <= 1e-12, err


@pytest.mark.parametrize("r", [1, 3])
def test_ko_order_independent_of_launch_shape(r):
    w = wl.small_fd(3)
    w.update(nz=203, nv=96, L=150.0, omega=0.2, lam=0.1, ko_order=r, ko_eps=0.2)
    y0 = wl.random_unit_state(203, 96, seed=5)
    base, info = run_gpu(w, 6, state=y0, fusion=False)
    assert info["launches_per_step"] == 4
    for seg in (1, 3, 8, 64, 203):
        got, _ = run_gpu(w, 6, state=y0, seg=seg, fusion=False)
        assert np.array_equal(got, base), seg
    fused, info = run_gpu(w, 6, state=y0, fusion=True)
    # stage pairs are fused for r <= 2 only; r = 3 keeps four launches
    assert info["launches_per_step"] == (2 if r == 1 else 4)
    assert np.array_equal(fused, base)
    assert maxabs(base, run_oracle(w, 6, state=y0)) <= 1e-12


@pytest.mark.parametrize("r", [1, 3])
def test_ko_order_fp32_form_linear_regime(r):
    w = wl.small_fd(1)
    w.update(ko_order=r, precision=wl.FP32_ACC64)
    got, _ = run_gpu(w, 100)
    ref = run_oracle(w, 100)
    for sl in (slice(0, 2), slice(2, 4), slice(4, 6), slice(6, 8)):
        rel = float(np.abs(got[sl] - ref[sl]).max() / np.abs(ref[sl]).max())
        assert rel <= 1e-5, (r, sl, rel)


QUADS = [(o.QUAD_TRAPEZOID, 32), (o.QUAD_SIMPSON, 33)]


@pytest.mark.parametrize("quad,nv", QUADS)
@pytest.mark.parametrize("scheme", [wl.FD_KO, wl.FV_WENO7])
def test_quadrature_fp64_matches_oracle_after_100_steps(quad, nv, scheme):
    w = wl.small_full_h(1, scheme)
    w.update(nv=nv, quadrature=quad)
    got, info = run_gpu(w, 100)
    ref = run_oracle(w, 100)
    err = maxabs(got, ref)
    print(f"quadrature {quad} scheme {scheme}: max|gpu-oracle| = {err:.3e}")
    assert err <= 1e-12, err
    assert abs(info["dv"] - 2.0 / (nv - 1)) < 1e-16
    assert abs(info["dt"] - w["cfl"] * w["L"] / w["nz"]) < 1e-15  # max|v| = 1 on the vertex grid
    assert maxabs(ref[2:4], o.initial_state_for(w)[2:4]) > 1e-8


@pytest.mark.parametrize("quad,nv,scheme", [(o.QUAD_SIMPSON, 129, wl.FV_WENO7), (o.QUAD_TRAPEZOID, 100, wl.FD_KO),
                                            (o.QUAD_SIMPSON, 65, wl.FD_KO), (o.QUAD_TRAPEZOID, 7, wl.FV_WENO7)])
def test_quadrature_ragged_nonlinear_and_diagnostics(quad, nv, scheme):
    nz = 61
    w = wl.small_fd(5)
    w.update(nz=nz, nv=nv, L=50.0, scheme=scheme, omega=0.3, lam=0.4, alpha=0.85, quadrature=quad, ko_order=3)
    y0 = wl.random_unit_state(nz, nv, seed=nv)
    p = o.problem_from_workload(w)
    with cosenu.Sim(w) as s:
        s.set_state(y0)
        s.step(8)
        y = s.get_state()
        m = s.moments()
        c = s.conserved()
    assert maxabs(y, o.rk4(p, y0, 8)) <= 1e-12
    np.testing.assert_allclose(m, o.moments(p, y), rtol=0, atol=1e-13)
    d = o.diagnostics(p, y)
    for k, name in enumerate(("M0_trace", "M0_x", "M0_y", "M0_z")):
        assert abs(c["M0"][k] - d[name]) < 1e-11
    for key in ("N_nu", "N_nubar", "dP_max", "dP_mean", "ee_nu", "ee_nubar", "B_dot_M0"):
        assert abs(c[key] - d[key]) < 1e-11 * max(1.0, abs(d[key])), key


@pytest.mark.parametrize("quad,nv", [(o.QUAD_TRAPEZOID, 128), (o.QUAD_SIMPSON, 129)])
def test_quadrature_fused_pairs_equal_single_stages(quad, nv):
    w = wl.small_fd(4)
    w.update(nz=300, nv=nv, L=200.0, omega=0.1, lam=0.2, quadrature=quad)
    y0 = wl.random_unit_state(300, nv, seed=3)
    single, _ = run_gpu(w, 7, state=y0, fusion=False)
    fused, info = run_gpu(w, 7, state=y0, fusion=True)
    assert info["launches_per_step"] == 2
    assert np.array_equal(fused, single)


def test_quadrature_fp32_form_linear_regime_and_drift():
    for quad, nv, scheme in ((o.QUAD_TRAPEZOID, 32, wl.FD_KO), (o.QUAD_SIMPSON, 33, wl.FV_WENO7)):
        w = wl.small_fd(1)
        w.update(nv=nv, quadrature=quad, scheme=scheme, precision=wl.FP32_ACC64)
        got, _ = run_gpu(w, 100)
        ref = run_oracle(w, 100)
        for sl in (slice(0, 2), slice(2, 4), slice(4, 6), slice(6, 8)):
            rel = float(np.abs(got[sl] - ref[sl]).max() / np.abs(ref[sl]).max())
            assert rel <= 1e-5, (quad, sl, rel)
        # omega = lambda = 0: M0 and N are exact invariants under any rule
        with cosenu.Sim(w) as s:
            s.set_state(wl.random_unit_state(w["nz"], nv, seed=1))
            c0 = s.conserved()
            s.step(100)
            c1 = s.conserved()
        scale = abs(c0["N_nu"]) + abs(c0["N_nubar"])
        drift = max(abs(c1["M0"][k] - c0["M0"][k]) for k in range(4)) / scale
        assert drift < 200 * 2.2e-16, drift


def test_batch_mixes_every_variant():
    """KO r = 1, 2, 3 and both rules in one batch: each instance advances
    bit for bit as it does alone (six kernel variants, fused pairs among them)."""
    specs = [(wl.FD_KO, 300, 32, 3, 0), (wl.FD_KO, 190, 100, 3, 1), (wl.FV_WENO7, 257, 65, 2, 2),
             (wl.FD_KO, 120, 64, 1, 0), (wl.FD_KO, 77, 16, 2, 2), (wl.FV_WENO7, 64, 16, 2, 1)]
    ws = []
    for i, (scheme, nz, nv, r, quad) in enumerate(specs):
        w = wl.small_fd(20 + i)
        if quad == o.QUAD_SIMPSON and nv % 2 == 0:
            nv += 1
        w.update(nz=nz, nv=nv, L=0.5 * nz, scheme=scheme, omega=0.05 * i, lam=0.1 * i, ko_order=r, quadrature=quad)
        ws.append(w)
    for prec in (wl.FP64, wl.FP32_ACC64):
        for w in ws:
            w["precision"] = prec
        with cosenu.Batch(ws) as b:
            b.step(5)
            segs = b.autotune()
            b.step(4)
            present = [k for k, s in enumerate(segs) if s > 0]
            assert present[:5] == [0, 2, 3, 4, 5] and len(present) == 6 and present[5] in (6, 10), segs
            for i, w in enumerate(ws):
                with cosenu.Sim(w) as s:
                    s.set_fusion(False)
                    s.step(9)
                    assert np.array_equal(b.get_state(i), s.get_state()), (prec, i)


MANY_BINS = [(wl.FD_KO, 513, 17, wl.FP64, o.QUAD_MIDPOINT), (wl.FV_WENO7, 700, 13, wl.FP64, o.QUAD_TRAPEZOID),
             (wl.FD_KO, 1100, 10, wl.FP32_ACC64, o.QUAD_MIDPOINT), (wl.FV_WENO7, 1089, 11, wl.FP32_ACC64, o.QUAD_SIMPSON)]


@pytest.mark.parametrize("scheme,nv,nz,prec,quad", MANY_BINS)
def test_many_bins_more_than_16_moment_parts(scheme, nv, nz, prec, quad):
    """nv > 512: a row has more than 16 moment parts (one per 64-bin chunk and
    species), which the kernels sum in a copy of their own.  Against the oracle
    from a random nonlinear state; bitwise the same at every launch shape and
    inside a batch."""
    w = wl.small_fd(9)
    w.update(nz=nz, nv=nv, L=0.7 * nz, scheme=scheme, precision=prec, quadrature=quad, omega=0.2, lam=0.3,
             alpha=0.9)
    y0 = wl.random_unit_state(nz, nv, seed=nv)
    print(f"many bins: scheme {scheme} nv {nv} nz {nz} form {prec} quadrature {quad}", flush=True)
    got, info = run_gpu(w, 3, state=y0)
    assert info["launches_per_step"] == 4
    err = maxabs(got, run_oracle(w, 3, state=y0))
    assert err <= (1e-12 if prec == wl.FP64 else 1e-5), err
    for seg in (1, 4, nz):
        alt, _ = run_gpu(w, 3, state=y0, seg=seg)
        assert np.array_equal(alt, got), seg
    with cosenu.Batch([w]) as b:
        b.set_state(0, y0)
        b.step(3)
        assert np.array_equal(b.get_state(0), got)
