"""Systems properties of the HIP path: bitwise determinism, checkpoint and
resume through get_state/set_state, batched instances equal to the same
instances run alone, stream binding, and detection of a blown-up state."""
import numpy as np
import pytest

from paper_2203_12866_amd import cosenu
from paper_2203_12866_amd import workloads as wl

pytestmark = pytest.mark.gpu


def test_run_twice_bitwise():
    for scheme in (wl.FD_KO, wl.FV_WENO7):
        w = wl.small_fd(5)
        w.update(scheme=scheme)
        outs = []
        for _ in range(2):
            with cosenu.Sim(w) as s:
                s.step(37)
                outs.append(s.get_state())
        assert np.array_equal(outs[0], outs[1])


def test_checkpoint_resume_bitwise():
    for prec in (wl.FP64, wl.FP32_ACC64):
        w = wl.small_fv(6)
        w.update(precision=prec, omega=0.1)
        with cosenu.Sim(w) as a:
            a.step(20)
            full = a.get_state()
            ca = a.conserved()
        with cosenu.Sim(w) as b:
            b.step(10)
            ck = b.get_state()
            t, step = b.info()["t"], b.info()["step"]
        with cosenu.Sim(w) as c:
            c.set_state(ck)
            c.set_clock(t, step)
            c.step(10)
            assert np.array_equal(c.get_state(), full)
            assert c.info()["step"] == 20


def test_get_set_roundtrip_and_clock():
    w = wl.small_fd(1)
    y = wl.random_state(512, 32, seed=3)
    with cosenu.Sim(w) as s:
        s.set_state(y)
        assert np.array_equal(s.get_state(), y)
        s.step(4)
        info = s.info()
        assert info["step"] == 4 and abs(info["t"] - 4 * info["dt"]) < 1e-12
        assert s.conserved()["Pee_nu"] != 0.0


def test_get_rows_is_a_periodic_slab_of_get_state():
    w = wl.small_fd(1)
    y = wl.random_state(512, 32, seed=4)
    with cosenu.Sim(w) as s:
        s.set_state(y)
        s.step(3)
        full = s.get_state()
        for z0, n in ((0, 512), (5, 17), (500, 40), (-3, 9), (1024 + 7, 1), (511, 512)):
            rows = np.arange(z0, z0 + n) % 512
            assert np.array_equal(s.get_rows(z0, n), full[:, rows, :]), (z0, n)
        for z0, n in ((0, 0), (0, 513)):
            with pytest.raises(cosenu.CosenuError):
                s.get_rows(z0, n)


def test_batch_instances_equal_solo_runs():
    ws = []
    for i, (scheme, nz, nv) in enumerate([(0, 300, 32), (1, 257, 64), (0, 190, 100), (1, 64, 16), (0, 1000, 8)]):
        w = wl.small_fd(10 + i)
        w.update(nz=nz, nv=nv, L=0.5 * nz, scheme=scheme, omega=0.05 * i, lam=0.2 * i, alpha=0.8 + 0.03 * i)
        ws.append(w)
    for prec in (wl.FP64, wl.FP32_ACC64):
        for w in ws:
            w["precision"] = prec
        b = cosenu.Batch(ws)
        b.step(9)
        for i, w in enumerate(ws):
            with cosenu.Sim(w) as s:
                s.step(9)
                solo = s.get_state()
            assert np.array_equal(b.get_state(i), solo), (prec, i)
            assert b.info(i)["step"] == 9
        c = b.conserved(3)
        assert c["nonfinite"] == 0
        b.close()


def test_batch_autotune_keeps_states_and_results():
    insts = [dict(wl.small_fd(1), nz=300, nv=128), dict(wl.small_fd(2), nz=97, nv=32, scheme=wl.FV_WENO7),
             dict(wl.small_fd(3), nz=160, nv=256, scheme=wl.FV_WENO7), dict(wl.small_fd(4), nz=64, nv=64)]
    insts = [dict(w, precision=wl.FP32_ACC64) for w in insts]
    with cosenu.Batch(insts) as b:
        b.step(3)
        before = [b.get_state(i) for i in range(len(insts))]
        segs = b.autotune()
        assert all(np.array_equal(b.get_state(i), before[i]) for i in range(len(insts)))
        # WENO7 single stages (nv 32: variant 2, nv 256: 3); FD fused pairs (nv 64: 6, nv 128: 7)
        # or whole steps (10, 11), whichever the tuner found faster per group
        present = [k for k, s in enumerate(segs) if s > 0]
        assert len(segs) == 14 and present[:2] == [2, 3] and len(present) == 4, segs
        assert present[2] in (6, 10) and present[3] in (7, 11), segs
        b.step(7)
        got = [b.get_state(i) for i in range(len(insts))]
    for w, g in zip(insts, got):
        with cosenu.Sim(w) as s:
            s.step(10)
            assert np.array_equal(s.get_state(), g)


def test_torch_stream_binding():
    import torch
    w = wl.small_fd(2)
    with cosenu.Sim(w) as s:
        ref_state = None
        st = torch.cuda.Stream()
        with torch.cuda.stream(st):
            s.bind_torch_stream()
            s.step(5)
        torch.cuda.synchronize()
        s.set_stream(None)
        got = s.get_state()
    with cosenu.Sim(w) as s2:
        s2.step(5)
        ref_state = s2.get_state()
    assert np.array_equal(got, ref_state)


def test_blow_up_is_reported_as_nonfinite():
    """A state with huge values under the FD scheme at cfl = 2 overflows; the
    diagnostics call reports it."""
    w = wl.small_fd(1)
    w.update(nz=64, nv=8, L=10.0, cfl=2.0, ko_eps=0.0)
    y = wl.random_state(64, 8, seed=1, scale=1e150)
    with cosenu.Sim(w) as s:
        s.set_state(y)
        s.step(50)
        with pytest.raises(cosenu.CosenuError) as e:
            s.conserved()
        assert e.value.code == cosenu.ENONFINITE
        assert s.conserved(allow_nonfinite=True)["nonfinite"] > 0


@pytest.mark.parametrize("precision", [wl.FP64, wl.FP32_ACC64])
def test_batch_fused_pairs_parity_and_checkpoint(precision):
    """FD + KO instances with 32 < nv <= 256 run as fused stage pairs inside
    the batch (2, 4, 6 and 8 waves per segment), their state alternating
    between two buffers: odd step counts, reading and restoring a state
    mid-run, and the result after the restore all match solo runs bit for bit."""
    shapes = [(wl.FD_KO, 300, 128), (wl.FD_KO, 100, 256), (wl.FD_KO, 97, 130), (wl.FD_KO, 64, 64),
              (wl.FV_WENO7, 90, 64), (wl.FD_KO, 150, 32), (wl.FD_KO, 5, 64), (wl.FD_KO, 6, 200)]
    ws = []
    for i, (scheme, nz, nv) in enumerate(shapes):
        w = wl.small_fd(30 + i)
        w.update(nz=nz, nv=nv, L=0.6 * nz, scheme=scheme, omega=0.04 * i, lam=0.1 * i, precision=precision)
        ws.append(w)
    solo3, solo8 = [], []
    for w in ws:
        with cosenu.Sim(w) as s:
            s.step(3)
            solo3.append(s.get_state())
            s.step(5)
            solo8.append(s.get_state())
    with cosenu.Batch(ws) as b:
        launches = [b.info(i)["launches_per_step"] for i in range(len(ws))]
        assert launches == [2, 2, 2, 2, 4, 4, 2, 2], launches
        b.step(3)
        mid = [b.get_state(i) for i in range(len(ws))]
        for i in range(len(ws)):
            assert np.array_equal(mid[i], solo3[i]), i
        b.step(5)
        for i in range(len(ws)):
            assert np.array_equal(b.get_state(i), solo8[i]), i
        # restore the step-3 states (the batch now sits at the other parity) and redo
        for i in range(len(ws)):
            b.set_state(i, mid[i])
            b.set_clock(i, 3 * b.info(i)["dt"], 3)
        b.step(1)
        b.step(4)
        assert all(b.info(i)["step"] == 8 for i in range(len(ws)))
        for i in range(len(ws)):
            assert np.array_equal(b.get_state(i), solo8[i]), i
            c = b.conserved(i)
            assert c["nonfinite"] == 0
        # per-instance moments and row slabs (across the periodic seam) as a solo run gives them
        for i, w in enumerate(ws):
            with cosenu.Sim(w) as s:
                s.set_state(solo8[i])
                m_solo = s.moments()
            assert np.array_equal(b.moments(i), m_solo), i
            nz = w["nz"]
            assert np.array_equal(b.get_rows(i, nz - 2, min(nz, 4)), np.roll(solo8[i], 2, axis=1)[:, :min(nz, 4)]), i


def test_degenerate_calls_are_no_ops_or_rejected():
    """Zero steps change nothing; empty, oversized or short requests are
    rejected with EINVAL and leave the handle usable."""
    import ctypes
    w = dict(wl.small_fd(3), nz=40, nv=70, L=30.0, omega=0.1)
    L = cosenu.lib()
    with cosenu.Sim(w) as s:
        s.step(2)
        y = s.get_state()
        info = s.info()
        s.step(0)
        assert s.time_steps(0) >= 0.0
        assert np.array_equal(s.get_state(), y)
        assert (s.info()["step"], s.info()["t"]) == (info["step"], info["t"])
        buf = np.zeros(8 * 41 * 70)
        p = buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        assert L.cosenu_get_rows(s._h, 0, 0, p, buf.size) == cosenu.EINVAL
        assert L.cosenu_get_rows(s._h, 0, 41, p, buf.size) == cosenu.EINVAL
        assert L.cosenu_get_rows(s._h, 0, 3, p, 8 * 3 * 70 - 1) == cosenu.EINVAL
        assert L.cosenu_set_state(s._h, p, 8 * 40 * 70 - 1) == cosenu.EINVAL
        assert L.cosenu_moments(s._h, p, 40 * 8 - 1) == cosenu.EINVAL
        assert L.cosenu_step(s._h, -1) == cosenu.EINVAL
        assert L.cosenu_set_seg_rows(s._h, -1) == cosenu.EINVAL
        assert L.cosenu_set_fusion(s._h, 3) == cosenu.EINVAL and L.cosenu_set_fusion(s._h, -1) == cosenu.EINVAL
        # the handle still works and has not moved
        assert np.array_equal(s.get_rows(-3, 40), np.roll(y, 3, axis=1))
        s.step(1)
        assert s.info()["step"] == info["step"] + 1
    with cosenu.Batch([w, dict(w, nv=16)]) as b:
        b.step(0)
        assert b.info(0)["step"] == 0
        assert L.cosenu_batch_step(b._h, -1) == cosenu.EINVAL
        assert L.cosenu_batch_get_state(b._h, 2, p, buf.size) == cosenu.EINVAL
        assert L.cosenu_batch_get_state(b._h, 0, p, 8 * 40 * 70 - 1) == cosenu.EINVAL


def test_batch_survives_failed_autotune():
    """A task-list rebuild that fails half-way through cosenu_batch_autotune
    (forced from the host) returns an error, and the batch then steps from its
    original launch shapes with step graphs rebuilt: every instance, fused
    pairs and single stages, still equals its solo run bitwise."""
    L = cosenu.lib()
    ws = [dict(wl.small_fd(11), nz=48, nv=70, L=40.0, precision=wl.FP32_ACC64),   # fused pairs
          dict(wl.small_fv(12), nz=33, nv=20, L=30.0, precision=wl.FP32_ACC64),   # WENO7, nv <= 32
          dict(wl.small_fd(13), nz=40, nv=96, L=35.0, precision=wl.FP32_ACC64, ko_order=3)]
    solo = []
    for w in ws:
        with cosenu.Sim(w) as s:
            s.step(5)
            solo.append(s.get_state())
    with cosenu.Batch(ws) as b:
        b.step(2)
        segs0 = [b.info(i)["seg_rows"] for i in range(len(ws))]
        assert L.cosenu_test_inject_failure(3, 2) == 0  # the third rebuild of the tuning loop fails
        try:
            rc = L.cosenu_batch_autotune(b._h, None)
        finally:
            L.cosenu_test_inject_failure(0, 0)
        assert rc == cosenu.EDEVICE
        assert "injected" in L.cosenu_batch_last_error(b._h).decode()
        assert [b.info(i)["seg_rows"] for i in range(len(ws))] == segs0
        b.step(3)
        for i in range(len(ws)):
            assert np.array_equal(b.get_state(i), solo[i]), i
        # a later autotune succeeds and changes nothing in the results
        b.autotune()
        b.step(0)
        for i in range(len(ws)):
            assert np.array_equal(b.get_state(i), solo[i]), i


def test_conserved_quantities_independent_of_launch_shape():
    """The diagnostics reduce over a fixed decomposition with compensated sums,
    so the same state gives the same conserved quantities, bit for bit,
    whatever segment length, workgroup size or path the stage kernels use (a
    drift measured across an autotuning is then the state's, not the sum's)."""
    nz, nv = 1000, 128
    w = dict(wl.small_fd(3), nz=nz, nv=nv, L=100.0, omega=0.05, lam=0.3)
    y0 = wl.random_unit_state(nz, nv, seed=5)
    with cosenu.Sim(w) as s:
        s.set_state(y0)
        ref = s.conserved()
        for seg in (1, 7, 64, nz):
            s.set_seg_rows(seg)
            assert s.conserved() == ref, seg
        s.set_fusion(2)
        assert s.conserved() == ref
        s.autotune()
        assert s.conserved() == ref
