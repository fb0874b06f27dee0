"""Host-side pieces of bench.py (no GPU): the one-GPU refusal, the tie of the
counter figures to the kernel source they were taken on, the VALU-issue
roofline arithmetic and the FP32-versus-FP64 comparison."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


@pytest.fixture
def fake_root(tmp_path, monkeypatch):
    """bench.py pointed at a copy of the kernel source and a profiles folder of
    the test's own."""
    src = os.path.join(tmp_path, bench.KERNEL_SOURCES[0])
    os.makedirs(os.path.dirname(src))
    with open(os.path.join(ROOT, bench.KERNEL_SOURCES[0]), "rb") as f, open(src, "wb") as g:
        g.write(f.read())
    os.makedirs(os.path.join(tmp_path, "profiles"))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    return tmp_path


def _write_profile(root, sha, entries):
    with open(os.path.join(root, "profiles", "hbm_traffic.json"), "w") as f:
        json.dump({"kernel_sha": sha, "entries": entries}, f)


def test_traffic_is_tied_to_the_kernel_source(fake_root):
    e = {"w/fp32acc": {"bytes_per_launch": 1.5e9, "valu_insts_per_launch": 6.144e8}}
    _write_profile(fake_root, bench.kernel_hash(), e)
    assert bench.measured_traffic("w", "fp32acc") == 1.5e9
    assert bench.measured_traffic("w", "fp64") is None  # no entry
    # a change to the kernel source voids the committed counters
    with open(os.path.join(fake_root, bench.KERNEL_SOURCES[0]), "ab") as f:
        f.write(b"\n// changed\n")
    assert bench.measured_traffic("w", "fp32acc") is None
    assert bench.alu_roofline("w", "fp32acc", 1e-3) is None


def test_missing_or_broken_profile_gives_none(fake_root):
    assert bench.measured_traffic("w", "fp32acc") is None
    with open(os.path.join(fake_root, "profiles", "hbm_traffic.json"), "w") as f:
        f.write("{not json")
    assert bench.measured_traffic("w", "fp32acc") is None


def test_valu_roofline_arithmetic(fake_root):
    # 6.144e8 wave instructions in 1 ms is 614.4 G/s: the whole chip's issue rate
    _write_profile(fake_root, bench.kernel_hash(), {"w/fp32acc": {"valu_insts_per_launch": 6.144e8}})
    a = bench.alu_roofline("w", "fp32acc", 1e-3)
    assert a["peak"] == pytest.approx(614.4)
    assert a["achieved"] == pytest.approx(614.4)
    assert a["frac"] == pytest.approx(1.0)
    a = bench.alu_roofline("w", "fp32acc", 4e-3)
    assert a["frac"] == pytest.approx(0.25)
    assert "priced_frac" not in a
    # priced issue cycles: 1024 SIMDs x 2.4e9 cycles/s x 1 ms = 2.4576e9 cycles is the whole chip
    _write_profile(fake_root, bench.kernel_hash(),
                   {"w/fp32acc": {"valu_insts_per_launch": 6.144e8, "valu_issue_cycles_per_launch": 1.2288e9}})
    assert bench.alu_roofline("w", "fp32acc", 1e-3)["priced_frac"] == pytest.approx(0.5)


def test_form_difference_whole_states_and_slabs():
    rng = np.random.default_rng(3)
    b = rng.standard_normal((8, 5, 7))
    a = b.copy()
    a[3, 2, 4] += 1e-6   # an off-diagonal (Im rho_ex) change
    a[0, 1, 1] += 2e-6   # a diagonal change
    d = bench.form_difference(a, b)
    assert d["max_abs"] == pytest.approx(2e-6)
    assert d["max_rel_offdiag"] == pytest.approx(1e-6 / np.abs(b[[2, 3, 6, 7]]).max())
    # slabs: dicts of [8][rows][nv] blocks, compared the same way
    ds = bench.form_difference({0: a[:, :2], 9: a[:, 2:]}, {0: b[:, :2], 9: b[:, 2:]})
    assert ds == d
