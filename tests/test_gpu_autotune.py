"""The launch-shape autotuner and its cache file (COSENU_TUNE_CACHE).

* A process that tunes writes the cache file; a second process that only
  creates the same problem starts with the same launch shape (path, segment
  length, waves per workgroup) and reaches the same state bit for bit.
* Shapes forced through the cache file (single stages instead of fused pairs,
  1 or 2 waves per workgroup, odd segment lengths), for FD with wave rows,
  FD with row groups (nv <= 32) and WENO7, give states bitwise equal to the
  default shapes' (results do not depend on the launch shape).
Every process here runs alone, one after the other.
"""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_2203_12866_amd import cosenu
from paper_2203_12866_amd import workloads as wl

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import json, sys
import numpy as np
sys.path.insert(0, {root!r})
from paper_2203_12866_amd import cosenu
w, tune, steps, out = json.loads(sys.argv[1]), sys.argv[2] == "1", int(sys.argv[3]), sys.argv[4]
with cosenu.Sim(w) as s:
    if tune:
        s.autotune()
    info = s.info()
    s.step(steps)
    np.save(out, s.get_state())
print(json.dumps(info))
"""


def _child(w, tune, steps, out, cache):
    env = dict(os.environ, COSENU_TUNE_CACHE=cache)
    r = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT), json.dumps(w), "1" if tune else "0",
                        str(steps), out], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    return json.loads(r.stdout.strip().splitlines()[-1]), np.load(out)


def _solo(w, steps):
    with cosenu.Sim(w) as s:
        s.step(steps)
        return s.get_state()


def _bucket(nz):
    b = 0
    while (1 << (b + 1)) <= nz:
        b += 1
    return b


def test_cache_file_is_reused_by_a_second_process(tmp_path):
    cache = str(tmp_path / "tune.txt")
    w = dict(wl.small_fd(2), nz=1024, nv=128, L=100.0, precision=wl.FP32_ACC64)
    info_a, ya = _child(w, True, 7, str(tmp_path / "a.npy"), cache)
    lines = [ln for ln in open(cache) if not ln.startswith("#")]
    assert len(lines) == 1, lines
    f = lines[0].split()
    assert f[1:5] == ["0", "1", "128", str(_bucket(1024))] and len(f) == 10
    info_b, yb = _child(w, False, 7, str(tmp_path / "b.npy"), cache)
    print(f"tuned: {lines[0].strip()}; first process {info_a}")
    for k in ("seg_rows", "launches_per_step", "waves_per_workgroup"):
        assert info_a[k] == info_b[k], k
    assert np.array_equal(ya, yb)
    assert np.array_equal(ya, _solo(w, 7))


@pytest.mark.parametrize("case", [
    # (workload, forced entry: seg_pairs seg_whole_step seg_single wpb path)
    (dict(nz=1024, nv=128, L=100.0), (0, 0, 5, 1, 0)),                 # FD, single stages instead of fusion
    (dict(nz=1024, nv=128, L=100.0), (7, 0, 9, 2, 1)),                 # FD, fused pairs at an odd segment
    (dict(nz=1024, nv=128, L=100.0), (0, 13, 9, 2, 2)),                # FD, the whole step in one launch
    (dict(nz=300, nv=20, L=30.0), (0, 0, 3, 1, -1)),                   # FD row groups (nv <= 32)
    (dict(nz=200, nv=96, L=20.0, scheme=wl.FV_WENO7, omega=0.1), (0, 0, 3, 2, -1)),  # WENO7 wave rows
    (dict(nz=200, nv=24, L=20.0, scheme=wl.FV_WENO7, lam=0.5), (0, 0, 11, 1, -1)),   # WENO7 row groups
])
def test_forced_shapes_from_cache_are_bitwise(tmp_path, case):
    shape, (sp, sq, ss, wpb, path) = case
    w = dict(wl.small_fd(3), **shape)
    cache = str(tmp_path / "tune.txt")
    # the device tag as the library writes it, from a tuning of a tiny problem
    _child(dict(wl.small_fd(1), nz=64, nv=64, L=10.0), True, 1, str(tmp_path / "t.npy"), cache)
    dev = [ln for ln in open(cache) if not ln.startswith("#")][0].split()[0]
    with open(cache, "w") as f:
        f.write(f"{dev} {w['scheme']} {w['precision']} {w['nv']} {_bucket(w['nz'])} {sp} {sq} {ss} {wpb} {path}\n")
    info, got = _child(w, False, 9, str(tmp_path / "g.npy"), cache)
    nl = info["launches_per_step"]
    print(f"forced {sp, sq, ss, wpb, path}: {info}")
    if path == 2:
        assert nl == 1 and info["seg_rows"] == sq
    elif path == 1:
        assert nl == 2 and info["seg_rows"] == sp
    else:
        assert nl == 4 and info["seg_rows"] == ss and info["waves_per_workgroup"] == wpb
    assert np.array_equal(got, _solo(w, 9))


BATCH_CHILD = r"""
import json, sys
import numpy as np
sys.path.insert(0, {root!r})
from paper_2203_12866_amd import cosenu
ws, steps, out = json.loads(sys.argv[1]), int(sys.argv[2]), sys.argv[3]
with cosenu.Batch(ws) as b:
    b.step(steps)
    launches = [b.info(i)["launches_per_step"] for i in range(len(ws))]
    np.savez(out, *[b.get_state(i) for i in range(len(ws))])
print(json.dumps(launches))
"""


def test_batch_whole_steps_from_cache_are_bitwise(tmp_path):
    """A batch whose FD + KO shapes were tuned to the whole step (forced
    through the cache file) runs them with the batched whole-step kernel, next
    to fused pairs and single stages; every instance equals its solo run."""
    cache = str(tmp_path / "tune.txt")
    _child(dict(wl.small_fd(1), nz=64, nv=64, L=10.0), True, 1, str(tmp_path / "t.npy"), cache)
    dev = [ln for ln in open(cache) if not ln.startswith("#")][0].split()[0]
    ws = [dict(wl.small_fd(21), nz=300, nv=128, L=30.0),            # whole step (forced)
          dict(wl.small_fd(22), nz=77, nv=256, L=20.0),             # whole step (forced), 8 waves
          dict(wl.small_fd(23), nz=129, nv=65, L=25.0),             # fused pairs (not in the cache)
          dict(wl.small_fv(24), nz=64, nv=96, L=10.0, omega=0.1),   # WENO7 single stages
          dict(wl.small_fd(25), nz=15, nv=64, L=5.0)]               # nz < 16: fused pairs
    with open(cache, "w") as f:
        for w, seg in ((ws[0], 13), (ws[1], 7), (ws[4], 5)):
            f.write(f"{dev} 0 0 {w['nv']} {_bucket(w['nz'])} 0 {seg} 0 0 2\n")
    env = dict(os.environ, COSENU_TUNE_CACHE=cache)
    out = str(tmp_path / "b.npz")
    r = subprocess.run([sys.executable, "-c", BATCH_CHILD.format(root=ROOT), json.dumps(ws), "7", out], env=env,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    launches = json.loads(r.stdout.strip().splitlines()[-1])
    print(f"launches per step: {launches}")
    assert launches == [1, 1, 2, 4, 2]
    got = np.load(out)
    for i, w in enumerate(ws):
        ref = _solo(w, 7)
        assert np.array_equal(got[f"arr_{i}"], ref), i


def test_cache_file_bad_lines_are_skipped(tmp_path):
    """Lines the loader cannot use (too few fields, text, negative lengths,
    waves per workgroup other than 1, 2, 4, an unknown path) are skipped; the
    valid line for the shape is used, and a segment longer than the grid is
    clamped to it; results stay bitwise the default's."""
    cache = str(tmp_path / "tune.txt")
    _child(dict(wl.small_fd(1), nz=64, nv=64, L=10.0), True, 1, str(tmp_path / "t.npy"), cache)
    dev = [ln for ln in open(cache) if not ln.startswith("#")][0].split()[0]
    w = dict(wl.small_fd(4), nz=300, nv=96, L=30.0, scheme=wl.FV_WENO7, omega=0.1)
    b = _bucket(w["nz"])
    key = f"{dev} {w['scheme']} {w['precision']} {w['nv']} {b}"
    with open(cache, "w") as f:
        f.write("# comment\n")
        f.write("not a cache line at all\n")
        f.write(f"{key} 0 0 5\n")                 # too few fields
        f.write(f"{key} 0 0 -3 4 -1\n")           # negative segment length
        f.write(f"{key} 0 0 5 3 -1\n")            # 3 waves per workgroup
        f.write(f"{key} 0 0 5 2 7\n")             # unknown path
        f.write(f"{key} 0 0 100000 2 -1\n")       # valid: a segment longer than the grid
    info, got = _child(w, False, 6, str(tmp_path / "g.npy"), cache)
    print(f"info {info}")
    assert info["seg_rows"] == w["nz"] and info["waves_per_workgroup"] == 2
    assert np.array_equal(got, _solo(w, 6))
