"""The C ABI from a plain C program (tests/c_abi_check.c, built by
__graft_entry__.build()), with no Python or torch in its process: its states
match the oracle to the FP64 bar."""
import os
import subprocess

import numpy as np
import pytest

from oracle import oracle as o
from paper_2203_12866_amd import workloads as wl

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
EXE = os.path.join(HERE, "c_abi_check")


def _params(**kw):
    # the library's defaults (cosenu_params_default) with the C program's changes
    w = wl.small_fd(1)
    w.update(phase=0.0, nz=96, nv=128, L=75.0, omega=0.1, lam=0.2, pert_amp=0.3, precision=wl.FP64)
    w.update(kw)
    return w


def test_c_caller_matches_oracle(tmp_path):
    if not os.path.exists(EXE):
        pytest.fail("tests/c_abi_check is not built (run __graft_entry__.build())")
    prefix = str(tmp_path / "out")
    r = subprocess.run([EXE, prefix], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    facts = dict(line.split(" = ") for line in open(prefix + ".txt").read().splitlines())
    assert facts["step"] == "10" and facts["nonfinite"] == "0" and facts["batch"] == "ok"
    assert facts["launches_per_step"] == "2"  # FD + KO at nv = 128: fused stage pairs

    w = _params()
    p = o.problem_from_workload(w)
    assert abs(float(facts["dt"]) - p.dt) < 1e-15 * p.dt
    got = np.fromfile(prefix + ".sim.bin", dtype=np.float64).reshape(8, 96, 128)
    ref = o.rk4(p, o.initial_state_for(w), 10)
    assert np.abs(got - ref).max() <= 1e-12
    assert np.abs(ref[2:4] - o.initial_state_for(w)[2:4]).max() > 1e-3  # a state that moved

    raw = np.fromfile(prefix + ".batch.bin", dtype=np.float64)
    w1 = _params(scheme=wl.FV_WENO7, nz=64, nv=33, quadrature=o.QUAD_SIMPSON)
    n0 = 8 * 96 * 128
    assert raw.size == n0 + 8 * 64 * 33
    for wi, arr in ((w, raw[:n0].reshape(8, 96, 128)), (w1, raw[n0:].reshape(8, 64, 33))):
        pi = o.problem_from_workload(wi)
        refi = o.rk4(pi, o.initial_state_for(wi), 7)
        assert np.abs(arr - refi).max() <= 1e-12
