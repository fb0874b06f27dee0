"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

oracle/sanitize_check.c includes the oracle's source as one translation unit;
it is built here with gcc -fsanitize=address,undefined (no recovery, so the
first report ends the run with an error) and run on cases that cover every
code path of the right-hand side: both schemes, Kreiss-Oliger orders 1-3, the
three velocity grids (Simpson with v = 0 on the grid), the vacuum and matter
terms, the minimum grid sizes (nz = 5 for FD, 9 for WENO7) and nv = 1.
Every buffer it hands the oracle has its exact size, so an access past the
end of any array, an uninitialised shift or a signed overflow is reported.
What it computes must equal the regular build's results (both are compiled
without floating-point contraction; the moment and diagnostic sums may be
associated differently by the regular build's OpenMP threads).
"""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

from oracle import oracle as o
from paper_2203_12866_amd import workloads as wl

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(HERE), "oracle", "sanitize_check.c")

CASES = [
    # scheme, ko_r, quad, nz, nv, omega, lam, steps
    (o.FD_KO, 2, o.QUAD_MIDPOINT, 17, 6, 0.3, 0.7, 3),
    (o.FD_KO, 1, o.QUAD_TRAPEZOID, 11, 5, 0.0, 1.1, 2),
    (o.FD_KO, 3, o.QUAD_SIMPSON, 13, 7, 0.2, 0.0, 2),
    (o.FD_KO, 2, o.QUAD_MIDPOINT, 5, 3, 0.1, 0.2, 2),
    (o.FD_KO, 2, o.QUAD_MIDPOINT, 6, 1, 0.0, 0.0, 1),
    (o.FV_WENO7, 2, o.QUAD_MIDPOINT, 19, 8, 0.05, 0.3, 3),
    (o.FV_WENO7, 2, o.QUAD_SIMPSON, 12, 5, 0.0, 0.4, 2),
    (o.FV_WENO7, 2, o.QUAD_TRAPEZOID, 9, 4, 0.2, 0.0, 2),
]


def _problem(case, seed):
    scheme, ko_r, quad, nz, nv, omega, lam, steps = case
    L = 0.7 * nz
    # nv = 1 has its one bin at v = 0, where dt = CFL dz / max|v| is unbounded: a fixed dt there
    dt = o.dt_from_cfl(nz, nv, L, 0.4, quad) if nv > 1 else 0.1
    return o.Problem(nz=nz, nv=nv, L=L, dt=dt, mu=1.0, omega=omega,
                     theta=0.6, lam=lam, alpha=0.9, scheme=scheme, ko_eps=0.1, ko_r=ko_r, weno_eps=1e-6,
                     g_nu=o.angular_dist(nv, 0.6, quad), g_nubar=o.angular_dist(nv, 0.5, quad), quad=quad)


@pytest.fixture(scope="module")
def sanitized_binary(tmp_path_factory):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not found")
    out = str(tmp_path_factory.mktemp("asan") / "sanitize_check")
    cmd = [gcc, "-std=c11", "-O1", "-g", "-ffp-contract=off", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", SRC, "-o", out, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return out


def test_oracle_clean_under_asan_and_ubsan(sanitized_binary, tmp_path):
    rng = np.random.default_rng(7)
    blobs, expected = [struct.pack("i", len(CASES))], []
    for n, case in enumerate(CASES):
        p = _problem(case, n)
        steps = case[-1]
        y = wl.random_unit_state(p.nz, p.nv, 100 + n)
        stencil = rng.normal(size=7)
        blobs.append(struct.pack("6i", p.nz, p.nv, p.scheme, p.ko_r, p.quad, steps))
        blobs.append(struct.pack("9d", p.L, p.dt, p.mu, p.omega, p.theta, p.lam, p.alpha, p.ko_eps, p.weno_eps))
        for a in (p.g_nu, p.g_nubar, y, stencil):
            blobs.append(np.ascontiguousarray(a, dtype=np.float64).tobytes())
        q, si, w = o.weno7_parts(stencil, p.weno_eps)
        d = o.diagnostics(p, y)
        expected.append([o.rhs(p, y).ravel(), o.moments(p, y).ravel(),
                         np.array([d[k] for k in o.DIAG_NAMES]), o.rk4(p, y, steps).ravel(),
                         q, si, w, np.array([o.weno7_minus(stencil, p.weno_eps)])])
    fin, fout = tmp_path / "in.bin", tmp_path / "out.bin"
    fin.write_bytes(b"".join(blobs))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=24")
    r = subprocess.run([sanitized_binary, str(fin), str(fout)], capture_output=True, text=True, env=env,
                       timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    got = np.frombuffer(fout.read_bytes(), dtype=np.float64)
    at = 0
    names = ["rhs", "moments", "diagnostics", "rk4", "q", "si", "w", "flux"]
    for n, parts in enumerate(expected):
        for name, ref in zip(names, parts):
            seg = got[at:at + ref.size]
            at += ref.size
            if name in ("moments", "diagnostics"):
                np.testing.assert_allclose(seg, ref, rtol=1e-13, atol=1e-15, err_msg=f"case {n} {name}")
            else:
                assert np.array_equal(seg, ref), (n, name, float(np.abs(seg - ref).max()))
    assert at == got.size
