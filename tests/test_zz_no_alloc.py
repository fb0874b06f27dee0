"""cosenu_step_noalloc (every intermediate buffer in the library's static
scratch array, nothing allocated) against cosenu_step on a handle created from
the same parameters: the same kernels and arithmetic, so the same state bit for
bit (and within the FP64 bar of 1e-12 / the FP32 form's 1e-5 relative in any
case).  Two calls in a row, the second on a smaller problem, so the second
reads a scratch array holding the first one's larger layout."""
import numpy as np
import pytest

from paper_2203_12866_amd import cosenu
from paper_2203_12866_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _handle_run(w, nsteps):
    with cosenu.Sim(w) as s:
        y0 = s.get_state()
        s.step(nsteps)
        return y0, s.get_state()


def _noalloc_run(torch, w, y0, nsteps):
    t = torch.from_numpy(np.ascontiguousarray(y0)).to("cuda")
    cosenu.step_noalloc(w, t.data_ptr(), nsteps, torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _compare(got, ref, fp64):
    assert got.shape == ref.shape
    if fp64:
        assert float(np.abs(got - ref).max()) <= 1e-12
    else:
        for grp in ([0, 1, 4, 5], [2, 3, 6, 7]):
            scale = max(float(np.abs(ref[grp]).max()), 1e-300)
            assert float(np.abs(got[grp] - ref[grp]).max()) / scale <= 1e-5
    assert np.array_equal(got, ref)


CASES = [
    # (first call, steps), (second, smaller call, steps)
    ((dict(wl.small_fd(3), nz=1024, nv=128, L=100.0), 7),          # fused pairs, odd step count
     (dict(wl.small_fd(4), nz=512, nv=32), 10)),                    # single stages, nv <= 32
    ((dict(wl.small_fd(5), nz=256, nv=256, L=40.0, scheme=cosenu.FV_WENO7, omega=0.05, lam=0.3,
           precision=cosenu.FP32_ACC64), 5),                        # WENO7, FP32 form, full H
     (dict(wl.small_fd(6), nz=64, nv=64, L=10.0, precision=cosenu.FP32_ACC64, ko_order=3), 4)),
]


@pytest.mark.parametrize("first,second", CASES)
def test_noalloc_matches_cosenu_step_twice(first, second):
    import torch
    torch.cuda.set_device(0)
    for w, n in (first, second):
        print(f"noalloc: nz={w['nz']} nv={w['nv']} scheme={w.get('scheme', 0)} "
              f"precision={w.get('precision', 0)} steps={n}", flush=True)
        y0, ref = _handle_run(w, n)
        got = _noalloc_run(torch, w, y0, n)
        _compare(got, ref, w.get("precision", 0) == cosenu.FP64)


def test_noalloc_zero_steps_and_oversize():
    import torch
    torch.cuda.set_device(0)
    w = dict(wl.small_fd(7), nz=64, nv=64, L=10.0)
    y0, _ = _handle_run(w, 0)
    assert np.array_equal(_noalloc_run(torch, w, y0, 0), y0)
    # 4096 x 128 needs more than the 64 MiB scratch array: refused before any launch
    big = dict(w, nz=4096, nv=128)
    t = torch.zeros((8, 4096, 128), dtype=torch.float64, device="cuda")
    with pytest.raises(cosenu.CosenuError) as e:
        cosenu.step_noalloc(big, t.data_ptr(), 1, torch.cuda.current_stream().cuda_stream)
    assert e.value.code == cosenu.EINVAL
    torch.cuda.synchronize()
    assert float(t.abs().max()) == 0.0
    # a null state or a negative step count is refused too
    with pytest.raises(cosenu.CosenuError):
        cosenu.step_noalloc(w, 0, 1)
    with pytest.raises(cosenu.CosenuError):
        cosenu.step_noalloc(w, t.data_ptr(), -1)
