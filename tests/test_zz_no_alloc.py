"""lqt_solve_noalloc (the solve whose scratch memory is the library's fixed device array) vs
lqt_solve with a workspace, through the C ABI: two calls in a row, the second with a smaller
problem (the array keeps the first call's contents), on the per-lane and the wave path, and a
problem too large for the array, refused before anything runs.  Same kernels and launch
sequence, so the outputs agree to rounding at most (checked at 1e-13 normwise, FP64)."""
import numpy as np
import pytest
import torch

from helpers import relerr
from lqt_layout import untile
from paper_2212_11744_amd import lqt
from paper_2212_11744_amd import workloads as W

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _compare(dp, label):
    ref = lqt.solve(dp, keep_elements=True)
    got = lqt.solve_noalloc(dp)
    torch.cuda.synchronize()
    for k in ("S", "v", "x", "u"):
        e = relerr(_np(got[k]), _np(ref[k]))
        assert e < 1e-13, f"{label} {k}: {e:.3e}"
    for b in range(dp.batch):  # elements: the T blocks of each problem (tile padding is unwritten)
        e = relerr(untile(_np(got["elts"][b]), dp.T), untile(_np(ref["elts"][b]), dp.T))
        assert e < 1e-13, f"{label} elts[{b}]: {e:.3e}"


def test_noalloc_matches_workspace_solve_twice_shrinking():
    assert torch.cuda.is_available()
    big = lqt.DeviceProblem.from_problems([W.point_mass(31, 5 * 512 + 77, 4)])
    small = lqt.DeviceProblem.from_problems([W.point_mass(32, 300, 4)])
    assert 0 < lqt.noalloc_scratch_size(small) < lqt.noalloc_scratch_size(big) <= lqt.NOALLOC_SCRATCH_BYTES
    _compare(big, "first call")
    _compare(small, "second call, smaller")


def test_noalloc_wave_path_and_batch():
    p5 = [W.random_stable(40 + i, nx=5, nu=2, T=700 - 300 * i, n=2, tf=3.0) for i in range(2)]
    _compare(lqt.DeviceProblem.from_problems([p5[0]]), "nx=5 first")
    _compare(lqt.DeviceProblem.from_problems([p5[1]]), "nx=5 second, smaller")
    batch = [W.point_mass(50 + i, 1000, 2) for i in range(3)]
    _compare(lqt.DeviceProblem.from_problems(batch), "batch of 3")


def test_noalloc_refuses_oversized_problem():
    # nx = 16 tree records at 2^16 blocks exceed the fixed array: refused before any launch
    p = W.random_stable(7, nx=16, nu=4, T=2 ** 16, n=1, tf=10.0, time_varying=False)
    dp = lqt.DeviceProblem.from_problems([p])
    assert lqt.noalloc_scratch_size(dp) > lqt.NOALLOC_SCRATCH_BYTES
    with pytest.raises(lqt.LQTError) as ei:
        lqt.solve_noalloc(dp)
    assert ei.value.status == lqt.LQT_EWORKSPACE
