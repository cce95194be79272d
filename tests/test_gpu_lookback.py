"""Single-pass value and trajectory scans (decoupled look-back) vs the oracle, through the C ABI.

The scans give every tile (one wave; 1, 2, 4 or 8 blocks per lane, chosen from the horizon: value
scan 1 up to 2^11 blocks, 2 up to 2^14, 4 up to 2^17, then 8; trajectory scan 1 up to 2^14, 2 up
to 2^15, then 4) a place in the flow order from a counter; a tile resolves the state at its free end from up
to 63 preceding tile records and then from group records (64 tiles each), 64 groups per round.
The horizons below use every chunk size, put the last tile just before, on and after group
boundaries, and go past the first 64 groups (a second round of group records); batches check
that every problem has its own counter and records; a reused workspace checks that the status
words are cleared before every call.  Stage tests feed oracle elements to the GPU scans, so only
the scans' rounding differs (1e-11 normwise); whole solves are held to 1e-9 (FP64) and 1e-4
(FP32).
"""
import numpy as np
import pytest
import torch

import oracle as O
from helpers import relerr
from lqt_layout import dense_to_soa
from paper_2212_11744_amd import lqt
from paper_2212_11744_amd import workloads as W

pytestmark = pytest.mark.gpu

VTILE, TTILE, GROUP = 512, 256, 64


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lqt.lib()
    yield
    torch.cuda.synchronize()


def _stage_check(p, tol=1e-11, reps=1):
    el = O.elements(p)
    S_ref, v_ref = O.value(el, p.Qf, p.rf)
    x_ref, u_ref = O.trajectory(p, el, S_ref, v_ref)
    dp = lqt.DeviceProblem.from_problems([p])
    elts = torch.as_tensor(dense_to_soa(el, p.nx)[None], device="cuda")
    wsv = lqt.workspace(dp, lqt.CALL_SCAN_VALUE)
    wst = lqt.workspace(dp, lqt.CALL_FORWARD_TRAJ)
    for rep in range(reps):
        S, v = lqt.scan_value(dp, elts, ws=wsv)
        x, u = lqt.forward_traj(dp, elts, torch.as_tensor(S_ref[None], device="cuda"),
                                torch.as_tensor(v_ref[None], device="cuda"), ws=wst)
        torch.cuda.synchronize()
        for name, got, ref in (("S", S, S_ref), ("v", v, v_ref), ("x", x, x_ref), ("u", u, u_ref)):
            e = relerr(_np(got[0]), ref)
            assert e < tol, f"T={p.T} rep {rep} {name}: {e:.3e}"


@pytest.mark.parametrize("T", [5, 64, 65, 256, 257, 512, 513, 4095, 4096, 4097, 63 * TTILE,
                               GROUP * TTILE, GROUP * TTILE + 1, GROUP * VTILE - 1, GROUP * VTILE,
                               GROUP * VTILE + 1, 65 * VTILE + 17, 2 * GROUP * VTILE + 255,
                               2 ** 17 + 5])
def test_stage_scans_across_group_boundaries(T):
    p = W.random_stable(900 + T % 1000, nx=3, nu=2, T=T, n=2, tf=0.002 * T + 0.5)
    _stage_check(p)


def test_stage_scans_second_round_of_group_records():
    """65 groups of value tiles (4100 tiles of 512 blocks; 129 groups of trajectory tiles): the
    look-back of the last groups passes 64 group records and goes on to further rounds.  nx = 2
    with one RK4 step per block keeps the oracle fast."""
    G = GROUP * GROUP + 4
    T = (G - 1) * VTILE + 97
    p = W.random_stable(77, nx=2, nu=1, T=T, n=1, tf=T * 1e-5, time_varying=False)
    _stage_check(p)


def test_reused_workspace_is_cleared():
    """Two scans in a row on one workspace (status words left set by the first call)."""
    p = W.point_mass(8, 70 * VTILE + 3, 2)
    _stage_check(p, reps=3)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_batch_counters_per_problem(dtype):
    """Three problems of 70 value tiles each in one launch: every problem owns its counter, tile
    and group records."""
    T = 70 * VTILE - 11
    probs = [W.point_mass(300 + i, T, 2, tf=8.0) for i in range(3)]
    dp = lqt.DeviceProblem.from_problems(probs, dtype=dtype)
    out = lqt.solve(dp)
    tol = 1e-9 if dtype == torch.float64 else 1e-4
    for b, p in enumerate(probs):
        ref = O.solve(p)
        for k in ("S", "v", "x", "u"):
            e = relerr(_np(out[k][b]), ref[k])
            assert e < tol, f"problem {b} {k}: {e:.3e}"


def test_full_solve_many_groups_fp64():
    """The whole solve over 300 value tiles (5 groups) against the oracle."""
    p = W.point_mass(12, 300 * VTILE - 100, 2, tf=3.0)
    ref = O.solve(p)
    out = lqt.solve(lqt.DeviceProblem.from_problems([p]))
    for k in ("S", "v", "x", "u"):
        assert relerr(_np(out[k][0]), ref[k]) < 1e-9, k
