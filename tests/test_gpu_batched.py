"""Batched solve of problems with uneven horizons and several sizes (lqt_ragged, lqt_plan).

Every member is checked against the oracle's sequential solve (normwise 1e-9 in FP64, 1e-4 in
FP32) and against lqt_solve on the member alone (1e-12 in FP64: the same kernels, only the scan
trees group the blocks differently).  The tuned plan is replayed several times with eager work
and in-place input updates in between, and every replay is checked.
"""
import numpy as np
import pytest
import torch

import oracle as O
from helpers import relerr
from paper_2212_11744_amd import lqt
from paper_2212_11744_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {torch.float64: 1e-9, torch.float32: 1e-4}


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lqt.lib()
    yield
    torch.cuda.synchronize()


def _mixed(seed=0):
    """Members of five classes: point mass in 1 and 2 axes, random stable nx = 8 (constant F),
    nx = 3 with sampled F(t) and a drift c(t), nx = 5 with sampled L(t)."""
    rng = np.random.default_rng(seed)
    out = []
    Ts = [1, 2, 5, 63, 64, 65, 257, 300, 3, 130]
    for j, T in enumerate(Ts):
        dt = 0.01
        kind = j % 5
        if kind == 0:
            p = W.point_mass(10 + j, T, 4, 0.0, dt * T, d=1)
        elif kind == 1:
            p = W.point_mass(10 + j, T, 4, 0.0, dt * T, d=2)
        elif kind == 2:
            p = W.random_stable(10 + j, 8, 4, T, 3, 0.0, dt * T + 0.2, time_varying=False)
        elif kind == 3:
            p = W.random_stable(10 + j, 3, 2, T, 2, 0.0, dt * T + 0.1, time_varying=True)
            p.c = 0.2 * np.cos(np.linspace(0, 2, p.r.shape[0]))[:, None] * rng.standard_normal(3)[None]
        else:
            p = W.random_stable(10 + j, 5, 2, T, 2, 0.0, dt * T + 0.1, time_varying=False)
            ts = W.half_step_times(p.t, p.n)
            p.L = p.L[None] * (1.0 + 0.3 * np.sin(ts))[:, None, None]
        out.append(p)
    return out


def _check_member(res, ref, tol, label):
    for k in ("S", "v", "x", "u"):
        e = relerr(_np(res[k]), ref[k])
        assert e < tol, f"{label} {k}: {e:.3e}"


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_mixed_classes_eager(dtype):
    probs = _mixed()
    bs = lqt.BatchedSolve(probs, dtype=dtype, plan=False)
    assert len(bs.classes) == 5
    bs.solve_eager()
    torch.cuda.synchronize()
    for i, p in enumerate(probs):
        res = bs.result(i)
        _check_member(res, O.solve(p), TOL[dtype], f"member {i} (nx={p.nx}, T={p.T})")
        if dtype == torch.float64:
            single = lqt.solve(lqt.DeviceProblem.from_problems([p]))
            for k in ("S", "v", "x", "u"):
                assert relerr(_np(res[k]), _np(single[k][0])) < 1e-12, f"member {i} {k} vs single"


def test_plan_replays_and_follows_inputs():
    probs = _mixed(1)
    bs = lqt.BatchedSolve(probs, autotune=True)
    assert bs.config()
    eager = lqt.BatchedSolve(probs, plan=False)
    eager.solve_eager()
    torch.cuda.synchronize()
    for rep in range(3):
        bs.launch()
        torch.cuda.synchronize()
        for i in range(len(probs)):
            a, b = bs.result(i), eager.result(i)
            for k in ("S", "v", "x", "u"):
                assert relerr(_np(a[k]), _np(b[k])) < 1e-12, f"replay {rep} member {i} {k}"
        # eager work between replays
        torch.cuda.synchronize()
        _ = (eager.classes[0]["x"] * 2.0).sum().item()
    # Refill inputs in place: new initial states, then one more replay against the oracle.
    rng = np.random.default_rng(5)
    for c in bs.classes:
        new = rng.standard_normal(tuple(c["x0"].shape))
        c["x0"].copy_(torch.as_tensor(new, dtype=c["x0"].dtype))
        for j, i in enumerate(c["members"]):
            probs[i].x0 = new[j]
    bs.launch()
    torch.cuda.synchronize()
    for i, p in enumerate(probs):
        _check_member(bs.result(i), O.solve(p), 1e-9, f"refilled member {i}")


def test_graph_plan_replays():
    """The tuned plan captured once into a HIP graph (LQT_PLAN_GRAPH) and replayed: every replay,
    with the program's own eager work and synchronisations between replays, equals the first and
    the eager solve at 1e-12 and the oracle at 1e-9; inputs refilled in place reach the next
    replay.  Replays are not compared bit for bit: a single-pass scan tile combines the records of
    the tiles before it in an order that depends on which of them have already published, so the
    rounding of the per-lane scans varies from run to run."""
    probs = _mixed(1)
    eager = lqt.BatchedSolve(probs, autotune=False, plan=False)
    eager.solve_eager()
    torch.cuda.synchronize()
    bs = lqt.BatchedSolve(probs, autotune=True, graph=True)
    first = None
    for rep in range(4):
        bs.launch()
        torch.cuda.synchronize()
        if first is None:
            first = [{k: t.clone() for k, t in bs.result(i).items()} for i in range(len(probs))]
        for i, p in enumerate(probs):
            a, b = bs.result(i), eager.result(i)
            for k in ("S", "v", "x", "u"):
                assert relerr(_np(a[k]), _np(first[i][k])) < 1e-12, f"replay {rep} member {i} {k}"
                assert relerr(_np(a[k]), _np(b[k])) < 1e-12, f"replay {rep} member {i} {k}"
            if rep == 0:
                _check_member(a, O.solve(p), 1e-9, f"replay {rep} member {i}")
        # eager work of the program between replays
        _ = (eager.classes[0]["x"] * 2.0).sum().item()
        eager.solve_eager()
        torch.cuda.synchronize()
    rng = np.random.default_rng(9)
    for c in bs.classes:
        new = rng.standard_normal(tuple(c["x0"].shape))
        c["x0"].copy_(torch.as_tensor(new, dtype=c["x0"].dtype))
        for j, i in enumerate(c["members"]):
            probs[i].x0 = new[j]
    bs.launch()
    torch.cuda.synchronize()
    for i, p in enumerate(probs):
        _check_member(bs.result(i), O.solve(p), 1e-9, f"refilled member {i}")
    bs.close()


def test_single_member_class_and_one_block_problems():
    probs = [W.point_mass(3, 1, 4, 0.0, 0.05), W.point_mass(4, 1, 4, 0.0, 0.05),
             W.point_mass(5, 7, 4, 0.0, 0.2, d=1)]
    bs = lqt.BatchedSolve(probs)
    bs.launch()
    torch.cuda.synchronize()
    for i, p in enumerate(probs):
        _check_member(bs.result(i), O.solve(p), 1e-9, f"member {i}")


def test_batched_mix_full_size():
    """1024 problems, nx in {2, 4, 8}, T_i ~ U{256..8192} (the batched workload at full size):
    every member against lqt_solve alone on sampled members, and the oracle on one per class."""
    probs = W.batched_mix()
    bs = lqt.BatchedSolve(probs, autotune=True)
    bs.launch()
    torch.cuda.synchronize()
    rng = np.random.default_rng(0)
    sample = sorted(set(rng.choice(len(probs), 24, replace=False).tolist()) | {0, 1, 2, 1021, 1022, 1023})
    for i in sample:
        p = probs[i]
        single = lqt.solve(lqt.DeviceProblem.from_problems([p]))
        res = bs.result(i)
        for k in ("S", "v", "x", "u"):
            assert relerr(_np(res[k]), _np(single[k][0])) < 1e-12, f"member {i} {k}"
    for i in (0, 1, 2):
        _check_member(bs.result(i), O.solve(probs[i]), 1e-9, f"member {i} vs oracle")


@pytest.mark.parametrize("Ts", [(1, 2), (20, 30), (100, 130), (300, 257, 500), (4000, 3000, 2500)],
                         ids=["L1", "L2", "L3", "L4", "L6"])
def test_wave_class_queue_tree_depths(Ts):
    """One wave-path class (nx = 6) in the single queue launch, with trees of 1 to 6 levels
    (8 blocks per wave at the bottom, 4 nodes per wave above; rows = sum of T_i + 1: 5 give one
    level, 52 two, 232 three, 1060 four, 9503 six): every member against the oracle and against
    lqt_solve alone."""
    probs = [W.random_stable(40 + i, 6, 3, T, 2, 0.0, 0.004 * T + 0.1, time_varying=False)
             for i, T in enumerate(Ts)]
    bs = lqt.BatchedSolve(probs, plan=False)
    bs.solve_eager()
    torch.cuda.synchronize()
    for i, p in enumerate(probs):
        res = bs.result(i)
        _check_member(res, O.solve(p), 1e-9, f"member {i} (T={p.T})")
        single = lqt.solve(lqt.DeviceProblem.from_problems([p]))
        for k in ("S", "v", "x", "u"):
            assert relerr(_np(res[k]), _np(single[k][0])) < 1e-12, f"member {i} {k} vs single"


@pytest.mark.parametrize("Ts,chunk", [((700, 900, 300), 1), ((5000, 7000, 129), 4),
                                      ((2 ** 18, 2 ** 18 + 77, 3), 8)])
def test_lane_class_queue_chunks(Ts, chunk):
    """One per-lane class (nx = 2) in the single queue launch at each value chunk of the eager
    solve (1 block per lane up to 2^11 rows, 4 below 2^19, 8 from there): members against
    lqt_solve alone (1e-12) and the smallest against the oracle (1e-9)."""
    probs = [W.point_mass(60 + i, T, 2, 0.0, 0.002 * T + 0.5, d=1) for i, T in enumerate(Ts)]
    rows = sum(T + 1 for T in Ts)
    assert (rows <= 2 ** 11) == (chunk == 1) and (rows >= 2 ** 19) == (chunk == 8)
    bs = lqt.BatchedSolve(probs, plan=False)
    bs.solve_eager()
    torch.cuda.synchronize()
    for i, p in enumerate(probs):
        res = bs.result(i)
        single = lqt.solve(lqt.DeviceProblem.from_problems([p]))
        for k in ("S", "v", "x", "u"):
            assert relerr(_np(res[k]), _np(single[k][0])) < 1e-12, f"member {i} {k} vs single"
    i = int(np.argmin(Ts))
    _check_member(bs.result(i), O.solve(probs[i]), 1e-9, f"member {i} vs oracle")
