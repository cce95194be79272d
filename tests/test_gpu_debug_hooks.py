"""Debugging aids of the C ABI on the GPU: canary-padded workspaces, simulated launch failures,
the tuner switch and its persisted cache (process-wide settings, reset after every test).

* Canaries (lqt_debug_canary(1)): every region of a call's workspace is followed by a 256-byte
  canary, filled before the call's first launch and checked at its end; the lane and wave paths'
  solves, every stage call and the adjoint run with them and leave them intact, with results
  equal to those of the ordinary layout (1e-12: the single-pass scans' record order may differ).
  Mode 2 spoils canary 0 itself, which the check must report (LQT_EWORKSPACE).
* lqt_debug_fail_launch(n): the n-th checked HIP call reports a failure (the call is made):
  the entry point returns LQT_EHIP naming the simulation, and the next call works.
* LQT_AUTOTUNE / LQT_TUNE_CACHE: "force" tunes and writes the cache file (GPU architecture and
  class signature), "off" gives the default configuration, "on" reuses the cached choice, and a
  fresh process reads the file back.
"""
import os
import subprocess
import sys

import numpy as np
import pytest
import torch

from helpers import relerr
from paper_2212_11744_amd import lqt
from paper_2212_11744_amd import workloads as W

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


@pytest.fixture(autouse=True)
def _reset():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lqt.lib()
    yield
    lqt.debug_canary(0)
    lqt.debug_fail_launch(0)
    for k in ("LQT_AUTOTUNE", "LQT_TUNE_CACHE"):
        os.environ.pop(k, None)
    torch.cuda.synchronize()


def _close(a, b, tol=1e-12):
    # outputs only: the element tiles' padding columns are never written
    for k in ("S", "v", "x", "u"):
        if k in a and k in b and a[k] is not None and b[k] is not None:
            assert relerr(_np(a[k]), _np(b[k])) < tol, k


@pytest.mark.parametrize("kind", ["lane", "wave"])
def test_canaries_intact_in_solve_and_stages(kind):
    if kind == "lane":
        p = W.point_mass(3, 700, 4, tf=3.0)
    else:
        p = W.random_stable(5, nx=6, nu=3, T=150, n=2, tf=1.5)
    dp = lqt.DeviceProblem.from_problems([p, p])
    ref = lqt.solve(dp, keep_elements=True)
    lqt.debug_canary(1)
    out = lqt.solve(dp, keep_elements=True)   # workspace sized with the canaries
    torch.cuda.synchronize()
    _close(out, ref)
    S, v = lqt.scan_value(dp, ref["elts"])
    _close({"S": S, "v": v}, ref)
    x, u = lqt.forward_traj(dp, ref["elts"], ref["S"], ref["v"])
    _close({"x": x, "u": u}, ref)
    if kind == "lane":
        x2, _ = lqt.forward_traj_method2(dp, ref["elts"], ref["S"], ref["v"])
        assert relerr(_np(x2), _np(ref["x"])) < 1e-9
        g = torch.zeros_like(ref["x"]) + 1.0
        lqt.debug_canary(0)
        gref = lqt.backward(dp, ref["S"], ref["v"], ref["x"], g)
        lqt.debug_canary(1)
        got = lqt.backward(dp, ref["S"], ref["v"], ref["x"], g)
        for k in gref:
            assert relerr(_np(got[k]), _np(gref[k])) < 1e-12, k


def test_spoilt_canary_is_reported():
    dp = lqt.DeviceProblem.from_problems([W.point_mass(4, 100, 4, tf=1.0)])
    lqt.debug_canary(2)
    with pytest.raises(lqt.LQTError) as ei:
        lqt.solve(dp)
    assert ei.value.status == lqt.LQT_EWORKSPACE
    assert "canary 0 of" in str(ei.value)
    lqt.debug_canary(1)
    lqt.solve(dp)  # intact again
    torch.cuda.synchronize()


@pytest.mark.parametrize("n", [1, 2, 4])
def test_simulated_launch_failure(n):
    dp = lqt.DeviceProblem.from_problems([W.point_mass(6, 300, 4, tf=2.0)])
    ref = lqt.solve(dp)
    torch.cuda.synchronize()
    lqt.debug_fail_launch(n)
    with pytest.raises(lqt.LQTError) as ei:
        lqt.solve(dp)
    assert ei.value.status == lqt.LQT_EHIP
    assert "simulated" in str(ei.value)
    torch.cuda.synchronize()
    out = lqt.solve(dp)   # the hook fired once; the library keeps working
    torch.cuda.synchronize()
    _close(out, ref)


def test_simulated_failure_in_plan_creation():
    probs = [W.point_mass(7 + i, 50 + 13 * i, 4, tf=1.0) for i in range(4)]
    lqt.debug_fail_launch(3)
    with pytest.raises(lqt.LQTError) as ei:
        lqt.BatchedSolve(probs, autotune=True)
    assert ei.value.status == lqt.LQT_EHIP and "simulated" in str(ei.value)
    torch.cuda.synchronize()
    bs = lqt.BatchedSolve(probs, autotune=True)
    bs.launch()
    torch.cuda.synchronize()
    bs.close()


def test_tuner_switch_and_persisted_cache(tmp_path):
    cache = str(tmp_path / "tune.txt")
    probs = [W.point_mass(20 + i, 200 + 37 * i, 4, tf=2.0) for i in range(3)]
    probs += [W.random_stable(30, nx=5, nu=2, T=90, n=2, tf=1.0, time_varying=False)]
    os.environ["LQT_TUNE_CACHE"] = cache
    os.environ["LQT_AUTOTUNE"] = "force"
    forced = lqt.BatchedSolve(probs, autotune=True)
    text = forced.config()
    forced.close()
    lines = open(cache).read().splitlines()
    assert any(l.startswith("gfx950 ") and l.endswith("|" + text) for l in lines), lines
    os.environ["LQT_AUTOTUNE"] = "off"
    off = lqt.BatchedSolve(probs, autotune=True)
    assert off.config() == "default configuration"
    off.close()
    os.environ["LQT_AUTOTUNE"] = "on"
    again = lqt.BatchedSolve(probs, autotune=True)
    assert again.config() == text
    again.close()
    # a fresh process reads the file (the tuned text holds measured times, so equal text means
    # the choice came from the cache, not from tuning again)
    code = ("import sys; sys.path.insert(0, '.'); sys.path.insert(0, 'tests'); "
            "from paper_2212_11744_amd import lqt, workloads as W; "
            "probs = [W.point_mass(20 + i, 200 + 37 * i, 4, tf=2.0) for i in range(3)]; "
            "probs += [W.random_stable(30, nx=5, nu=2, T=90, n=2, tf=1.0, time_varying=False)]; "
            "b = lqt.BatchedSolve(probs, autotune=True); print(b.config()); b.close()")
    env = dict(os.environ, LQT_TUNE_CACHE=cache, LQT_AUTOTUNE="on")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    assert r.stdout.strip().splitlines()[-1] == text
