"""The finite check of the C ABI (environment variable LQT_CHECK_FINITE): with it set, entry points
scan their outputs and return LQT_ENONFINITE when one holds NaN or Inf; unset, nothing is
scanned.  Non-finite outputs are produced by a NaN in one reference sample (memory-safe: every
index of every kernel is independent of the data)."""
import numpy as np
import pytest
import torch

import oracle as O
from helpers import relerr
from paper_2212_11744_amd import lqt
from paper_2212_11744_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _device(monkeypatch):
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lqt.lib()
    yield monkeypatch
    torch.cuda.synchronize()


def _nan_problem():
    p = W.point_mass(3, 64, 4)
    p.r = p.r.copy()
    p.r[37, 0] = np.nan
    return p


@pytest.mark.parametrize("nx", [4, 8])
def test_valid_problem_passes_with_the_check(monkeypatch, nx):
    monkeypatch.setenv("LQT_CHECK_FINITE", "1")
    p = W.point_mass(3, 64, 4) if nx == 4 else W.random_stable(3, nx=8, nu=4, T=64, n=4, tf=1.0)
    dp = lqt.DeviceProblem.from_problems([p])
    out = lqt.solve(dp, keep_elements=True)
    S, v = lqt.scan_value(dp, out["elts"])
    x, u = lqt.forward_traj(dp, out["elts"], S, v)
    torch.cuda.synchronize()
    ref = O.solve(p)
    assert relerr(out["x"][0].cpu().numpy(), ref["x"]) < 1e-9
    assert relerr(x[0].cpu().numpy(), ref["x"]) < 1e-9


def test_nan_input_reported_by_every_stage(monkeypatch):
    monkeypatch.setenv("LQT_CHECK_FINITE", "1")
    dp = lqt.DeviceProblem.from_problems([_nan_problem()])
    with pytest.raises(lqt.LQTError) as ei:
        lqt.build_elements(dp)
    assert ei.value.status == lqt.LQT_ENONFINITE
    for call in (lambda: lqt.solve(dp), lambda: lqt.build_elements_split(dp),
                 lambda: lqt.build_elements_forward(dp)):
        with pytest.raises(lqt.LQTError) as ei:
            call()
        assert ei.value.status == lqt.LQT_ENONFINITE


def test_nan_input_without_the_check_returns_nan_outputs(monkeypatch):
    monkeypatch.delenv("LQT_CHECK_FINITE", raising=False)
    dp = lqt.DeviceProblem.from_problems([_nan_problem()])
    out = lqt.solve(dp)
    torch.cuda.synchronize()
    assert torch.isfinite(out["S"]).all()  # S does not depend on r
    assert not torch.isfinite(out["v"]).all()
    monkeypatch.setenv("LQT_CHECK_FINITE", "0")
    out = lqt.solve(dp)
    torch.cuda.synchronize()
    assert not torch.isfinite(out["x"]).all()
