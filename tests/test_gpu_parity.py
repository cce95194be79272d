"""GPU path vs the CPU oracle, element by element, through the C ABI.

Tolerances (normwise, see helpers.relerr): 1e-9 in FP64 and 1e-4 in FP32 against the FP64 oracle
for elements, value matrices, trajectories and controls; exact for the integer-valued scan example.
Sizes span several scan tiles and ragged tails; the full-size T = 2^20 case is in test_gpu_fullsize.py.
"""
import json
import os

import numpy as np
import pytest
import torch

import oracle as O
from helpers import relerr
from lqt_layout import dense_to_soa, soa_to_dense
from paper_2212_11744_amd import lqt
from paper_2212_11744_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
TOL = {torch.float64: 1e-9, torch.float32: 1e-4}


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _check_solution(p, out, ref, dtype, b=0, label=""):
    tol = TOL[dtype]
    for k in ("S", "v", "x", "u"):
        e = relerr(_np(out[k][b]), ref[k])
        assert e < tol, f"{label} {k}: {e:.3e} >= {tol:.0e}"


def _check_elements(el_gpu, el_ref, tol, label=""):
    for k in ("A", "b", "C", "eta", "J"):
        e = relerr(el_gpu[k], el_ref[k])
        assert e < tol, f"{label} {k}: {e:.3e}"


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lqt.lib()
    yield
    torch.cuda.synchronize()


def test_elements_config1():
    p = W.point_mass(1, 64, 10)
    dp = lqt.DeviceProblem.from_problems([p])
    el = soa_to_dense(_np(lqt.build_elements(dp)[0]), p.nx, p.T)
    ref = O.elements(p)
    _check_elements(el, ref, 1e-9, "config1")
    assert relerr(el["Ad"], ref["A"] - np.eye(p.nx)) < 1e-9


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_solve_config1(dtype):
    p = W.point_mass(1, 64, 10)
    ref = O.solve(p)
    dp = lqt.DeviceProblem.from_problems([p], dtype=dtype)
    out = lqt.solve(dp)
    torch.cuda.synchronize()
    _check_solution(p, out, ref, dtype, label="lqt_solve")
    # Stage-split calls give the same results.
    elts = lqt.build_elements(dp)
    S, v = lqt.scan_value(dp, elts)
    x, u = lqt.forward_traj(dp, elts, S, v)
    _check_solution(p, {"S": S, "v": v, "x": x, "u": u}, ref, dtype, label="stage calls")
    if dtype == torch.float64:
        for a, b in ((S, out["S"]), (x, out["x"]), (u, out["u"])):
            assert relerr(_np(a), _np(b)) < 1e-13


@pytest.mark.parametrize("T", [1, 2, 3, 4, 5, 7, 31, 33, 64, 65, 129, 257, 1000, 4097])
def test_ragged_horizons_fp64(T):
    nx = [1, 2, 3, 4][T % 4]
    nu = max(1, nx // 2)
    p = W.random_stable(100 + T, nx=nx, nu=nu, T=T, n=3, tf=0.01 * T + 0.5)
    ref = O.solve(p)
    dp = lqt.DeviceProblem.from_problems([p])
    out = lqt.solve(dp, keep_elements=True)
    _check_solution(p, out, ref, torch.float64, label=f"T={T} nx={nx}")
    _check_elements(soa_to_dense(_np(out["elts"][0]), nx, T), O.elements(p), 1e-9, f"T={T}")


@pytest.mark.parametrize("nx,nu", [(1, 1), (2, 1), (2, 2), (3, 1), (3, 2), (3, 3), (4, 1), (4, 2), (4, 3), (4, 4)])
def test_every_size_with_time_varying_F_and_drift(nx, nu):
    """Sampled F(t) (config-3 style) plus a sampled drift c(t), every instantiated (nx, nu)."""
    p = W.random_stable(7 * nx + nu, nx=nx, nu=nu, T=300, n=4, tf=3.0, time_varying=True)
    rng = np.random.default_rng(nx * 10 + nu)
    p.c = 0.3 * np.sin(np.linspace(0, 3, p.r.shape[0]))[:, None] * rng.standard_normal(nx)[None, :]
    ref = O.solve(p)
    out = lqt.solve(lqt.DeviceProblem.from_problems([p]))
    _check_solution(p, out, ref, torch.float64, label=f"nx={nx} nu={nu}")


def test_sampled_L():
    p = W.random_stable(5, nx=4, nu=2, T=200, n=4, tf=2.0)
    ts = W.half_step_times(p.t, p.n)
    p.L = p.L[None] * (1.0 + 0.2 * np.cos(ts))[:, None, None]
    ref = O.solve(p)
    out = lqt.solve(lqt.DeviceProblem.from_problems([p]))
    _check_solution(p, out, ref, torch.float64, label="sampled L")


def test_value_scan_from_oracle_elements():
    """Stage test: oracle elements in, GPU value scan out (only scan rounding differs)."""
    p = W.random_stable(11, nx=4, nu=2, T=777, n=4, tf=5.0)
    el = O.elements(p)
    S_ref, v_ref = O.value(el, p.Qf, p.rf)
    dp = lqt.DeviceProblem.from_problems([p])
    elts = torch.as_tensor(dense_to_soa(el, p.nx)[None], device="cuda")
    S, v = lqt.scan_value(dp, elts)
    assert relerr(_np(S[0]), S_ref) < 1e-11
    assert relerr(_np(v[0]), v_ref) < 1e-11
    x_ref, u_ref = O.trajectory(p, el, S_ref, v_ref)
    x, u = lqt.forward_traj(dp, elts, torch.as_tensor(S_ref[None], device="cuda"),
                            torch.as_tensor(v_ref[None], device="cuda"))
    assert relerr(_np(x[0]), x_ref) < 1e-11
    assert relerr(_np(u[0]), u_ref) < 1e-11


def test_scan_example_exact():
    """The printed all-prefix-sums example (Sec. II-C, Example 1) through the GPU value scan."""
    g = json.load(open(os.path.join(GOLDEN, "scan_example.json")))
    A, b, C, eta, J = W.scan_example_elements(g["a"])
    T = len(g["a"])
    el = {"A": A.reshape(T, 1, 1), "b": b.reshape(T, 1), "C": C.reshape(T, 1, 1),
          "eta": eta.reshape(T, 1), "J": J.reshape(T, 1, 1)}
    p = W.point_mass(0, T, 1, d=1)
    dp = lqt.DeviceProblem.from_problems([p])
    dp.nx, dp.nu = 1, 1
    dp.Qf = torch.zeros(1, 1, 1, dtype=torch.float64, device="cuda")
    dp.rf = torch.zeros(1, 1, dtype=torch.float64, device="cuda")
    S, v = lqt.scan_value(dp, torch.as_tensor(dense_to_soa(el, 1)[None], device="cuda"))
    assert np.array_equal(_np(v[0, :T, 0]), np.array(g["suffix"], dtype=float))
    assert not _np(S).any()


@pytest.mark.parametrize("T", [1023, 1024, 1025, 4 * 256 * 256 + 3])
def test_tree_shapes(T):
    """Horizons that give one, two and three scan-tree levels (4 blocks per lane, 256 nodes per
    wave above level 1), with ragged last nodes."""
    p = W.point_mass(3, T, 2, tf=10.0 * T / 2 ** 16)
    ref = O.solve(p)
    out = lqt.solve(lqt.DeviceProblem.from_problems([p]))
    _check_solution(p, out, ref, torch.float64, label=f"T={T}")


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_batch_matches_single_problems(dtype):
    probs = [W.point_mass(50 + i, 513, 4) for i in range(3)]
    dp = lqt.DeviceProblem.from_problems(probs, dtype=dtype)
    out = lqt.solve(dp)
    for b, p in enumerate(probs):
        _check_solution(p, out, O.solve(p), dtype, b=b, label=f"batch member {b}")
        single = lqt.solve(lqt.DeviceProblem.from_problems([p], dtype=dtype))
        for k in ("S", "x"):
            assert relerr(_np(out[k][b]), _np(single[k][0])) < (1e-13 if dtype == torch.float64 else 1e-6)


@pytest.mark.parametrize("T", [2 ** 12, 2 ** 16])
def test_point_mass_fp32_against_fp64_oracle(T):
    p = W.point_mass(2, T, 4)
    ref = O.solve(p)
    out = lqt.solve(lqt.DeviceProblem.from_problems([p], dtype=torch.float32))
    _check_solution(p, out, ref, torch.float32, label=f"fp32 T={T}")


def test_point_mass_fp64_2pow16():
    p = W.point_mass(2, 2 ** 16, 4)
    ref = O.solve(p)
    out = lqt.solve(lqt.DeviceProblem.from_problems([p]))
    _check_solution(p, out, ref, torch.float64, label="T=2^16")
