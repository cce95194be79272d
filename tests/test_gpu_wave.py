"""GPU path for state sizes above 4 (one wavefront per tuple, matrices in LDS) vs the CPU oracle.

Same tolerances as the per-lane path: normwise 1e-9 in FP64 and 1e-4 in FP32 against the FP64
oracle, for elements, value matrices, trajectories and controls.  The scan trees of this path
reduce 4 blocks per wave at the bottom level and 4 children per node above it (single solves), so
horizons around multiples and powers of 4 and 8 exercise ragged last nodes (of 1, 2 and 3
children) and one to six tree levels.  Levels of at most 512 nodes run on two waves per node
(pair products, the last node sequential); 8193 blocks give a level of 513 nodes on one wave
below levels on two.  The random time-varying nx = 16 workload
(T = 2^14, F(t) sampled) is compared at full size.
"""
import numpy as np
import pytest
import torch

import oracle as O
from helpers import relerr
from lqt_layout import dense_to_soa, soa_to_dense
from paper_2212_11744_amd import lqt
from paper_2212_11744_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {torch.float64: 1e-9, torch.float32: 1e-4}


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _check(out, ref, dtype, b=0, label=""):
    for k in ("S", "v", "x", "u"):
        e = relerr(_np(out[k][b]), ref[k])
        assert e < TOL[dtype], f"{label} {k}: {e:.3e}"


def _with_drift(p, seed):
    rng = np.random.default_rng(seed)
    p.c = 0.3 * np.sin(np.linspace(0, 3, p.r.shape[0]))[:, None] * rng.standard_normal(p.nx)[None, :]
    return p


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lqt.lib()
    yield
    torch.cuda.synchronize()


@pytest.mark.parametrize("nx,nu", [(5, 1), (5, 3), (6, 2), (7, 7), (8, 4), (11, 5), (16, 4), (16, 16)])
def test_sizes_with_time_varying_F_and_drift(nx, nu):
    p = _with_drift(W.random_stable(31 * nx + nu, nx=nx, nu=nu, T=75, n=3, tf=2.0), nx + nu)
    ref = O.solve(p)
    out = lqt.solve(lqt.DeviceProblem.from_problems([p]), keep_elements=True)
    _check(out, ref, torch.float64, label=f"nx={nx} nu={nu}")
    el = soa_to_dense(_np(out["elts"][0]), nx, p.T)
    el_ref = O.elements(p)
    for k in ("A", "b", "C", "eta", "J"):
        assert relerr(el[k], el_ref[k]) < 1e-9, f"element {k}"


@pytest.mark.parametrize("T", [1, 2, 3, 4, 5, 7, 8, 9, 17, 22, 26, 32, 63, 64, 65, 257, 513, 4097,
                               8193])
def test_tree_shapes(T):
    """One to six tree levels with 4 children per node, ragged last nodes."""
    p = W.random_stable(200 + T, nx=6, nu=3, T=T, n=2, tf=0.004 * T + 0.3, time_varying=False)
    ref = O.solve(p)
    out = lqt.solve(lqt.DeviceProblem.from_problems([p]))
    _check(out, ref, torch.float64, label=f"T={T}")


def test_stage_calls_match_fused_solve():
    p = W.random_stable(9, nx=8, nu=4, T=300, n=4, tf=3.0)
    dp = lqt.DeviceProblem.from_problems([p])
    fused = lqt.solve(dp)
    elts = lqt.build_elements(dp)
    S, v = lqt.scan_value(dp, elts)
    x, u = lqt.forward_traj(dp, elts, S, v)
    _check({"S": S, "v": v, "x": x, "u": u}, O.solve(p), torch.float64, label="split")
    for a, b in ((S, fused["S"]), (v, fused["v"]), (x, fused["x"]), (u, fused["u"])):
        assert relerr(_np(a), _np(b)) < 1e-13


def test_value_scan_and_trajectory_from_oracle_elements():
    """Stage test with the oracle's elements as input: only the scans' rounding differs."""
    p = W.random_stable(12, nx=10, nu=3, T=150, n=4, tf=3.0)
    el = O.elements(p)
    S_ref, v_ref = O.value(el, p.Qf, p.rf)
    x_ref, u_ref = O.trajectory(p, el, S_ref, v_ref)
    dp = lqt.DeviceProblem.from_problems([p])
    elts = torch.as_tensor(dense_to_soa(el, p.nx)[None], device="cuda")
    S, v = lqt.scan_value(dp, elts)
    assert relerr(_np(S[0]), S_ref) < 1e-11
    assert relerr(_np(v[0]), v_ref) < 1e-11
    x, u = lqt.forward_traj(dp, elts, torch.as_tensor(S_ref[None], device="cuda"),
                            torch.as_tensor(v_ref[None], device="cuda"))
    assert relerr(_np(x[0]), x_ref) < 1e-11
    assert relerr(_np(u[0]), u_ref) < 1e-11


def test_sampled_L():
    p = W.random_stable(15, nx=8, nu=3, T=120, n=4, tf=2.0)
    ts = W.half_step_times(p.t, p.n)
    p.L = p.L[None] * (1.0 + 0.2 * np.cos(ts))[:, None, None]
    out = lqt.solve(lqt.DeviceProblem.from_problems([p]))
    _check(out, O.solve(p), torch.float64, label="sampled L")


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_batch(dtype):
    probs = [W.random_stable(70 + i, nx=8, nu=4, T=200, n=4, tf=2.0) for i in range(3)]
    for p in probs[1:]:
        p.L = probs[0].L  # a constant L is shared by the batch
    out = lqt.solve(lqt.DeviceProblem.from_problems(probs, dtype=dtype))
    for b, p in enumerate(probs):
        _check(out, O.solve(p), dtype, b=b, label=f"member {b}")


def test_batch_one_and_two_wave_levels():
    """8 problems of 1100 blocks: a level of 69 nodes per problem (552 in the launch) on one wave
    per node under levels of 18, 5 and 2 nodes on two (ragged last nodes of 2 and 1 children)."""
    probs = [W.random_stable(90 + i, nx=6, nu=3, T=1100, n=2, tf=4.7) for i in range(8)]
    for p in probs[1:]:
        p.L = probs[0].L
    out = lqt.solve(lqt.DeviceProblem.from_problems(probs))
    for b, p in enumerate(probs):
        _check(out, O.solve(p), torch.float64, b=b, label=f"member {b}")


def test_fp32_nx16():
    p = W.random_stable(3, nx=16, nu=4, T=512, n=4, tf=10.0 * 512 / 2 ** 14)
    out = lqt.solve(lqt.DeviceProblem.from_problems([p], dtype=torch.float32))
    _check(out, O.solve(p), torch.float32, label="fp32 nx=16")


def test_random_time_varying_nx16_full_size():
    """nx = 16, nu = 4, F(t) = F0 + 0.1 sin(t) F1 sampled, T = 2^14 blocks x 4 RK4 steps on
    [0, 10], FP64: every output compared with the oracle's sequential solve."""
    p = W.random_stable(3, nx=16, nu=4, T=2 ** 14, n=4)
    ref = O.solve(p)
    out = lqt.solve(lqt.DeviceProblem.from_problems([p]))
    _check(out, ref, torch.float64, label="nx=16 T=2^14")


def test_backward_needs_small_state():
    p = W.random_stable(1, nx=6, nu=2, T=16, n=2, time_varying=False)
    dp = lqt.DeviceProblem.from_problems([p])
    out = lqt.solve(dp)
    with pytest.raises(lqt.LQTError) as ei:
        lqt.backward(dp, out["S"], out["v"], out["x"], torch.zeros_like(out["x"]))
    assert ei.value.status == lqt.LQT_EUNSUPPORTED
