"""Method 2 trajectory (Sec. IV-E: prefix products of conditional value functions combined with
the value function at t_k) on the GPU.

Against the oracle's Method 2 solve (normwise 1e-9 FP64, 1e-4 FP32) and against the Method 1
trajectory of the same elements and values (the two routes agree up to rounding).  Sizes span
one to three levels of the scan tree with ragged last nodes, every (nx, nu) of the per-lane path,
state sizes 5 .. 16 (one wavefront per tree node, one to five tree levels), sampled F, L, a drift
c, and batches.
"""
import json
import os

import numpy as np
import pytest
import torch

import oracle as O
from helpers import relerr
from paper_2212_11744_amd import lqt
from paper_2212_11744_amd import workloads as W

pytestmark = pytest.mark.gpu
TOL = {torch.float64: 1e-9, torch.float32: 1e-4}
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fullsize_point_mass_T2p20.json")


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lqt.lib()
    yield
    torch.cuda.synchronize()


def _run(p, dtype=torch.float64, batch=None):
    probs = batch or [p]
    dp = lqt.DeviceProblem.from_problems(probs, dtype=dtype)
    out = lqt.solve(dp, keep_elements=True)
    x2, u2 = lqt.forward_traj_method2(dp, out["elts"], out["S"], out["v"])
    torch.cuda.synchronize()
    return out, x2, u2


@pytest.mark.parametrize("T", [1, 2, 5, 64, 257, 1023, 1025, 4 * 256 * 256 + 3])
def test_point_mass_against_oracle_method2(T):
    p = W.point_mass(30 + T % 7, T, 2, tf=10.0 * T / 2 ** 16 + 0.05)
    ref = O.solve(p, method2=True)
    out, x2, u2 = _run(p)
    assert relerr(_np(x2[0]), ref["x"]) < 1e-9
    assert relerr(_np(u2[0]), ref["u"]) < 1e-9
    assert relerr(_np(x2[0]), _np(out["x"][0])) < 1e-10


@pytest.mark.parametrize("nx,nu", [(1, 1), (2, 1), (2, 2), (3, 1), (3, 2), (3, 3), (4, 1), (4, 2), (4, 3), (4, 4)])
def test_every_size_time_varying_with_drift(nx, nu):
    p = W.random_stable(11 * nx + nu, nx=nx, nu=nu, T=300, n=3, tf=3.0, time_varying=True)
    rng = np.random.default_rng(nx + 3 * nu)
    p.c = 0.3 * np.sin(np.linspace(0, 3, p.r.shape[0]))[:, None] * rng.standard_normal(nx)[None, :]
    ref = O.solve(p, method2=True)
    _, x2, u2 = _run(p)
    assert relerr(_np(x2[0]), ref["x"]) < 1e-9
    assert relerr(_np(u2[0]), ref["u"]) < 1e-9


def test_sampled_L_and_batch():
    probs = [W.random_stable(40 + i, nx=4, nu=2, T=200, n=4, tf=2.0) for i in range(3)]
    for p in probs:
        ts = W.half_step_times(p.t, p.n)
        p.L = probs[0].L[None] * (1.0 + 0.2 * np.cos(ts))[:, None, None] if np.ndim(probs[0].L) == 2 \
            else probs[0].L
    _, x2, u2 = _run(None, batch=probs)
    for b, p in enumerate(probs):
        ref = O.solve(p, method2=True)
        assert relerr(_np(x2[b]), ref["x"]) < 1e-9, b
        assert relerr(_np(u2[b]), ref["u"]) < 1e-9, b


def test_fp32():
    p = W.point_mass(2, 2 ** 12, 4, tf=10.0 * 2 ** 12 / 2 ** 16)
    ref = O.solve(p, method2=True)
    _, x2, _ = _run(p, torch.float32)
    assert relerr(_np(x2[0]), ref["x"]) < 1e-4


# ---- state sizes 5 .. 16 (one wavefront per tree node) ----

@pytest.mark.parametrize("nx,nu,T", [(5, 1, 1), (6, 3, 9), (6, 2, 27), (8, 4, 33), (11, 5, 150),
                                     (16, 4, 600), (16, 16, 7), (7, 2, 2049), (5, 2, 8193)])
def test_wave_sizes_time_varying_with_drift(nx, nu, T):
    """One to six tree levels (4 blocks per leaf, 4 children per upper node), ragged last nodes of
    1, 2 and 3 children; levels of at most 512 nodes run on two waves per node (left pair
    products), and 8193 blocks give a 513-node level on one wave below levels on two."""
    p = W.random_stable(17 * nx + T, nx=nx, nu=nu, T=T, n=3, tf=0.01 * T + 0.5, time_varying=True)
    rng = np.random.default_rng(nx + T)
    p.c = 0.3 * np.sin(np.linspace(0, 3, p.r.shape[0]))[:, None] * rng.standard_normal(nx)[None, :]
    ref = O.solve(p, method2=True)
    out, x2, u2 = _run(p)
    assert relerr(_np(x2[0]), ref["x"]) < 1e-9
    assert relerr(_np(u2[0]), ref["u"]) < 1e-9
    assert relerr(_np(x2[0]), _np(out["x"][0])) < 1e-10


def test_wave_sampled_L_and_batch():
    probs = [W.random_stable(80 + i, nx=9, nu=3, T=100, n=4, tf=2.0) for i in range(2)]
    for p in probs:
        ts = W.half_step_times(p.t, p.n)
        p.L = probs[0].L[None] * (1.0 + 0.2 * np.cos(ts))[:, None, None] if np.ndim(probs[0].L) == 2 \
            else probs[0].L
    _, x2, u2 = _run(None, batch=probs)
    for b, p in enumerate(probs):
        ref = O.solve(p, method2=True)
        assert relerr(_np(x2[b]), ref["x"]) < 1e-9, b
        assert relerr(_np(u2[b]), ref["u"]) < 1e-9, b


def test_wave_fp32():
    p = W.random_stable(3, nx=16, nu=4, T=256, n=4, tf=10.0 * 256 / 2 ** 14)
    ref = O.solve(p, method2=True)
    _, x2, _ = _run(p, torch.float32)
    assert relerr(_np(x2[0]), ref["x"]) < 1e-4


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_full_size_against_oracle_samples(dtype):
    """T = 2^20 blocks x 4 steps (the benchmark's problem): Method 2 at the stored oracle samples
    (Method 1 and Method 2 give the same x up to rounding, pinned in the oracle) and against the
    GPU's Method 1 trajectory on every boundary."""
    with open(GOLDEN) as f:
        g = json.load(f)
    p = W.point_mass(g["seed"], g["T"], g["n_steps"])
    out, x2, u2 = _run(p, dtype)
    idx = torch.as_tensor(g["k"], device="cuda")
    for got, name in ((x2, "x"), (u2, "u")):
        e = relerr(got[0].index_select(0, idx).double().cpu().numpy(), np.asarray(g[name]))
        assert e < TOL[dtype], f"{name}: {e:.3e}"
    assert relerr(_np(x2[0]), _np(out["x"][0])) < (1e-10 if dtype == torch.float64 else 1e-4)
