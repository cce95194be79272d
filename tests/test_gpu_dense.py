"""Values inside the blocks (Sec. VI-A: S, v by RK4 on their backward ODEs over each block, x by the
forward Theorem 9 parts and the Method 2 formula, u by the control law) on the GPU.

Against the oracle's dense output of the oracle's solve (normwise 1e-9 in FP64, 1e-4 in FP32), for
every (nx, nu) of the per-lane path, state sizes 5 .. 16 (one wavefront per block), sampled F and
L, a drift c, n = 1 (no interior nodes), T = 1, ragged tiles and batches.  At the full size (point mass, T = 2^20 blocks x 4 steps) the stored
oracle boundary values of tests/golden/fullsize_point_mass_T2p20.json give, for each sampled
block whose two ends are both stored, the oracle's interior values of that block; every output is
also checked for properties that hold at any size (boundary nodes copied unchanged, S symmetric,
the two axes of the point mass uncoupled).
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


def _run(probs, dtype=torch.float64, lti=False):
    dp = lqt.DeviceProblem.from_problems(probs, dtype=dtype, lti=lti)
    out = lqt.solve(dp)
    d = lqt.dense_output(dp, out["S"], out["v"], out["x"])
    torch.cuda.synchronize()
    return out, d


def _check(p, d, dtype, b=0, label=""):
    ref = O.dense(p, O.solve(p))
    for k in ("S", "v", "x", "u"):
        e = relerr(_np(d[k][b]), ref[k])
        assert e < TOL[dtype], f"{label} {k}: {e:.3e}"


def test_point_mass_config1():
    p = W.point_mass(1, 64, 10)
    _, d = _run([p])
    _check(p, d, torch.float64, label="point mass T=64 n=10")


@pytest.mark.parametrize("nx,nu", [(1, 1), (2, 1), (2, 2), (3, 1), (3, 2), (3, 3), (4, 1), (4, 2),
                                   (4, 3), (4, 4)])
def test_every_size_time_varying_with_drift(nx, nu):
    p = W.random_stable(13 * nx + nu, nx=nx, nu=nu, T=300, n=3, tf=3.0, time_varying=True)
    rng = np.random.default_rng(nx + 5 * nu)
    p.c = 0.3 * np.sin(np.linspace(0, 3, p.r.shape[0]))[:, None] * rng.standard_normal(nx)[None, :]
    _, d = _run([p])
    _check(p, d, torch.float64, label=f"nx={nx} nu={nu}")


def test_sampled_L():
    p = W.random_stable(5, nx=4, nu=2, T=200, n=4, tf=2.0)
    ts = W.half_step_times(p.t, p.n)
    p.L = p.L[None] * (1.0 + 0.2 * np.cos(ts))[:, None, None]
    _, d = _run([p])
    _check(p, d, torch.float64, label="sampled L")


@pytest.mark.parametrize("T,n", [(1, 1), (1, 5), (2, 2), (7, 1), (257, 6), (1025, 2)])
def test_horizon_shapes(T, n):
    p = W.random_stable(40 + T + n, nx=3, nu=2, T=T, n=n, tf=0.01 * T + 0.5, time_varying=True)
    out, d = _run([p])
    _check(p, d, torch.float64, label=f"T={T} n={n}")
    for k in ("S", "v", "x", "u"):  # block boundaries: the solve's values unchanged
        assert torch.equal(d[k][0, ::n], out[k][0]), k
    if n == 1:
        assert d["S"].shape[1] == T + 1


def test_non_uniform_grid():
    t = np.sort(np.r_[0.0, np.random.default_rng(3).uniform(0.0, 2.0, 62), 2.0])
    p = W.point_mass(4, 63, 4, t_grid=t)
    _, d = _run([p])
    _check(p, d, torch.float64, label="non-uniform grid")


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_batch(dtype):
    probs = [W.point_mass(70 + i, 513, 4) for i in range(3)]
    _, d = _run(probs, dtype=dtype)
    for b, p in enumerate(probs):
        _check(p, d, dtype, b=b, label=f"member {b}")


def test_time_invariant_dims_give_the_same_values():
    p = W.point_mass(6, 400, 4)
    _, d_lti = _run([p], lti=True)
    _, d = _run([p])
    for k in ("S", "v", "x", "u"):
        assert relerr(_np(d_lti[k]), _np(d[k])) < 1e-11, k
    _check(p, d_lti, torch.float64, label="lti")


def test_without_control_output():
    p = W.point_mass(8, 64, 3)
    dp = lqt.DeviceProblem.from_problems([p])
    out = lqt.solve(dp)
    d = lqt.dense_output(dp, out["S"], out["v"], out["x"], want_u=False)
    torch.cuda.synchronize()
    assert "u" not in d
    ref = O.dense(p, O.solve(p))
    assert relerr(_np(d["x"][0]), ref["x"]) < 1e-9


# ---- state sizes 5 .. 16 (one wavefront per block) ----

@pytest.mark.parametrize("nx,nu,T,n", [(5, 2, 40, 3), (8, 4, 65, 4), (16, 4, 20, 3), (16, 16, 3, 2),
                                       (6, 1, 1, 1), (7, 3, 1, 5), (9, 2, 9, 2)])
def test_wave_sizes_time_varying_with_drift(nx, nu, T, n):
    p = W.random_stable(19 * nx + T + n, nx=nx, nu=nu, T=T, n=n, tf=0.02 * T + 0.5,
                        time_varying=True)
    rng = np.random.default_rng(nx + 7 * nu)
    p.c = 0.3 * np.sin(np.linspace(0, 3, p.r.shape[0]))[:, None] * rng.standard_normal(nx)[None, :]
    out, d = _run([p])
    _check(p, d, torch.float64, label=f"nx={nx} nu={nu} T={T} n={n}")
    for k in ("S", "v", "x"):  # block boundaries: the solve's values unchanged
        assert torch.equal(d[k][0, ::n], out[k][0]), k
    assert relerr(_np(d["u"][0, ::n]), _np(out["u"][0])) < 1e-13


def test_wave_sampled_L():
    p = W.random_stable(6, nx=10, nu=3, T=50, n=4, tf=2.0)
    ts = W.half_step_times(p.t, p.n)
    p.L = p.L[None] * (1.0 + 0.2 * np.cos(ts))[:, None, None]
    _, d = _run([p])
    _check(p, d, torch.float64, label="sampled L nx=10")


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_wave_batch(dtype):
    probs = [W.random_stable(90 + i, nx=8, nu=2, T=70, n=4, tf=1.5) for i in range(2)]
    probs[1].L = probs[0].L  # a constant L is shared by a batch
    _, d = _run(probs, dtype=dtype)
    for b, p in enumerate(probs):
        _check(p, d, dtype, b=b, label=f"member {b}")


def test_wave_without_control_output():
    p = W.random_stable(4, nx=6, nu=2, T=30, n=3, tf=1.0)
    dp = lqt.DeviceProblem.from_problems([p])
    out = lqt.solve(dp)
    d = lqt.dense_output(dp, out["S"], out["v"], out["x"], want_u=False)
    torch.cuda.synchronize()
    assert "u" not in d
    ref = O.dense(p, O.solve(p))
    assert relerr(_np(d["x"][0]), ref["x"]) < 1e-9


def test_full_size_blocks_against_oracle():
    with open(GOLDEN) as f:
        g = json.load(f)
    p = W.point_mass(g["seed"], g["T"], g["n_steps"])
    n = p.n
    dp = lqt.DeviceProblem.from_problems([p])
    out = lqt.solve(dp, ws=lqt.workspace(dp, lqt.CALL_SOLVE))
    d = lqt.dense_output(dp, out["S"], out["v"], out["x"])
    torch.cuda.synchronize()
    # properties at every node
    S = d["S"][0]
    assert torch.equal(S, S.transpose(1, 2))
    assert not S[:, [0, 2]][:, :, [1, 3]].any()
    for k in ("S", "v", "x", "u"):
        assert torch.equal(d[k][0, ::n], out[k][0]), k
        assert torch.isfinite(d[k]).all(), k
    # sampled blocks whose two ends are stored: the oracle's interior values of that block
    pos = {k: i for i, k in enumerate(g["k"])}
    blocks = [k for k in g["k"] if k + 1 in pos]
    assert len(blocks) >= 15
    got = {name: [] for name in ("S", "v", "x", "u")}
    want = {name: [] for name in ("S", "v", "x", "u")}
    for k in blocks:
        sub = W.Problem(p.nx, p.nu, 1, n, p.t[k:k + 2].copy(), p.F, p.L, p.Q, p.R, p.Qf, p.rf,
                        p.x0, p.r[2 * n * k:2 * n * (k + 1) + 1].copy(), None, None, None)
        sol = {name: np.asarray([g[name][pos[k]], g[name][pos[k + 1]]]) for name in ("S", "v", "x")}
        ref = O.dense(sub, sol)
        for name in got:
            got[name].append(_np(d[name][0, n * k:n * k + n + 1]))
            want[name].append(ref[name])
    for name in got:
        e = relerr(np.asarray(got[name]), np.asarray(want[name]))
        assert e < 1e-9, f"{name}: {e:.3e}"
