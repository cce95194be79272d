"""Time-invariant path (lqt_dims.lti: F, L constant, c = 0, uniform grid) vs the CPU oracle.

The oracle integrates every block with RK4 (Theorem 8); the GPU path integrates one block per
problem with unit-impulse references and forms each block's b, eta as weighted sums of its
samples.  The two agree up to rounding: normwise 1e-9 in FP64, 1e-4 in FP32 against the oracle,
and 1e-11 against the general GPU build.  The full-size case uses the stored oracle samples of
tests/golden/fullsize_point_mass_T2p20.json.
"""
import json
import os

import numpy as np
import pytest
import torch

import oracle as O
from helpers import relerr
from lqt_layout import soa_to_dense
from paper_2212_11744_amd import lqt
from paper_2212_11744_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fullsize_point_mass_T2p20.json")
TOL = {torch.float64: 1e-9, torch.float32: 1e-4}


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _check(out, ref, dtype, b=0, label=""):
    for k in ("S", "v", "x", "u"):
        e = relerr(_np(out[k][b]), ref[k])
        assert e < TOL[dtype], f"{label} {k}: {e:.3e}"


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lqt.lib()
    yield
    torch.cuda.synchronize()


def test_elements_and_solve_config1():
    p = W.point_mass(1, 64, 10)
    dp = lqt.DeviceProblem.from_problems([p], lti=True)
    el = soa_to_dense(_np(lqt.build_elements(dp)[0]), p.nx, p.T)
    ref = O.elements(p)
    for k in ("A", "b", "C", "eta", "J"):
        assert relerr(el[k], ref[k]) < 1e-9, k
    out = lqt.solve(dp)
    _check(out, O.solve(p), torch.float64, label="lti config 1")
    gen = lqt.solve(lqt.DeviceProblem.from_problems([p]))
    for k in ("S", "v", "x", "u"):
        assert relerr(_np(out[k]), _np(gen[k])) < 1e-11, k


@pytest.mark.parametrize("nx,nu,T,n", [(1, 1, 1, 1), (2, 1, 7, 2), (3, 2, 300, 4), (4, 4, 1000, 3),
                                       (4, 1, 65, 1), (2, 2, 257, 6)])
def test_random_time_invariant(nx, nu, T, n):
    p = W.random_stable(17 * nx + T, nx=nx, nu=nu, T=T, n=n, tf=0.01 * T + 0.3, time_varying=False)
    out = lqt.solve(lqt.DeviceProblem.from_problems([p], lti=True), keep_elements=True)
    _check(out, O.solve(p), torch.float64, label=f"nx={nx} T={T} n={n}")
    el = soa_to_dense(_np(out["elts"][0]), nx, T)
    ref = O.elements(p)
    for k in ("A", "b", "C", "eta", "J"):
        assert relerr(el[k], ref[k]) < 1e-9, k


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_batch(dtype):
    probs = [W.point_mass(60 + i, 513, 4) for i in range(3)]
    out = lqt.solve(lqt.DeviceProblem.from_problems(probs, dtype=dtype, lti=True))
    for b, p in enumerate(probs):
        _check(out, O.solve(p), dtype, b=b, label=f"member {b}")


def test_point_mass_fp32_2pow16():
    p = W.point_mass(2, 2 ** 16, 4)
    out = lqt.solve(lqt.DeviceProblem.from_problems([p], dtype=torch.float32, lti=True))
    _check(out, O.solve(p), torch.float32, label="fp32")


def test_full_size_against_oracle_samples():
    with open(GOLDEN) as f:
        g = json.load(f)
    p = W.point_mass(g["seed"], g["T"], g["n_steps"])
    dp = lqt.DeviceProblem.from_problems([p], lti=True)
    out = lqt.solve(dp, ws=lqt.workspace(dp, lqt.CALL_SOLVE))
    torch.cuda.synchronize()
    idx = torch.as_tensor(g["k"], device="cuda")
    for k in ("S", "v", "x", "u"):
        got = out[k][0].index_select(0, idx).cpu().numpy()
        e = relerr(got, np.asarray(g[k]))
        assert e < 1e-9, f"{k}: {e:.3e}"


@pytest.mark.parametrize("nx,nu,T,n", [(5, 2, 1, 1), (8, 4, 300, 4), (11, 3, 65, 2), (16, 4, 129, 3),
                                       (16, 16, 9, 5)])
def test_wave_sizes_time_invariant(nx, nu, T, n):
    """State sizes 5 .. 16 (one wavefront per impulse and per block): elements and the solve
    against the oracle, and the solve against the general GPU build."""
    p = W.random_stable(23 * nx + T, nx=nx, nu=nu, T=T, n=n, tf=0.01 * T + 0.3, time_varying=False)
    out = lqt.solve(lqt.DeviceProblem.from_problems([p], lti=True), keep_elements=True)
    _check(out, O.solve(p), torch.float64, label=f"nx={nx} T={T} n={n}")
    el = soa_to_dense(_np(out["elts"][0]), nx, T)
    ref = O.elements(p)
    for k in ("A", "b", "C", "eta", "J"):
        assert relerr(el[k], ref[k]) < 1e-9, k
    gen = lqt.solve(lqt.DeviceProblem.from_problems([p]))
    for k in ("S", "v", "x", "u"):
        assert relerr(_np(out[k]), _np(gen[k])) < 1e-11, k


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_wave_batch_build(dtype):
    probs = [W.random_stable(30 + i, nx=9, nu=3, T=200, n=4, tf=2.0, time_varying=False)
             for i in range(2)]
    probs[1].F, probs[1].L = probs[0].F, probs[0].L  # constant F, L are shared by a batch
    dp = lqt.DeviceProblem.from_problems(probs, dtype=dtype, lti=True)
    e = lqt.build_elements(dp, lqt.empty_elements(dp).zero_())  # tile padding zeroed
    for b, p in enumerate(probs):
        el = soa_to_dense(_np(e[b]), 9, 200)
        ref = O.elements(p)
        for k in ("A", "b", "C", "eta", "J"):
            assert relerr(el[k], ref[k]) < TOL[dtype], (b, k)


def test_host_checks_refuse_non_uniform_grids():
    p = W.point_mass(1, 16, 2, t_grid=np.sort(np.r_[0.0, np.random.default_rng(0).uniform(0, 10, 15), 10.0]))
    with pytest.raises(ValueError):
        lqt.DeviceProblem.from_problems([p], lti=True)
