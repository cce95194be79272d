"""Element builds from the forward conditional ODEs (Theorem 9, Sec. IV-C) and with every block
split in two (Sec. IV-D: Theorem 9 on the first floor(n/2) RK4 steps, Theorem 8 on the rest,
joined by Lemma 7) on the GPU vs the oracle's builds of the same kind: normwise 1e-9 in FP64,
1e-4 in FP32; per-lane kernels for nx <= 4, one wavefront per block for nx 5 .. 16.  These builds and the backward build describe the same conditional value functions,
so they agree only to the order of RK4: their difference falls by about 2^4 when the number of
steps per block doubles.  Value functions and trajectories computed from these elements are
compared with the oracle's fold and trajectory of the oracle's elements of the same kind.
"""
import numpy as np
import pytest
import torch

import oracle as O
from helpers import relerr
from lqt_layout import soa_to_dense
from paper_2212_11744_amd import lqt
from paper_2212_11744_amd import workloads as W

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


MODES = ["forward", "split"]


def _elements(p, dtype=torch.float64, mode="forward"):
    dp = lqt.DeviceProblem.from_problems([p], dtype=dtype)
    f = lqt.build_elements_forward if mode == "forward" else lqt.build_elements_split
    return dp, f(dp)


def _ref(p, mode):
    return O.elements(p, forward=mode == "forward", split=mode == "split")


def _check_el(el, ref, tol, label):
    for k in ("A", "b", "C", "eta", "J"):
        e = relerr(el[k], ref[k])
        assert e < tol, f"{label} {k}: {e:.3e}"


@pytest.fixture(scope="module", autouse=True)
def _device():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lqt.lib()
    yield
    torch.cuda.synchronize()


@pytest.mark.parametrize("mode", MODES)
def test_config1(mode):
    p = W.point_mass(1, 64, 10)
    _, e = _elements(p, mode=mode)
    _check_el(soa_to_dense(_np(e[0]), p.nx, p.T), _ref(p, mode), 1e-9, "config 1")


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("nx,nu,T", [(1, 1, 5), (2, 1, 33), (3, 2, 257), (4, 2, 300), (4, 4, 1)])
def test_time_varying_with_drift(nx, nu, T, mode):
    p = W.random_stable(5 * nx + T, nx=nx, nu=nu, T=T, n=3, tf=0.01 * T + 0.5, time_varying=True)
    rng = np.random.default_rng(nx)
    p.c = 0.3 * np.sin(np.linspace(0, 3, p.r.shape[0]))[:, None] * rng.standard_normal(nx)[None, :]
    _, e = _elements(p, mode=mode)
    _check_el(soa_to_dense(_np(e[0]), nx, T), _ref(p, mode), 1e-9, f"nx={nx}")


@pytest.mark.parametrize("mode", MODES)
def test_sampled_L(mode):
    p = W.random_stable(8, nx=4, nu=3, T=100, n=4, tf=2.0)
    ts = W.half_step_times(p.t, p.n)
    p.L = p.L[None] * (1.0 + 0.2 * np.cos(ts))[:, None, None]
    _, e = _elements(p, mode=mode)
    _check_el(soa_to_dense(_np(e[0]), 4, 100), _ref(p, mode), 1e-9, "sampled L")


@pytest.mark.parametrize("mode", MODES)
def test_fp32(mode):
    p = W.point_mass(2, 4096, 4, tf=10.0 * 4096 / 2 ** 16)
    _, e = _elements(p, torch.float32, mode=mode)
    _check_el(soa_to_dense(_np(e[0]), 4, p.T), _ref(p, mode), 1e-4, "fp32")


@pytest.mark.parametrize("T,n", [(1, 1), (63, 1), (65, 2), (129, 5), (1000, 7)])
def test_split_step_counts(T, n):
    """Odd and even step counts, one step (the first part is empty), ragged last workgroups."""
    p = W.random_stable(90 + n, nx=4, nu=2, T=T, n=n, tf=0.01 * T + 0.5, time_varying=True)
    dp, e = _elements(p, mode="split")
    _check_el(soa_to_dense(_np(e[0]), 4, T), _ref(p, "split"), 1e-9, f"T={T} n={n}")
    if n == 1:
        eb = soa_to_dense(_np(lqt.build_elements(dp)[0]), 4, T)
        _check_el(soa_to_dense(_np(e[0]), 4, T), eb, 1e-14, "n=1 vs backward build")


def test_split_batch():
    probs = [W.point_mass(200 + i, 300, 6) for i in range(3)]
    dp = lqt.DeviceProblem.from_problems(probs)
    e = lqt.build_elements_split(dp)
    for b, p in enumerate(probs):
        _check_el(soa_to_dense(_np(e[b]), 4, 300), _ref(p, "split"), 1e-9, f"member {b}")


@pytest.mark.parametrize("mode", MODES)
def test_value_and_trajectory_from_these_elements(mode):
    p = W.random_stable(21, nx=4, nu=2, T=500, n=4, tf=5.0)
    dp, e = _elements(p, mode=mode)
    S, v = lqt.scan_value(dp, e)
    x, u = lqt.forward_traj(dp, e, S, v)
    el = _ref(p, mode)
    S_ref, v_ref = O.value(el, p.Qf, p.rf)
    x_ref, u_ref = O.trajectory(p, el, S_ref, v_ref)
    for got, ref, name in ((S, S_ref, "S"), (v, v_ref, "v"), (x, x_ref, "x"), (u, u_ref, "u")):
        assert relerr(_np(got[0]), ref) < 1e-9, name


@pytest.mark.parametrize("mode", MODES)
def test_agrees_with_backward_build_at_fourth_order(mode):
    """GPU forward (or split) vs GPU backward build of the point-mass elements (as the oracle's
    own pin): the gap shrinks by about 16 when the number of RK4 steps per block doubles."""
    gaps = []
    for n in (10, 20):
        p = W.point_mass(1, 8, n)
        dp = lqt.DeviceProblem.from_problems([p])
        _, e = _elements(p, mode=mode)
        ef = soa_to_dense(_np(e[0]), 4, 8)
        eb = soa_to_dense(_np(lqt.build_elements(dp)[0]), 4, 8)
        gaps.append(max(relerr(ef[k], eb[k]) for k in ("A", "b", "C", "eta", "J")))
    assert gaps[1] < 5e-5 and 12.0 < gaps[0] / gaps[1] < 20.0, gaps


# ---- state sizes 5 .. 16 (one wavefront per block, matrices in LDS) ----

@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("nx,nu,T", [(5, 1, 3), (6, 2, 70), (8, 4, 129), (11, 5, 40), (16, 4, 33),
                                     (16, 16, 7)])
def test_wave_sizes_time_varying_with_drift(nx, nu, T, mode):
    p = W.random_stable(7 * nx + T, nx=nx, nu=nu, T=T, n=3, tf=0.01 * T + 0.5, time_varying=True)
    rng = np.random.default_rng(nx + 100)
    p.c = 0.3 * np.sin(np.linspace(0, 3, p.r.shape[0]))[:, None] * rng.standard_normal(nx)[None, :]
    _, e = _elements(p, mode=mode)
    _check_el(soa_to_dense(_np(e[0]), nx, T), _ref(p, mode), 1e-9, f"nx={nx} nu={nu}")


@pytest.mark.parametrize("mode", MODES)
def test_wave_sampled_L(mode):
    p = W.random_stable(18, nx=9, nu=3, T=60, n=4, tf=2.0)
    ts = W.half_step_times(p.t, p.n)
    p.L = p.L[None] * (1.0 + 0.2 * np.cos(ts))[:, None, None]
    _, e = _elements(p, mode=mode)
    _check_el(soa_to_dense(_np(e[0]), 9, 60), _ref(p, mode), 1e-9, "sampled L")


@pytest.mark.parametrize("mode", MODES)
def test_wave_fp32(mode):
    p = W.random_stable(3, nx=16, nu=4, T=256, n=4, tf=10.0 * 256 / 2 ** 14)
    _, e = _elements(p, torch.float32, mode=mode)
    _check_el(soa_to_dense(_np(e[0]), 16, p.T), _ref(p, mode), 1e-4, "fp32 nx=16")


@pytest.mark.parametrize("T,n", [(1, 1), (9, 2), (17, 5)])
def test_wave_split_step_counts(T, n):
    p = W.random_stable(40 + n, nx=7, nu=3, T=T, n=n, tf=0.05 * T + 0.5, time_varying=True)
    dp, e = _elements(p, mode="split")
    _check_el(soa_to_dense(_np(e[0]), 7, T), _ref(p, "split"), 1e-9, f"T={T} n={n}")
    if n == 1:
        eb = soa_to_dense(_np(lqt.build_elements(dp)[0]), 7, T)
        _check_el(soa_to_dense(_np(e[0]), 7, T), eb, 1e-13, "n=1 vs backward build")


@pytest.mark.parametrize("mode", MODES)
def test_wave_batch_and_scans(mode):
    """Two problems of nx = 8 in one batch; value functions and trajectories from these elements
    against the oracle's fold and trajectory of its elements of the same kind."""
    probs = [W.random_stable(60 + i, nx=8, nu=4, T=150, n=4, tf=3.0) for i in range(2)]
    probs[1].L = probs[0].L  # a constant L is shared by a batch
    dp = lqt.DeviceProblem.from_problems(probs)
    f = lqt.build_elements_forward if mode == "forward" else lqt.build_elements_split
    e = f(dp)
    S, v = lqt.scan_value(dp, e)
    x, u = lqt.forward_traj(dp, e, S, v)
    for b, p in enumerate(probs):
        el = _ref(p, mode)
        _check_el(soa_to_dense(_np(e[b]), 8, 150), el, 1e-9, f"member {b}")
        S_ref, v_ref = O.value(el, p.Qf, p.rf)
        x_ref, u_ref = O.trajectory(p, el, S_ref, v_ref)
        for got, ref, name in ((S, S_ref, "S"), (v, v_ref, "v"), (x, x_ref, "x"), (u, u_ref, "u")):
            assert relerr(_np(got[b]), ref) < 1e-9, (b, name)


@pytest.mark.parametrize("mode", MODES)
def test_wave_agrees_with_backward_build_at_fourth_order(mode):
    gaps = []
    for n in (10, 20):
        p = W.random_stable(5, nx=6, nu=2, T=6, n=n, tf=3.0, time_varying=False)
        dp = lqt.DeviceProblem.from_problems([p])
        _, e = _elements(p, mode=mode)
        ef = soa_to_dense(_np(e[0]), 6, 6)
        eb = soa_to_dense(_np(lqt.build_elements(dp)[0]), 6, 6)
        gaps.append(max(relerr(ef[k], eb[k]) for k in ("A", "b", "C", "eta", "J")))
    assert gaps[1] < 5e-5 and 12.0 < gaps[0] / gaps[1] < 20.0, gaps
