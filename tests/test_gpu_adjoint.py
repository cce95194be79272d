"""GPU adjoint (lqt_backward) vs the oracle: its sequential adjoint (tape), its exact JVP (dual
numbers) along random directions, and central differences of the GPU forward pass; constant and
sampled F(t), L(t), with and without a drift c(t).

Gradients of Q, R, Qf are symmetric (derivative for symmetric perturbations), so the oracle's
entrywise gradients are symmetrised before comparison.  Tolerance: 1e-9 normwise against the
oracle; central differences (h = 1e-6) 1e-6 for Q, R and 1e-8 for r, x0 (x is affine in them).
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

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _sym(a):
    return 0.5 * (a + np.swapaxes(a, -1, -2))


def _gpu_grads(probs, W_list, dtype=torch.float64):
    dp = lqt.DeviceProblem.from_problems(probs, dtype=dtype)
    out = lqt.solve(dp)
    dLdx = torch.as_tensor(np.stack(W_list), device="cuda", dtype=dtype)
    return lqt.backward(dp, out["S"], out["v"], out["x"], dLdx)


@pytest.mark.parametrize("T,seed", [(1, 0), (5, 1), (12, 2), (65, 3), (300, 4)])
def test_adjoint_matches_sequential_adjoint(T, seed):
    p = W.point_mass(500 + seed, T, 4, tf=max(0.2, 0.04 * T))
    rng = np.random.default_rng(seed)
    Wt = rng.standard_normal((T + 1, p.nx))
    _, go = O.objective_grad(p, Wt)
    g = _gpu_grads([p], [Wt])
    for k, ref in (("Q", _sym(go["Q"])), ("R", _sym(go["R"])), ("Qf", _sym(go["Qf"])),
                   ("rf", go["rf"]), ("x0", go["x0"]), ("r", go["r"])):
        e = relerr(_np(g[k][0]), ref)
        assert e < 1e-9, f"T={T} d{k}: {e:.3e}"


@pytest.mark.parametrize("nx,nu", [(1, 1), (2, 1), (3, 2), (4, 4)])
def test_adjoint_other_sizes(nx, nu):
    p = W.random_stable(60 + nx, nx=nx, nu=nu, T=40, n=3, tf=2.0, time_varying=False)
    Wt = np.random.default_rng(nx).standard_normal((p.T + 1, nx))
    _, go = O.objective_grad(p, Wt)
    g = _gpu_grads([p], [Wt])
    for k, ref in (("Q", _sym(go["Q"])), ("R", _sym(go["R"])), ("r", go["r"]), ("x0", go["x0"])):
        assert relerr(_np(g[k][0]), ref) < 1e-9, (nx, nu, k)


def test_adjoint_large_against_dual_jvp():
    """Config-5 shape (point mass, T = 2^16, n = 4), two problems in one batch: <grad, d> vs the
    oracle's exact directional derivative along random symmetric directions."""
    T = 2 ** 16
    probs = [W.point_mass(5000 + i, T, 4) for i in range(2)]
    rng = np.random.default_rng(77)
    Ws = [rng.standard_normal((T + 1, 4)) for _ in probs]
    g = _gpu_grads(probs, Ws)
    for b, p in enumerate(probs):
        for name in ("Q", "R", "r", "x0", "Qf", "rf"):
            d = rng.standard_normal(np.shape(getattr(p, name)))
            if name in ("Q", "R", "Qf"):
                d = d + d.T
            _, df = O.objective_jvp(p, Ws[b], {name: d})
            got = float(np.sum(_np(g[name][b]) * d))
            assert abs(got - df) <= 1e-9 * max(1.0, abs(df)), (b, name, got, df)


def test_adjoint_full_size_entrywise_against_golden():
    """The differentiated workload's shape (point mass, T = 2^16 blocks x 4 RK4 steps, two problems
    in one batch): every entry of dQ, dR, dQf, drf, dx0 and dr at 64 sampled samples against the
    oracle's exact directional derivatives along unit directions (tests/golden/
    adjoint_point_mass_T2p16.json, written by make_adjoint_golden.py, which calls only the
    oracle).  1e-9 normwise per gradient (for dr, over the sampled entries)."""
    g = json.load(open(os.path.join(GOLDEN, "adjoint_point_mass_T2p16.json")))
    T, n = g["T"], g["n_steps"]
    probs = [W.point_mass(s, T, n) for s in g["seeds"]]
    Ws = [np.random.default_rng(g["w_seed0"] + b).standard_normal((T + 1, 4)) for b in range(len(probs))]
    got = _gpu_grads(probs, Ws)
    for b in range(len(probs)):
        for name, entries in g["grads"][b].items():
            ref = np.array([v for _, v in entries])
            arr = _np(got[name][b])
            mine = np.array([arr[tuple(idx)] for idx, _ in entries])
            e = relerr(mine, ref)
            assert e < 1e-9, f"problem {b} d{name}: {e:.3e} over {len(entries)} entries"


def test_autograd_function_and_central_differences():
    """Loss sum_k ||x_k - g_k||^2 through torch.autograd with the GPU adjoint, checked by central
    differences of the GPU forward pass."""
    T = 512
    p = W.point_mass(9, T, 4, tf=3.0)
    target = W.tracking_targets(19, p.t)
    dp = lqt.DeviceProblem.from_problems([p])
    gt = torch.as_tensor(target[None], device="cuda")

    def loss_of(Q, R, r, x0, Qf, rf):
        x = lqt.solve_trajectory(Q, R, r, x0, Qf, rf, dp)
        return ((x - gt) ** 2).sum()

    leaves = [dp.Q.clone().requires_grad_(), dp.R.clone().requires_grad_(),
              dp.r.clone().requires_grad_(), dp.x0.clone().requires_grad_(),
              dp.Qf.clone().requires_grad_(), dp.rf.clone().requires_grad_()]
    L = loss_of(*leaves)
    L.backward()
    rng = np.random.default_rng(3)
    for idx, (name, h, tol) in enumerate((("Q", 1e-6, 1e-6), ("R", 1e-6, 1e-6), ("r", 1.0, 1e-8),
                                          ("x0", 1.0, 1e-8), ("Qf", 1e-6, 1e-6), ("rf", 1.0, 1e-8))):
        d = torch.as_tensor(rng.standard_normal(tuple(leaves[idx].shape)), device="cuda")
        if name in ("Q", "R", "Qf"):
            d = d + d.transpose(-1, -2)
        with torch.no_grad():
            args_p = [a.detach().clone() for a in leaves]
            args_m = [a.detach().clone() for a in leaves]
            args_p[idx] += h * d
            args_m[idx] -= h * d
            fd = float((loss_of(*args_p) - loss_of(*args_m)) / (2 * h))
        ad = float((leaves[idx].grad * d).sum())
        assert abs(ad - fd) <= tol * max(1.0, abs(fd)), (name, ad, fd)


def _sampled(kind, nx, nu, T, n, seed):
    """F(t) sampled (random stable time-varying), L(t) sampled, a drift c(t), or all three."""
    p = W.random_stable(seed, nx=nx, nu=nu, T=T, n=n, tf=0.02 * T + 0.5,
                        time_varying=kind in ("F", "all"))
    ts = W.half_step_times(p.t, p.n)
    rng = np.random.default_rng(seed)
    if kind in ("L", "all"):
        p.L = np.asarray(p.L)[None] * (1.0 + 0.3 * np.sin(1.7 * ts))[:, None, None]
    if kind in ("c", "all"):
        p.c = 0.3 * np.cos(0.9 * ts)[:, None] * rng.standard_normal(nx)[None]
    return p


@pytest.mark.parametrize("kind", ["F", "L", "c", "all"])
@pytest.mark.parametrize("nx,nu,T", [(4, 2, 37), (3, 3, 20), (2, 1, 65)])
def test_adjoint_sampled_coefficients_against_tape(kind, nx, nu, T):
    """Sampled F(t), sampled L(t) (R enters through G(t) = L(t) R^-1 L(t)^T sample by sample), a
    drift c(t), and all three: every gradient against the oracle's sequential adjoint (tape),
    entrywise, 1e-9 normwise."""
    p = _sampled(kind, nx, nu, T, 3, 70 + T)
    Wt = np.random.default_rng(T).standard_normal((T + 1, nx))
    _, go = O.objective_grad(p, Wt)
    g = _gpu_grads([p], [Wt])
    for k, ref in (("Q", _sym(go["Q"])), ("R", _sym(go["R"])), ("Qf", _sym(go["Qf"])),
                   ("rf", go["rf"]), ("x0", go["x0"]), ("r", go["r"])):
        e = relerr(_np(g[k][0]), ref)
        assert e < 1e-9, f"{kind} nx={nx} nu={nu} d{k}: {e:.3e}"


def test_adjoint_sampled_all_batch_against_dual_jvp():
    """All three time-varying inputs, two problems of T = 1500 in one batch: <grad, d> against the
    oracle's exact directional derivative along random (symmetric) directions."""
    probs = [_sampled("all", 4, 2, 1500, 4, 90 + i) for i in range(2)]
    rng = np.random.default_rng(11)
    Ws = [rng.standard_normal((1501, 4)) for _ in probs]
    g = _gpu_grads(probs, Ws)
    for b, p in enumerate(probs):
        for name in ("Q", "R", "r", "x0", "Qf", "rf"):
            d = rng.standard_normal(np.shape(getattr(p, name)))
            if name in ("Q", "R", "Qf"):
                d = d + d.T
            _, df = O.objective_jvp(p, Ws[b], {name: d})
            got = float(np.sum(_np(g[name][b]) * d))
            assert abs(got - df) <= 1e-9 * max(1.0, abs(df)), (b, name, got, df)


@pytest.mark.parametrize("kind", ["const", "all"])
def test_adjoint_fp32(kind):
    """FP32 adjoint (constant coefficients; sampled F, L with a drift) against the oracle's FP64
    sequential adjoint, 1e-4 normwise."""
    if kind == "const":
        p = W.point_mass(31, 60, 4, tf=2.0)
    else:
        p = _sampled("all", 4, 2, 45, 3, 33)
    Wt = np.random.default_rng(8).standard_normal((p.T + 1, p.nx))
    _, go = O.objective_grad(p, Wt)
    g = _gpu_grads([p], [Wt], dtype=torch.float32)
    for k, ref in (("Q", _sym(go["Q"])), ("R", _sym(go["R"])), ("Qf", _sym(go["Qf"])),
                   ("rf", go["rf"]), ("x0", go["x0"]), ("r", go["r"])):
        e = relerr(_np(g[k][0]), ref)
        assert e < 1e-4, f"{kind} d{k}: {e:.3e}"


def test_backward_refuses_unsupported_sizes():
    p = W.random_stable(1, nx=5, nu=2, T=8, n=2, time_varying=True)
    dp = lqt.DeviceProblem.from_problems([p])
    out = lqt.solve(dp)
    with pytest.raises(lqt.LQTError) as ei:
        lqt.backward(dp, out["S"], out["v"], out["x"], torch.zeros_like(out["x"]))
    assert ei.value.status == lqt.LQT_EUNSUPPORTED
