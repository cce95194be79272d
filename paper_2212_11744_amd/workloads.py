"""Seeded synthetic LQT workloads.

Input generation only: random draws, the problem matrices and the evaluation of the synthetic
reference signals.  No step of the solver (element ODEs, combination rule, scans) lives here, so
both the GPU path and the CPU oracle can take their inputs from this module.

Workloads follow the continuous-time LQT experiment of the paper (Section 6.1, point mass with
state [p_x, p_y, v_x, v_y] driven by accelerations).  The paper's reference trajectory was a
Fourier fit to data that is not available, so a seeded sum of sinusoids per axis stands in for it.

Sampling convention (shared by the GPU path and the oracle): every time-varying input (r, and F, L,
c when sampled) is given on the half-step grid of the RK4 integrator.  Block k = [t_k, t_{k+1}] is
integrated with n RK4 steps of h_k = (t_{k+1} - t_k) / n, and sample j of block k sits at
t_k + j * h_k / 2, j = 0..2n, with global index 2*n*k + j (block ends are shared), so a horizon of
T blocks has 2*n*T + 1 samples.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np

__all__ = [
    "Problem",
    "half_step_times",
    "point_mass",
    "random_stable",
    "batched_mix",
    "tracking_targets",
    "scan_example_elements",
]


@dataclass
class Problem:
    """One LQT problem in the paper's notation with H = I (state-space reference).

    F, L: (nx, nx), (nx, nu) if constant, else sampled (2nT+1, nx, nx), (2nT+1, nx, nu).
    c: None (zero) or sampled (2nT+1, nx).  Q = H^T X H (nx, nx), R = U (nu, nu),
    Qf = H_f^T X_f H_f, rf the terminal reference (state space), r sampled (2nT+1, nx).
    """

    nx: int
    nu: int
    T: int
    n: int
    t: np.ndarray
    F: np.ndarray
    L: np.ndarray
    Q: np.ndarray
    R: np.ndarray
    Qf: np.ndarray
    rf: np.ndarray
    x0: np.ndarray
    r: np.ndarray
    c: Optional[np.ndarray] = None
    ref: Optional[Callable[[np.ndarray], np.ndarray]] = field(default=None, repr=False)
    F_of_t: Optional[Callable[[np.ndarray], np.ndarray]] = field(default=None, repr=False)

    @property
    def F_sampled(self) -> bool:
        return self.F.ndim == 3

    @property
    def L_sampled(self) -> bool:
        return self.L.ndim == 3

    def astype(self, dtype) -> "Problem":
        cast = lambda a: None if a is None else np.ascontiguousarray(a, dtype=dtype)
        return Problem(self.nx, self.nu, self.T, self.n, cast(self.t), cast(self.F), cast(self.L),
                       cast(self.Q), cast(self.R), cast(self.Qf), cast(self.rf), cast(self.x0),
                       cast(self.r), cast(self.c), self.ref, self.F_of_t)


def half_step_times(t: np.ndarray, n: int) -> np.ndarray:
    """Times of the 2nT+1 half-step samples for block boundaries t (length T+1)."""
    t = np.asarray(t, dtype=np.float64)
    T = t.size - 1
    h = (t[1:] - t[:-1]) / n
    j = np.arange(2 * n)
    out = np.empty(2 * n * T + 1)
    out[:-1] = (t[:-1, None] + j[None, :] * (h[:, None] / 2.0)).reshape(-1)
    out[-1] = t[-1]
    return out


def _sinusoids(rng: np.random.Generator, n_axes: int, n_terms: int, amp, freq):
    params = []
    for _ in range(n_axes):
        a = rng.uniform(amp[0], amp[1], n_terms)
        f = rng.uniform(freq[0], freq[1], n_terms)
        ph = rng.uniform(0.0, 2.0 * np.pi, n_terms)
        params.append((a, f, ph))
    return params


def _eval_sinusoids(params, ts: np.ndarray, derivative: bool = False) -> np.ndarray:
    ts = np.asarray(ts, dtype=np.float64)
    out = np.zeros((ts.size, len(params)))
    for i, (a, f, ph) in enumerate(params):
        w = 2.0 * np.pi * f
        arg = ts[:, None] * w[None, :] + ph[None, :]
        if derivative:
            out[:, i] = (np.cos(arg) * (a * w)[None, :]).sum(axis=1)
        else:
            out[:, i] = (np.sin(arg) * a[None, :]).sum(axis=1)
    return out


def _point_mass_matrices(d: int):
    nx, nu = 2 * d, d
    F = np.zeros((nx, nx))
    F[:d, d:] = np.eye(d)
    L = np.zeros((nx, nu))
    L[d:, :] = np.eye(d)
    Q = np.diag(np.r_[np.ones(d), np.zeros(d)])
    R = 0.1 * np.eye(nu)
    Qf = np.diag(np.r_[10.0 * np.ones(d), np.zeros(d)])
    return F, L, Q, R, Qf


def point_mass(seed: int, T: int, n: int, t0: float = 0.0, tf: float = 10.0, d: int = 2,
               t_grid: Optional[np.ndarray] = None) -> Problem:
    """Point mass in d axes (d=2 is the paper's model): x = [positions, velocities].

    Q = diag(1 on positions, 0 on velocities), R = 0.1 I, Qf = diag(10 on positions, 0).
    Reference per axis: sum of 4 sinusoids, amplitude U[0.5, 2], frequency U[0.1, 1] Hz, phase
    U[0, 2 pi); the velocity reference is its derivative.  rf = r(tf).  x0 ~ N(0, I).
    Draw order: per axis (amplitudes, frequencies, phases), then x0.
    """
    rng = np.random.default_rng(seed)
    params = _sinusoids(rng, d, 4, (0.5, 2.0), (0.1, 1.0))
    x0 = rng.standard_normal(2 * d)
    F, L, Q, R, Qf = _point_mass_matrices(d)

    def ref(ts):
        ts = np.atleast_1d(np.asarray(ts, dtype=np.float64))
        return np.concatenate([_eval_sinusoids(params, ts), _eval_sinusoids(params, ts, True)], axis=1)

    t = np.linspace(t0, tf, T + 1) if t_grid is None else np.asarray(t_grid, dtype=np.float64)
    r = ref(half_step_times(t, n))
    rf = ref(np.array([t[-1]]))[0]
    return Problem(2 * d, d, T, n, t, F, L, Q, R, Qf, rf, x0, r, None, ref)


def _haar_orthogonal(rng: np.random.Generator, m: int) -> np.ndarray:
    Z = rng.standard_normal((m, m))
    Qm, Rm = np.linalg.qr(Z)
    return Qm * np.sign(np.diag(Rm))[None, :]


def random_stable(seed: int, nx: int = 16, nu: int = 4, T: int = 2 ** 14, n: int = 4,
                  t0: float = 0.0, tf: float = 10.0, time_varying: bool = True) -> Problem:
    """Random stable LQT.  F(t) = F0 + 0.1 sin(t) F1, sampled on the half-step grid.

    F0 = O blockdiag([[s_i, w_i], [-w_i, s_i]]) O^T with s_i ~ U[-1, -0.05], w_i ~ U[0, 1] and O
    Haar orthogonal (eigenvalue real parts in [-1, -0.05]); F1 entries ~ N(0, 1/nx);
    L entries ~ N(0, 1/nu); Q = Oq diag(U[0.1, 2]) Oq^T; R = Or diag(U[0.05, 1]) Or^T.
    Reference: every state component a sum of 4 sinusoids (amplitude U[0.5, 2], frequency
    U[0.1, 1] Hz).  Qf = Q, rf = r(tf), x0 ~ N(0, I).  With time_varying=False, F = F0 (constant).
    """
    rng = np.random.default_rng(seed)
    O = _haar_orthogonal(rng, nx)
    blocks = np.zeros((nx, nx))
    for i in range(nx // 2):
        s = rng.uniform(-1.0, -0.05)
        w = rng.uniform(0.0, 1.0)
        blocks[2 * i:2 * i + 2, 2 * i:2 * i + 2] = [[s, w], [-w, s]]
    if nx % 2:
        blocks[-1, -1] = rng.uniform(-1.0, -0.05)
    F0 = O @ blocks @ O.T
    F1 = rng.standard_normal((nx, nx)) / np.sqrt(nx)
    L = rng.standard_normal((nx, nu)) / np.sqrt(nu)
    Oq = _haar_orthogonal(rng, nx)
    Q = Oq @ np.diag(rng.uniform(0.1, 2.0, nx)) @ Oq.T
    Q = 0.5 * (Q + Q.T)
    Or = _haar_orthogonal(rng, nu)
    R = Or @ np.diag(rng.uniform(0.05, 1.0, nu)) @ Or.T
    R = 0.5 * (R + R.T)
    params = _sinusoids(rng, nx, 4, (0.5, 2.0), (0.1, 1.0))
    x0 = rng.standard_normal(nx)

    def ref(ts):
        return _eval_sinusoids(params, np.atleast_1d(np.asarray(ts, dtype=np.float64)))

    t = np.linspace(t0, tf, T + 1)
    ts = half_step_times(t, n)
    r = ref(ts)
    rf = ref(np.array([tf]))[0]
    if time_varying:
        F_of_t = lambda tt: F0[None] + 0.1 * np.sin(np.asarray(tt))[:, None, None] * F1[None]
        F = F_of_t(ts)
    else:
        F_of_t = lambda tt: np.broadcast_to(F0, (np.size(tt), nx, nx)).copy()
        F = F0.copy()
    return Problem(nx, nu, T, n, t, F, L, Q, R, Q.copy(), rf, x0, r, None, ref, F_of_t)


def batched_mix(seed: int = 4, count: int = 1024, n: int = 4, block: float = 10.0 / 1024,
                t_min: int = 256, t_max: int = 8192, nx_cycle=(2, 4, 8)):
    """Many problems of uneven horizons and state sizes.

    Problem i has nx = nx_cycle[i mod len], nu = nx / 2; it is a point mass in nx/2 axes when i is
    even and a time-invariant random stable system otherwise.  T_i ~ U{t_min..t_max}; every block
    has the same length, so horizons differ.  Seeds of the members derive from `seed`.
    """
    rng = np.random.default_rng(seed)
    Ts = rng.integers(t_min, t_max + 1, size=count)
    out = []
    for i in range(count):
        nx = nx_cycle[i % len(nx_cycle)]
        T = int(Ts[i])
        tf = T * block
        sub = seed * 100000 + i
        if i % 2 == 0:
            out.append(point_mass(sub, T, n, 0.0, tf, d=nx // 2))
        else:
            out.append(random_stable(sub, nx, nx // 2, T, n, 0.0, tf, time_varying=False))
    return out


def tracking_targets(seed: int, t: np.ndarray, d: int = 2) -> np.ndarray:
    """Smooth target g(t_k) for a trajectory loss: positions are sums of 3 sinusoids (amplitude
    U[0.5, 2], frequency U[0.05, 0.5] Hz), velocities their derivatives.  Shape (t.size, 2d)."""
    rng = np.random.default_rng(seed)
    params = _sinusoids(rng, d, 3, (0.5, 2.0), (0.05, 0.5))
    return np.concatenate([_eval_sinusoids(params, t), _eval_sinusoids(params, t, True)], axis=1)


def scan_example_elements(values):
    """Scalar (nx = 1) tuples whose combination reduces to addition.

    With A = 1, C = 0, J = 0 the combination rule adds b and eta, so a reverse scan of these
    elements, closed by a terminal tuple, yields reverse cumulative sums and a forward scan
    yields cumulative sums: the all-prefix-sums example printed in the paper (Section 2.3).
    Returns (A, b, C, eta, J) arrays of shape (T,) with b = eta = values.
    """
    v = np.asarray(values, dtype=np.float64)
    return np.ones_like(v), v.copy(), np.zeros_like(v), v.copy(), np.zeros_like(v)
