"""ctypes wrapper of the oracle library (test infrastructure only).

Every function takes a `Problem` from the seeded input generators (or plain numpy arrays) and
returns numpy float64 arrays.  Matrices are plain (A is A itself, C and J full symmetric).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

__all__ = [
    "build",
    "lib",
    "elements",
    "combine",
    "value",
    "solve",
    "trajectory",
    "dense",
    "riccati",
    "objective_jvp",
    "objective_grad",
    "pack_tuple",
    "unpack_tuple",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lqt_oracle.cpp")
_SO = os.path.join(_HERE, "liblqt_oracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (generic x86-64 code, so it runs on any host)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-o", tmp, _SRC], check=True)
        os.replace(tmp, _SO)
    return _SO


class _Problem(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("nu", ctypes.c_int32), ("T", ctypes.c_int32), ("n", ctypes.c_int32),
        ("F_sampled", ctypes.c_int32), ("L_sampled", ctypes.c_int32), ("has_c", ctypes.c_int32),
        ("t", ctypes.c_void_p), ("F", ctypes.c_void_p), ("L", ctypes.c_void_p), ("c", ctypes.c_void_p),
        ("Q", ctypes.c_void_p), ("R", ctypes.c_void_p), ("r", ctypes.c_void_p), ("Qf", ctypes.c_void_p),
        ("rf", ctypes.c_void_p), ("x0", ctypes.c_void_p),
    ]


class _Tangent(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("Q", "R", "r", "Qf", "rf", "x0")]


_lib = None


def lib():
    global _lib
    if _lib is None:
        # LQT_ORACLE_LIB: another build of lqt_oracle.cpp (the sanitizer test loads one built
        # with AddressSanitizer and UndefinedBehaviorSanitizer)
        path = os.environ.get("LQT_ORACLE_LIB")
        if not path:
            path = _SO
            if not os.path.exists(_SO):
                build(force=True)
        L = ctypes.CDLL(path)
        P = ctypes.POINTER
        d = P(ctypes.c_double)
        L.oracle_elements.argtypes = [P(_Problem), ctypes.c_int, d, d, d, d, d]
        L.oracle_combine.argtypes = [ctypes.c_int, d, d, d]
        L.oracle_value.argtypes = [ctypes.c_int, ctypes.c_int, d, d, d, d, d, d, d, d, d]
        L.oracle_solve.argtypes = [P(_Problem), ctypes.c_int, d, d, d, d]
        L.oracle_trajectory.argtypes = [P(_Problem), d, d, d, d, d, d, d]
        L.oracle_riccati.argtypes = [ctypes.c_int, ctypes.c_int, d, d, d, d, d, d, d, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_int, d, d, d, d]
        L.oracle_objective_jvp.argtypes = [P(_Problem), d, P(_Tangent), d, d]
        L.oracle_objective_grad.argtypes = [P(_Problem), d, d, d, d, d, d, d, d]
        _lib = L
    return _lib


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class _Keep:
    """Holds the contiguous float64 copies alive while the library reads them."""

    def __init__(self, prob):
        self.arrs = {k: _f64(getattr(prob, k)) for k in ("t", "F", "L", "c", "Q", "R", "r", "Qf", "rf", "x0")}
        a = self.arrs
        self.s = _Problem(
            prob.nx, prob.nu, prob.T, prob.n, int(a["F"].ndim == 3), int(a["L"].ndim == 3),
            int(a["c"] is not None),
            *[None if a[k] is None else a[k].ctypes.data for k in ("t", "F", "L", "c", "Q", "R", "r", "Qf", "rf", "x0")],
        )


def elements(prob, forward: bool = False, split: bool = False):
    """Elements a_0..a_{T-1}: dict of A, C, J (T, nx, nx) and b, eta (T, nx).  Theorem 8 by
    default, Theorem 9 with forward=True, the split block (Theorem 9 on the first floor(n/2) steps,
    Theorem 8 on the rest, joined by Lemma 7) with split=True."""
    k = _Keep(prob)
    T, nx = prob.T, prob.nx
    out = {"A": np.zeros((T, nx, nx)), "b": np.zeros((T, nx)), "C": np.zeros((T, nx, nx)),
           "eta": np.zeros((T, nx)), "J": np.zeros((T, nx, nx))}
    mode = 2 if split else int(forward)
    lib().oracle_elements(ctypes.byref(k.s), mode, *[_ptr(out[n]) for n in ("A", "b", "C", "eta", "J")])
    return out


def pack_tuple(A, b, C, eta, J):
    return np.concatenate([np.ravel(A), np.ravel(b), np.ravel(C), np.ravel(eta), np.ravel(J)]).astype(np.float64)


def unpack_tuple(v, nx):
    v = np.asarray(v)
    o = 0
    A = v[o:o + nx * nx].reshape(nx, nx); o += nx * nx
    b = v[o:o + nx]; o += nx
    C = v[o:o + nx * nx].reshape(nx, nx); o += nx * nx
    eta = v[o:o + nx]; o += nx
    J = v[o:o + nx * nx].reshape(nx, nx)
    return A, b, C, eta, J


def combine(nx, e1, e2):
    """Lemma 7 on packed tuples (see pack_tuple)."""
    e1, e2 = _f64(e1), _f64(e2)
    out = np.zeros(2 * nx * nx + 2 * nx + nx * nx)
    lib().oracle_combine(nx, _ptr(e1), _ptr(e2), _ptr(out))
    return out


def value(el, Qf, rf):
    """Value functions S (T+1, nx, nx), v (T+1, nx) from elements (dict as returned by elements)."""
    A = _f64(el["A"]); b = _f64(el["b"]); C = _f64(el["C"]); eta = _f64(el["eta"]); J = _f64(el["J"])
    T, nx = A.shape[0], A.shape[1]
    S = np.zeros((T + 1, nx, nx)); v = np.zeros((T + 1, nx))
    Qf = _f64(Qf); rf = _f64(rf)
    lib().oracle_value(nx, T, _ptr(A), _ptr(b), _ptr(C), _ptr(eta), _ptr(J), _ptr(Qf), _ptr(rf), _ptr(S), _ptr(v))
    return S, v


def solve(prob, method2: bool = False):
    """The whole discrete scheme: dict of S, v, x, u at the T+1 block boundaries."""
    k = _Keep(prob)
    T, nx, nu = prob.T, prob.nx, prob.nu
    out = {"S": np.zeros((T + 1, nx, nx)), "v": np.zeros((T + 1, nx)), "x": np.zeros((T + 1, nx)),
           "u": np.zeros((T + 1, nu))}
    lib().oracle_solve(ctypes.byref(k.s), int(method2), *[_ptr(out[n]) for n in ("S", "v", "x", "u")])
    return out


def trajectory(prob, el, S, v):
    k = _Keep(prob)
    T, nx, nu = prob.T, prob.nx, prob.nu
    x = np.zeros((T + 1, nx)); u = np.zeros((T + 1, nu))
    A, b, C = _f64(el["A"]), _f64(el["b"]), _f64(el["C"])
    S, v = _f64(S), _f64(v)
    lib().oracle_trajectory(ctypes.byref(k.s), _ptr(A), _ptr(b), _ptr(C), _ptr(S), _ptr(v), _ptr(x), _ptr(u))
    return x, u


def dense(prob, sol):
    """Values inside the blocks at the nT+1 RK4 nodes t_k + m h_k (and t_T) from the block-boundary
    solution `sol` (dict with S, v, x): dict of S, v, x, u."""
    k = _Keep(prob)
    nodes = prob.n * prob.T + 1
    nx, nu = prob.nx, prob.nu
    out = {"S": np.zeros((nodes, nx, nx)), "v": np.zeros((nodes, nx)), "x": np.zeros((nodes, nx)),
           "u": np.zeros((nodes, nu))}
    S, v, x = _f64(sol["S"]), _f64(sol["v"]), _f64(sol["x"])
    lib().oracle_dense(ctypes.byref(k.s), _ptr(S), _ptr(v), _ptr(x),
                       *[_ptr(out[n]) for n in ("S", "v", "x", "u")])
    return out


def riccati(F, L, Q, R, Qf, rf, x0, t0, tf, N, rfine, want_x=True):
    """Sequential fine-grid RK4 on the S, v ODEs and on the closed-loop state ODE.

    rfine: r at the 2N+1 times t0 + j (tf - t0) / (2N).  Returns S (N+1, nx, nx), v (N+1, nx) at
    the nodes t0 + i (tf - t0)/N and x (N/2+1, nx) at every second node.
    """
    F, L, Q, R, Qf, rf, x0, rfine = map(_f64, (F, L, Q, R, Qf, rf, x0, rfine))
    nx, nu = L.shape
    S = np.zeros((N + 1, nx, nx)); v = np.zeros((N + 1, nx))
    x = np.zeros((N // 2 + 1, nx)) if want_x else None
    lib().oracle_riccati(nx, nu, _ptr(F), _ptr(L), _ptr(Q), _ptr(R), _ptr(Qf), _ptr(rf), _ptr(x0),
                         float(t0), float(tf), int(N), _ptr(rfine), _ptr(S), _ptr(v), _ptr(x))
    return S, v, x


def objective_jvp(prob, W, tangent: dict):
    """f = sum_k <W_k, x_k> and its derivative along tangent (keys among Q, R, r, Qf, rf, x0)."""
    k = _Keep(prob)
    W = _f64(W)
    tg = {n: _f64(tangent.get(n)) for n in ("Q", "R", "r", "Qf", "rf", "x0")}
    ts = _Tangent(*[None if tg[n] is None else tg[n].ctypes.data for n in ("Q", "R", "r", "Qf", "rf", "x0")])
    f = ctypes.c_double(); df = ctypes.c_double()
    lib().oracle_objective_jvp(ctypes.byref(k.s), _ptr(W), ctypes.byref(ts), ctypes.byref(f), ctypes.byref(df))
    return f.value, df.value


def objective_grad(prob, W):
    """Sequential adjoint: gradient of sum_k <W_k, x_k> w.r.t. Q, R, r, Qf, rf, x0 (entrywise)."""
    k = _Keep(prob)
    W = _f64(W)
    nx, nu = prob.nx, prob.nu
    g = {"Q": np.zeros((nx, nx)), "R": np.zeros((nu, nu)), "r": np.zeros_like(k.arrs["r"]),
         "Qf": np.zeros((nx, nx)), "rf": np.zeros(nx), "x0": np.zeros(nx)}
    f = ctypes.c_double()
    lib().oracle_objective_grad(ctypes.byref(k.s), _ptr(W), ctypes.byref(f),
                                *[_ptr(g[n]) for n in ("Q", "R", "r", "Qf", "rf", "x0")])
    return f.value, g
