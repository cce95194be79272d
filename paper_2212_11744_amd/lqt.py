"""Python binding of the C ABI in include/lqt.h (argument marshalling only).

Every stage runs in the gfx950 HIP library `liblqt.so`; this module turns torch tensors into
device pointers, allocates outputs and workspaces with torch, passes the current HIP stream and
raises on error.  There is no fallback: if the library is missing or does not load, every entry
point raises.  Functions mirror the C entry points:

    build_elements(prob) -> elts
    scan_value(prob, elts) -> S, v
    forward_traj(prob, elts, S, v) -> x, u
    solve(prob) -> dict(elts?, S, v, x, u)
    backward(prob, S, v, x, dLdx) -> dict of gradients

`prob` is a `DeviceProblem`: the arrays of one or more equally sized problems resident on the GPU.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# LQT_LIBRARY: another build of the same sources (the sanitizer test loads one whose host code is
# built with AddressSanitizer and UndefinedBehaviorSanitizer)
LIB_PATH = os.environ.get("LQT_LIBRARY") or os.path.join(_HERE, "liblqt.so")

LQT_OK, LQT_EINVAL, LQT_EUNSUPPORTED, LQT_EWORKSPACE, LQT_EHIP, LQT_ENONFINITE = 0, -1, -2, -3, -4, -5
LQT_F64, LQT_F32 = 0, 1
CALL_BUILD, CALL_SCAN_VALUE, CALL_FORWARD_TRAJ, CALL_SOLVE, CALL_BACKWARD, CALL_TRAJ_METHOD2 = range(6)


class LQTError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"lqt status {status}: {message}")
        self.status = status


class Dims(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in
                ("nx", "nu", "T", "n_steps", "batch", "dtype", "F_sampled", "L_sampled", "has_c",
                 "lti")]


class Problem(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("t", "F", "L", "c", "Q", "R", "r", "Qf", "rf", "x0")]


class Ragged(ctypes.Structure):
    """lqt_ragged: one class of the batched solve (include/lqt.h)."""
    _fields_ = [(n, ctypes.c_int32) for n in
                ("nx", "nu", "n_steps", "dtype", "count", "F_sampled", "L_sampled", "has_c")] + [
        ("rows", ctypes.c_int64), ("start", ctypes.c_void_p), ("prob", Problem),
        ("S", ctypes.c_void_p), ("v", ctypes.c_void_p), ("x", ctypes.c_void_p), ("u", ctypes.c_void_p)]


LQT_PLAN_AUTOTUNE, LQT_PLAN_GRAPH = 1, 2

_lib = None


def lib():
    """Load liblqt.so (raises if it is missing: there is no CPU fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} not found: build it with `python -m paper_2212_11744_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        vp, sz, st = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p
        L.lqt_debug_canary.argtypes = [ctypes.c_int32]
        L.lqt_debug_canary.restype = None
        L.lqt_debug_fail_launch.argtypes = [ctypes.c_int32]
        L.lqt_debug_fail_launch.restype = None
        L.lqt_element_count.argtypes = [ctypes.c_int32]
        L.lqt_element_count.restype = sz
        L.lqt_workspace_size.argtypes = [P(Dims), ctypes.c_int]
        L.lqt_workspace_size.restype = sz
        L.lqt_build_elements.argtypes = [P(Dims), P(Problem), vp, vp, sz, st]
        L.lqt_build_elements_forward.argtypes = [P(Dims), P(Problem), vp, vp, sz, st]
        L.lqt_build_elements_split.argtypes = [P(Dims), P(Problem), vp, vp, sz, st]
        L.lqt_scan_value.argtypes = [P(Dims), vp, vp, vp, vp, vp, vp, sz, st]
        L.lqt_forward_traj.argtypes = [P(Dims), P(Problem), vp, vp, vp, vp, vp, vp, sz, st]
        L.lqt_forward_traj_method2.argtypes = [P(Dims), P(Problem), vp, vp, vp, vp, vp, vp, sz, st]
        L.lqt_dense_output.argtypes = [P(Dims), P(Problem), vp, vp, vp, vp, vp, vp, vp, vp, sz, st]
        L.lqt_solve.argtypes = [P(Dims), P(Problem), vp, vp, vp, vp, vp, vp, sz, st]
        L.lqt_solve_noalloc.argtypes = [P(Dims), P(Problem), vp, vp, vp, vp, vp, st]
        L.lqt_solve_noalloc.restype = ctypes.c_int
        L.lqt_noalloc_scratch_size.argtypes = [P(Dims)]
        L.lqt_noalloc_scratch_size.restype = sz
        L.lqt_backward.argtypes = [P(Dims), P(Problem), vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, st]
        for f in ("lqt_build_elements", "lqt_build_elements_forward", "lqt_build_elements_split",
                  "lqt_scan_value",
                  "lqt_forward_traj", "lqt_forward_traj_method2", "lqt_dense_output", "lqt_solve",
                  "lqt_backward"):
            getattr(L, f).restype = ctypes.c_int
        L.lqt_batched_workspace_size.argtypes = [P(Ragged), ctypes.c_int32]
        L.lqt_batched_workspace_size.restype = sz
        L.lqt_solve_batched.argtypes = [P(Ragged), ctypes.c_int32, vp, sz, st]
        L.lqt_solve_batched.restype = ctypes.c_int
        L.lqt_plan_create.argtypes = [P(Ragged), ctypes.c_int32, vp, sz, ctypes.c_int32, st, P(vp)]
        L.lqt_plan_create.restype = ctypes.c_int
        L.lqt_plan_launch.argtypes = [vp, st]
        L.lqt_plan_launch.restype = ctypes.c_int
        L.lqt_plan_config.argtypes = [vp]
        L.lqt_plan_config.restype = ctypes.c_char_p
        L.lqt_plan_destroy.argtypes = [vp]
        L.lqt_plan_destroy.restype = None
        L.lqt_status_string.argtypes = [ctypes.c_int]
        L.lqt_status_string.restype = ctypes.c_char_p
        L.lqt_last_error.restype = ctypes.c_char_p
        L.lqt_version.restype = ctypes.c_int32
        _lib = L
    return _lib


def _check(status: int):
    if status != LQT_OK:
        raise LQTError(status, lib().lqt_last_error().decode())


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


@dataclass
class DeviceProblem:
    """Arrays of `batch` equally sized LQT problems on the GPU (layouts of include/lqt.h)."""

    nx: int
    nu: int
    T: int
    n: int
    batch: int
    dtype: torch.dtype
    t: torch.Tensor
    F: torch.Tensor
    L: torch.Tensor
    Q: torch.Tensor
    R: torch.Tensor
    r: torch.Tensor
    Qf: torch.Tensor
    rf: torch.Tensor
    x0: torch.Tensor
    c: Optional[torch.Tensor] = None
    F_sampled: bool = False
    L_sampled: bool = False
    lti: bool = False  # time-invariant path (lqt_dims.lti): F, L constant, c = 0, uniform grid

    @property
    def nsamp(self) -> int:
        return 2 * self.n * self.T + 1

    def dims(self) -> Dims:
        return Dims(self.nx, self.nu, self.T, self.n, self.batch,
                    LQT_F64 if self.dtype == torch.float64 else LQT_F32,
                    int(self.F_sampled), int(self.L_sampled), int(self.c is not None),
                    int(self.lti))

    def ptrs(self) -> Problem:
        return Problem(*[None if getattr(self, k) is None else getattr(self, k).data_ptr()
                         for k in ("t", "F", "L", "c", "Q", "R", "r", "Qf", "rf", "x0")])

    @classmethod
    def from_problems(cls, problems: Sequence, dtype=torch.float64, device="cuda",
                      lti: bool = False) -> "DeviceProblem":
        """Stack host problems (objects with the fields of `workloads.Problem`) onto the device.
        All members must share nx, nu, T, n and, when constant, F and L.  lti=True selects the
        time-invariant path; it is checked here on the host data (constant F and L, no drift,
        block lengths equal to within 1e-12 relative)."""
        p0 = problems[0]
        for p in problems:
            if (p.nx, p.nu, p.T, p.n) != (p0.nx, p0.nu, p0.T, p0.n):
                raise ValueError("batched problems must share nx, nu, T and n")
        F_s, L_s = np.ndim(p0.F) == 3, np.ndim(p0.L) == 3
        has_c = getattr(p0, "c", None) is not None
        for i, p in enumerate(problems):
            _check_arrays(p, i, F_s, L_s, has_c)
        for name, sampled in (("F", F_s), ("L", L_s)):
            if not sampled and any(not np.array_equal(getattr(p, name), getattr(p0, name)) for p in problems):
                raise ValueError(f"a constant {name} is shared by the batch: members differ")
        to = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=device)
        stack = lambda name: to(np.stack([np.asarray(getattr(p, name)) for p in problems]))
        if lti:
            if F_s or L_s or has_c:
                raise ValueError("the time-invariant path needs constant F, L and no drift")
            for p in problems:
                d = np.diff(np.asarray(p.t, dtype=np.float64))
                if np.max(np.abs(d - d[0])) > 1e-12 * abs(d[0]):
                    raise ValueError("the time-invariant path needs a uniform grid")
        return cls(p0.nx, p0.nu, p0.T, p0.n, len(problems), dtype,
                   stack("t"), stack("F") if F_s else to(p0.F), stack("L") if L_s else to(p0.L),
                   stack("Q"), stack("R"), stack("r"), stack("Qf"), stack("rf"), stack("x0"),
                   stack("c") if has_c else None, F_s, L_s, lti)


def _check_arrays(p, i: int, F_s: bool, L_s: bool, has_c: bool) -> None:
    """Host check of one problem's arrays: the kernels index them by the dims alone, so a short
    array would be read past its end.  Also: the grid must be strictly increasing."""
    nx, nu, T, ns = p.nx, p.nu, p.T, 2 * p.n * p.T + 1
    want = {"t": (T + 1,), "F": (ns, nx, nx) if F_s else (nx, nx),
            "L": (ns, nx, nu) if L_s else (nx, nu), "Q": (nx, nx), "R": (nu, nu), "r": (ns, nx),
            "Qf": (nx, nx), "rf": (nx,), "x0": (nx,)}
    if has_c:
        want["c"] = (ns, nx)
    for name, shape in want.items():
        a = getattr(p, name, None)
        if a is None or np.shape(a) != shape:
            raise ValueError(f"problem {i}: {name} has shape {np.shape(a)}, expected {shape}")
    if (getattr(p, "c", None) is not None) != has_c:
        raise ValueError(f"problem {i}: a drift c must be given for every member or none")
    if not np.all(np.diff(np.asarray(p.t, dtype=np.float64)) > 0):
        raise ValueError(f"problem {i}: the grid t must be strictly increasing")


def element_count(nx: int) -> int:
    return int(lib().lqt_element_count(nx))


ELEMENT_TILE = 512


def element_tiles(T: int) -> int:
    """Number of 512-block tiles of the element layout."""
    return (T + ELEMENT_TILE - 1) // ELEMENT_TILE


def empty_elements(prob: "DeviceProblem") -> torch.Tensor:
    """Element array [batch][ceil(T/512)][NE][512] (tiled structure of arrays, include/lqt.h)."""
    return torch.empty(prob.batch, element_tiles(prob.T), element_count(prob.nx), ELEMENT_TILE,
                       dtype=prob.dtype, device=prob.t.device)


def workspace_size(prob: DeviceProblem, call: int) -> int:
    d = prob.dims()
    n = int(lib().lqt_workspace_size(ctypes.byref(d), call))
    if n == 0:
        raise LQTError(LQT_EINVAL, "invalid dims for workspace query")
    return n


def workspace(prob: DeviceProblem, call: int) -> torch.Tensor:
    n = workspace_size(prob, call)
    ws = torch.empty(n + 256, dtype=torch.uint8, device=prob.t.device)
    off = (-ws.data_ptr()) % 256
    return ws[off:off + n]


def _empty(prob, *shape):
    return torch.empty(*shape, dtype=prob.dtype, device=prob.t.device)


def build_elements(prob: DeviceProblem, elts: Optional[torch.Tensor] = None,
                   ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Elements [batch][ceil(T/512)][NE][512] (tiled structure of arrays, A stored as A - I)."""
    elts = empty_elements(prob) if elts is None else elts
    ws = workspace(prob, CALL_BUILD) if ws is None else ws
    d, p = prob.dims(), prob.ptrs()
    _check(lib().lqt_build_elements(ctypes.byref(d), ctypes.byref(p), _ptr(elts), _ptr(ws),
                                    ws.numel(), _stream()))
    return elts


def build_elements_forward(prob: DeviceProblem, elts: Optional[torch.Tensor] = None,
                           ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Elements from the forward conditional ODEs (Theorem 9); same layout as build_elements."""
    elts = empty_elements(prob) if elts is None else elts
    ws = workspace(prob, CALL_BUILD) if ws is None else ws
    d, p = prob.dims(), prob.ptrs()
    _check(lib().lqt_build_elements_forward(ctypes.byref(d), ctypes.byref(p), _ptr(elts), _ptr(ws),
                                            ws.numel(), _stream()))
    return elts


def build_elements_split(prob: DeviceProblem, elts: Optional[torch.Tensor] = None,
                         ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Elements with every block split: Theorem 9 on the first floor(n/2) steps, Theorem 8 on the
    rest, joined by Lemma 7; same layout as build_elements."""
    elts = empty_elements(prob) if elts is None else elts
    ws = workspace(prob, CALL_BUILD) if ws is None else ws
    d, p = prob.dims(), prob.ptrs()
    _check(lib().lqt_build_elements_split(ctypes.byref(d), ctypes.byref(p), _ptr(elts), _ptr(ws),
                                          ws.numel(), _stream()))
    return elts


def scan_value(prob: DeviceProblem, elts: torch.Tensor, S=None, v=None, ws=None):
    """Value function S [batch][T+1][nx][nx], v [batch][T+1][nx]."""
    S = _empty(prob, prob.batch, prob.T + 1, prob.nx, prob.nx) if S is None else S
    v = _empty(prob, prob.batch, prob.T + 1, prob.nx) if v is None else v
    ws = workspace(prob, CALL_SCAN_VALUE) if ws is None else ws
    d = prob.dims()
    _check(lib().lqt_scan_value(ctypes.byref(d), _ptr(elts), _ptr(prob.Qf), _ptr(prob.rf), _ptr(S),
                                _ptr(v), _ptr(ws), ws.numel(), _stream()))
    return S, v


def forward_traj(prob: DeviceProblem, elts, S, v, x=None, u=None, ws=None, want_u=True):
    """Trajectory x [batch][T+1][nx] and control u [batch][T+1][nu]."""
    x = _empty(prob, prob.batch, prob.T + 1, prob.nx) if x is None else x
    if want_u and u is None:
        u = _empty(prob, prob.batch, prob.T + 1, prob.nu)
    ws = workspace(prob, CALL_FORWARD_TRAJ) if ws is None else ws
    d, p = prob.dims(), prob.ptrs()
    _check(lib().lqt_forward_traj(ctypes.byref(d), ctypes.byref(p), _ptr(elts), _ptr(S), _ptr(v),
                                  _ptr(x), _ptr(u), _ptr(ws), ws.numel(), _stream()))
    return x, u


def forward_traj_method2(prob: DeviceProblem, elts, S, v, x=None, u=None, ws=None, want_u=True):
    """Trajectory and control by Method 2 (forward prefix scan of conditional value functions)."""
    x = _empty(prob, prob.batch, prob.T + 1, prob.nx) if x is None else x
    if want_u and u is None:
        u = _empty(prob, prob.batch, prob.T + 1, prob.nu)
    ws = workspace(prob, CALL_TRAJ_METHOD2) if ws is None else ws
    d, p = prob.dims(), prob.ptrs()
    _check(lib().lqt_forward_traj_method2(ctypes.byref(d), ctypes.byref(p), _ptr(elts), _ptr(S),
                                          _ptr(v), _ptr(x), _ptr(u), _ptr(ws), ws.numel(),
                                          _stream()))
    return x, u


def dense_output(prob: DeviceProblem, S, v, x, out: Optional[dict] = None, ws=None, want_u=True):
    """S, v, x, u at the n T + 1 RK4 nodes inside the blocks from the block-boundary S, v, x.
    Returns dict with S [batch][nT+1][nx][nx], v, x [batch][nT+1][nx], u [batch][nT+1][nu]."""
    nodes = prob.n * prob.T + 1
    if out is None:
        out = {"S": _empty(prob, prob.batch, nodes, prob.nx, prob.nx),
               "v": _empty(prob, prob.batch, nodes, prob.nx),
               "x": _empty(prob, prob.batch, nodes, prob.nx)}
        if want_u:
            out["u"] = _empty(prob, prob.batch, nodes, prob.nu)
    ws = workspace(prob, CALL_BUILD) if ws is None else ws
    d, p = prob.dims(), prob.ptrs()
    _check(lib().lqt_dense_output(ctypes.byref(d), ctypes.byref(p), _ptr(S), _ptr(v), _ptr(x),
                                  _ptr(out["S"]), _ptr(out["v"]), _ptr(out["x"]), _ptr(out.get("u")),
                                  _ptr(ws), ws.numel(), _stream()))
    return out


def solve_noalloc(prob: DeviceProblem, out: Optional[dict] = None):
    """lqt_solve_noalloc: the whole solve with the library's fixed scratch array instead of a
    workspace (the library allocates nothing; torch allocates the outputs here unless `out` is
    given).  Returns dict with elts, S, v, x, u."""
    if out is None:
        out = {"elts": empty_elements(prob),
               "S": _empty(prob, prob.batch, prob.T + 1, prob.nx, prob.nx),
               "v": _empty(prob, prob.batch, prob.T + 1, prob.nx),
               "x": _empty(prob, prob.batch, prob.T + 1, prob.nx),
               "u": _empty(prob, prob.batch, prob.T + 1, prob.nu)}
    d, p = prob.dims(), prob.ptrs()
    _check(lib().lqt_solve_noalloc(ctypes.byref(d), ctypes.byref(p), _ptr(out["elts"]),
                                   _ptr(out["S"]), _ptr(out["v"]), _ptr(out["x"]),
                                   _ptr(out.get("u")), _stream()))
    return out


def debug_canary(mode: int) -> None:
    """Canary-padded workspaces (lqt_debug_canary): 1 on, 2 on with canary 0 spoilt by every call
    (the check must report it), 0 off.  Workspaces must be sized after changing the mode."""
    lib().lqt_debug_canary(int(mode))


def debug_fail_launch(n: int) -> None:
    """The n-th checked HIP call from now on reports a launch failure (lqt_debug_fail_launch)."""
    lib().lqt_debug_fail_launch(int(n))


def noalloc_scratch_size(prob: DeviceProblem) -> int:
    """Bytes of the fixed scratch array lqt_solve_noalloc needs for this problem."""
    d = prob.dims()
    return int(lib().lqt_noalloc_scratch_size(ctypes.byref(d)))


NOALLOC_SCRATCH_BYTES = 64 << 20


def solve(prob: DeviceProblem, out: Optional[dict] = None, ws=None, keep_elements=False):
    """All stages in one call.  Returns dict with S, v, x, u (and elts if keep_elements)."""
    if out is None:
        out = {"S": _empty(prob, prob.batch, prob.T + 1, prob.nx, prob.nx),
               "v": _empty(prob, prob.batch, prob.T + 1, prob.nx),
               "x": _empty(prob, prob.batch, prob.T + 1, prob.nx),
               "u": _empty(prob, prob.batch, prob.T + 1, prob.nu)}
        if keep_elements:
            out["elts"] = empty_elements(prob)
    ws = workspace(prob, CALL_SOLVE) if ws is None else ws
    d, p = prob.dims(), prob.ptrs()
    _check(lib().lqt_solve(ctypes.byref(d), ctypes.byref(p), _ptr(out.get("elts")), _ptr(out["S"]),
                           _ptr(out["v"]), _ptr(out["x"]), _ptr(out.get("u")), _ptr(ws), ws.numel(),
                           _stream()))
    return out


def backward(prob: DeviceProblem, S, v, x, dLdx, ws=None, want_terminal=True):
    """Gradients of a trajectory loss (dLdx [batch][T+1][nx]) w.r.t. Q, R, r, x0, Qf, rf."""
    g = {"Q": _empty(prob, prob.batch, prob.nx, prob.nx), "R": _empty(prob, prob.batch, prob.nu, prob.nu),
         "r": _empty(prob, prob.batch, prob.nsamp, prob.nx), "x0": _empty(prob, prob.batch, prob.nx)}
    if want_terminal:
        g["Qf"] = _empty(prob, prob.batch, prob.nx, prob.nx)
        g["rf"] = _empty(prob, prob.batch, prob.nx)
    ws = workspace(prob, CALL_BACKWARD) if ws is None else ws
    d, p = prob.dims(), prob.ptrs()
    _check(lib().lqt_backward(ctypes.byref(d), ctypes.byref(p), _ptr(S), _ptr(v), _ptr(x), _ptr(dLdx),
                              _ptr(g["Q"]), _ptr(g["R"]), _ptr(g["r"]), _ptr(g["x0"]), _ptr(g.get("Qf")),
                              _ptr(g.get("rf")), _ptr(ws), ws.numel(), _stream()))
    return g


# --------------------------------------------------------------------------------------------
# Element layout helpers (structure of arrays, see include/lqt.h).
# --------------------------------------------------------------------------------------------
def element_slices(nx: int):
    ns = nx * (nx + 1) // 2
    o = 0
    out = {}
    for name, size in (("A", nx * nx), ("b", nx), ("C", ns), ("eta", nx), ("J", ns)):
        out[name] = slice(o, o + size)
        o += size
    return out


def upper_indices(nx: int):
    return np.triu_indices(nx)


# --------------------------------------------------------------------------------------------
# Autograd: x = solve(Q, R, r, x0, Qf, rf) with the hand-written adjoint as backward.
# --------------------------------------------------------------------------------------------
class SolveTrajectory(torch.autograd.Function):
    """Optimal trajectory x [batch][T+1][nx] as a differentiable function of Q, R, r, x0, Qf, rf.

    The forward pass is lqt_solve; the backward pass is lqt_backward (the exact adjoint of the
    discrete scheme), which receives dL/dx and returns symmetric gradients for Q, R, Qf.
    `template` supplies the fixed parts of the problem (grid, F, L, sizes)."""

    @staticmethod
    def forward(ctx, Q, R, r, x0, Qf, rf, template: DeviceProblem):
        prob = DeviceProblem(template.nx, template.nu, template.T, template.n, template.batch,
                             template.dtype, template.t, template.F, template.L,
                             Q.contiguous(), R.contiguous(), r.contiguous(), Qf.contiguous(),
                             rf.contiguous(), x0.contiguous(), template.c, template.F_sampled,
                             template.L_sampled, template.lti)
        out = solve(prob)
        ctx.prob = prob
        ctx.save_for_backward(out["S"], out["v"], out["x"])
        return out["x"]

    @staticmethod
    def backward(ctx, gx):
        S, v, x = ctx.saved_tensors
        g = backward(ctx.prob, S, v, x, gx.contiguous())
        return g["Q"], g["R"], g["r"], g["x0"], g["Qf"], g["rf"], None


def solve_trajectory(Q, R, r, x0, Qf, rf, template: DeviceProblem):
    return SolveTrajectory.apply(Q, R, r, x0, Qf, rf, template)


# --------------------------------------------------------------------------------------------
# Batched solve of problems with uneven horizons and sizes (lqt_ragged / lqt_plan).
# --------------------------------------------------------------------------------------------
def _class_key(p):
    return (p.nx, p.nu, p.n, np.ndim(p.F) == 3, np.ndim(p.L) == 3, getattr(p, "c", None) is not None)


class BatchedSolve:
    """Problems of any horizons and sizes, grouped into classes of equal (nx, nu, n, sampling
    flags), each class concatenated along time (layout of lqt_ragged).  `launch()` replays the
    plan (tuned configuration, one stream per class); `solve_eager()` calls lqt_solve_batched.
    Inputs can be refilled in place between launches (`classes[c]` holds the device arrays)."""

    def __init__(self, problems: Sequence, dtype=torch.float64, device="cuda", autotune=True,
                 plan=True, graph=False):
        self.dtype, self.device = dtype, device
        keys, groups = [], {}
        for i, p in enumerate(problems):
            _check_arrays(p, i, np.ndim(p.F) == 3, np.ndim(p.L) == 3, getattr(p, "c", None) is not None)
            k = _class_key(p)
            if k not in groups:
                groups[k] = []
                keys.append(k)
            groups[k].append(i)
        to = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=device)
        self.classes, self.where = [], {}
        for ci, k in enumerate(keys):
            members = [problems[i] for i in groups[k]]
            nx, nu, n, F_s, L_s, has_c = k
            Ts = np.array([p.T for p in members], dtype=np.int64)
            start = np.concatenate([[0], np.cumsum(Ts + 1)]).astype(np.int64)
            rows = int(start[-1])
            cat = lambda name: to(np.concatenate([np.asarray(getattr(p, name)) for p in members]))
            stack = lambda name: to(np.stack([np.asarray(getattr(p, name)) for p in members]))
            c = {"members": groups[k], "nx": nx, "nu": nu, "n": n, "rows": rows,
                 "F_sampled": F_s, "L_sampled": L_s,
                 "start": torch.as_tensor(start, device=device), "start_host": start,
                 "t": cat("t"), "r": cat("r"), "F": cat("F") if F_s else stack("F"),
                 "L": cat("L") if L_s else stack("L"), "c": cat("c") if has_c else None,
                 "Q": stack("Q"), "R": stack("R"), "Qf": stack("Qf"), "rf": stack("rf"),
                 "x0": stack("x0"),
                 "S": torch.empty(rows, nx, nx, dtype=dtype, device=device),
                 "v": torch.empty(rows, nx, dtype=dtype, device=device),
                 "x": torch.empty(rows, nx, dtype=dtype, device=device),
                 "u": torch.empty(rows, nu, dtype=dtype, device=device)}
            self.classes.append(c)
            for j, i in enumerate(groups[k]):
                self.where[i] = (ci, int(start[j]), int(Ts[j]))
        self._structs = (Ragged * len(self.classes))()
        for ci, c in enumerate(self.classes):
            pr = Problem(*[None if c[k] is None else c[k].data_ptr()
                           for k in ("t", "F", "L", "c", "Q", "R", "r", "Qf", "rf", "x0")])
            self._structs[ci] = Ragged(c["nx"], c["nu"], c["n"],
                                       LQT_F64 if dtype == torch.float64 else LQT_F32,
                                       len(c["members"]), int(c["F_sampled"]), int(c["L_sampled"]),
                                       int(c["c"] is not None), c["rows"], c["start"].data_ptr(), pr,
                                       c["S"].data_ptr(), c["v"].data_ptr(), c["x"].data_ptr(),
                                       c["u"].data_ptr())
        nbytes = int(lib().lqt_batched_workspace_size(self._structs, len(self.classes)))
        if nbytes == 0:
            raise LQTError(LQT_EINVAL, "invalid classes for the batched solve")
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        off = (-ws.data_ptr()) % 256
        self.ws = ws[off:off + nbytes]
        self.plan = None
        if plan:
            h = ctypes.c_void_p()
            _check(lib().lqt_plan_create(self._structs, len(self.classes), _ptr(self.ws),
                                         self.ws.numel(),
                                         (LQT_PLAN_AUTOTUNE if autotune else 0) | (LQT_PLAN_GRAPH if graph else 0),
                                         _stream(), ctypes.byref(h)))
            self.plan = h

    def launch(self):
        _check(lib().lqt_plan_launch(self.plan, _stream()))

    def solve_eager(self):
        _check(lib().lqt_solve_batched(self._structs, len(self.classes), _ptr(self.ws),
                                       self.ws.numel(), _stream()))

    def config(self) -> str:
        return lib().lqt_plan_config(self.plan).decode() if self.plan else "eager"

    def result(self, i: int) -> dict:
        """S, v, x, u of problem i (views of the class outputs, T_i + 1 rows)."""
        ci, r0, T = self.where[i]
        c = self.classes[ci]
        return {k: c[k][r0:r0 + T + 1] for k in ("S", "v", "x", "u")}

    def close(self):
        if self.plan is not None:
            lib().lqt_plan_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
