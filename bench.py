"""Benchmark: full parallel-in-time LQT solve (elements + value scan + trajectory scan) on one GPU.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--T 1048576] [--dtype f64|f32]

Workload: the point-mass tracking problem (nx = 4, nu = 2) on [0, 10] with T = 2^20 blocks of
4 RK4 steps each, FP64, seeded synthetic reference (sum of sinusoids), inputs resident in HBM.
A step is one call of lqt_solve: per-block elements, the value scan (S_k, v_k) and the
trajectory scan (x_k, u_k) at all T + 1 block boundaries.  Prints one JSON line.

The dominant kernel (the element build, bound by FP64 vector arithmetic) is timed on its own with
HIP events on the stream it is launched on; its algorithmic flop count is the FMA count of the
kernel's formulation (see build_flops_per_block), the same figure the design notes derive.
The CPU baseline is the oracle (single-threaded, unmodified) on a bounded sample of the same
workload: the first M blocks of the grid (same block length and reference) solved as a horizon
of their own.

Also reported (not the headline): the differentiated workload (64 point-mass problems, T = 2^16,
FP64: one batched lqt_solve plus one lqt_backward of a tracking loss, "fwd+bwd ms") and the
random time-varying nx = 16 workload (T = 2^14, F(t) sampled).  `--copy-probe MIB` adds a plain
device copy of that size after the timed work, so that a counter run (rocprofv3 --pmc FETCH_SIZE
/ WRITE_SIZE) can scale the element build's counter readings by those of a copy of known size.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK = {"hbm_GBps": 8000.0, "f64_TFLOPs": 78.6, "f32_TFLOPs": 157.3}


def build_flops_per_block(nx: int, nu: int, n: int, has_c: bool = False) -> int:
    """FP64/FP32 flops (FMA = 2) of one block of the element build as the kernel computes it.

    Per RK4 stage: K = G J - F (nx^3), G eta (nx^2), b increment (nx^2 + nx), A Lc (nx^2 nu),
    C increment (ns nu + ns), eta derivative (2 nx^2, + nx^2 with a drift c), J derivative
    (nx^2 (nx + 1)), A-row derivative (nx^3) and the RK4 accumulations (2 nx^2 + 2 nx + 2 ns,
    minus the stage-input updates in the last stage).  ns = nx (nx + 1) / 2.
    """
    ns = nx * (nx + 1) // 2
    per_stage = (nx ** 3 + nx ** 2 + nx ** 2 + nx + nx * nx * nu + ns * nu + ns + 2 * nx ** 2
                 + (nx ** 2 if has_c else 0) + nx ** 2 * (nx + 1) + nx ** 3
                 + 2 * nx ** 2 + 2 * nx + 2 * ns)
    last_stage = per_stage - (nx ** 2 + nx + ns)
    return 2 * n * (3 * per_stage + last_stage)


# Dense-generic flop estimate of one block of the element build (nx = 4, nu = 2, n = 4): the
# theorem's right-hand sides evaluated as written, FMA = 2 (the survey's per-sub-interval figure).
DENSE_GENERIC_BUILD_FLOPS = 19000
# Algorithmic HBM bytes per block of the two scan stages at nx = 4, nu = 2 in FP64 (halved in FP32):
# value scan 352 (element) + 128 (S, full) + 32 (v) = 512; trajectory 240 (A, b, C of the element)
# + 160 (S, v) + 32 (x) + 16 (u) = 448.
SCAN_VALUE_BYTES, FORWARD_TRAJ_BYTES = 512, 448


def _hbm_frac(nbytes: int, ms: float) -> dict:
    gbps = nbytes / (ms * 1e-3) / 1e9
    return {"bytes": nbytes, "ms": ms, "achieved_GBps": gbps, "peak_GBps": PEAK["hbm_GBps"],
            "frac": gbps / PEAK["hbm_GBps"]}


def build_bytes_per_block(nx: int, n: int, es: int) -> int:
    """HBM bytes per block of the element build: 2n new reference samples read, one element
    (2 nx^2 + 3 nx values) written."""
    return es * (2 * n * nx + 2 * nx * nx + 3 * nx)


def _events_time(fn, reps, torch, warm=True):
    # One untimed call first (warm=True): the first launch from a code object that has not run
    # yet in this process loads it, a one-time cost of tens of ms that is not the call's own.
    if warm:
        fn()
        torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(s)
    for _ in range(reps):
        fn()
    b.record(s)
    b.synchronize()
    return a.elapsed_time(b) / reps  # ms


def cpu_baseline(T: int, target_s: float):
    """The oracle on the first M blocks of the workload grid (M sized for ~target_s seconds)."""
    import oracle as O
    from paper_2212_11744_amd import workloads as W

    def run(M):
        p = W.point_mass(2, M, 4, 0.0, 10.0 * M / T)
        t0 = time.perf_counter()
        O.solve(p)
        return time.perf_counter() - t0

    M = 2048
    dt = run(M)
    M = int(min(T, max(2048, M * target_s / max(dt, 1e-3))))
    dt = run(M)
    return {"value": M / dt, "unit": "sub-intervals/s", "cores": 1, "kind": "oracle",
            "sample": f"first {M} of the {T} blocks (same block length, reference and weights) "
                      f"solved as their own horizon by the sequential FP64 oracle: elements, value "
                      f"fold and trajectory; {dt:.1f} s on one host thread"}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--T", type=int, default=2 ** 20)
    ap.add_argument("--dtype", choices=["f64", "f32"], default="f64")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "k_build_point_mass_T2p20_traffic.txt"))
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-nx16", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-lti", action="store_true")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: the library has no multi-GPU path (asked for "
              f"--gpus {args.gpus}); the design notes describe how the solve would shard.",
              file=sys.stderr)
        return 2

    import torch
    from paper_2212_11744_amd import lqt
    from paper_2212_11744_amd import workloads as W

    dtype = torch.float64 if args.dtype == "f64" else torch.float32
    es = 8 if args.dtype == "f64" else 4
    T, n = args.T, 4
    p = W.point_mass(2, T, n)
    dp = lqt.DeviceProblem.from_problems([p], dtype=dtype)
    out = {"S": torch.empty(1, T + 1, 4, 4, dtype=dtype, device="cuda"),
           "v": torch.empty(1, T + 1, 4, dtype=dtype, device="cuda"),
           "x": torch.empty(1, T + 1, 4, dtype=dtype, device="cuda"),
           "u": torch.empty(1, T + 1, 2, dtype=dtype, device="cuda"),
           "elts": None}
    out["elts"] = lqt.empty_elements(dp)
    ws = lqt.workspace(dp, lqt.CALL_SOLVE)
    ws_b = lqt.workspace(dp, lqt.CALL_BUILD)
    step = lambda: lqt.solve(dp, out, ws)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ms = _events_time(step, args.steps, torch, warm=False)  # after the W warmup steps above
    torch.cuda.synchronize()

    # Dominant kernel on its own: lqt_build_elements = per-problem constants (one tiny launch) +
    # the element build.
    build = lambda: lqt.build_elements(dp, out["elts"], ws_b)
    build()
    ms_build = _events_time(build, args.steps, torch)
    flops = build_flops_per_block(4, 2, n) * T
    achieved = flops / (ms_build * 1e-3) / 1e12
    peak = PEAK["f64_TFLOPs" if es == 8 else "f32_TFLOPs"]
    traffic = _traffic(args.traffic, T, args.dtype)
    # Stage breakdown (each stage call timed on its own).
    S, v = out["S"], out["v"]
    ws_v = lqt.workspace(dp, lqt.CALL_SCAN_VALUE)
    ws_t = lqt.workspace(dp, lqt.CALL_FORWARD_TRAJ)
    ms_scan = _events_time(lambda: lqt.scan_value(dp, out["elts"], S, v, ws_v), max(3, args.steps // 2), torch)
    ms_traj = _events_time(lambda: lqt.forward_traj(dp, out["elts"], S, v, out["x"], out["u"], ws_t),
                           max(3, args.steps // 2), torch)
    # Method 2 trajectory (forward prefix scan) from the same elements and values.
    ws_m2 = lqt.workspace(dp, lqt.CALL_TRAJ_METHOD2)
    ms_m2 = _events_time(lambda: lqt.forward_traj_method2(dp, out["elts"], S, v, out["x"], out["u"], ws_m2),
                         max(3, args.steps // 2), torch)
    # Elements from the forward conditional ODEs (Theorem 9) on the same problem.
    ms_fwd = _events_time(lambda: lqt.build_elements_forward(dp, out["elts"], ws_b),
                          max(3, args.steps // 2), torch)
    # Elements with every block split (Theorem 9 on the first half, Theorem 8 on the second).
    ms_split = _events_time(lambda: lqt.build_elements_split(dp, out["elts"], ws_b),
                            max(3, args.steps // 2), torch)
    # Values inside the blocks: S, v, x, u at the n T + 1 RK4 nodes from the boundary values.
    nodes = n * T + 1
    dense = {"S": torch.empty(1, nodes, 4, 4, dtype=dtype, device="cuda"),
             "v": torch.empty(1, nodes, 4, dtype=dtype, device="cuda"),
             "x": torch.empty(1, nodes, 4, dtype=dtype, device="cuda"),
             "u": torch.empty(1, nodes, 2, dtype=dtype, device="cuda")}
    ms_dense = _events_time(lambda: lqt.dense_output(dp, S, v, out["x"], dense, ws_b),
                            max(3, args.steps // 2), torch)
    del dense

    rec = {
        "metric": "sub-intervals/s for full LQT solve (value+trajectory) at nx=4",
        "value": T / (ms * 1e-3),
        "unit": "sub-intervals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": f"point-mass LQT tracking, nx=4 nu=2, T={T} blocks x {n} RK4 steps on [0,10], "
                               f"single problem, elements + value scan + trajectory scan",
                   "T": T, "nx": 4, "nu": 2, "n_steps": n, "batch": 1, "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "kernel": "k_build (element build)", "achieved": achieved,
                     "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak, "traffic": traffic,
                     "flops_per_launch": flops, "launch_ms": ms_build,
                     "flops_per_block": build_flops_per_block(4, 2, n),
                     "flops_per_block_counting": "the kernel's own formulation (K = G J - F factored "
                                                 "out, packed symmetric products); frac uses it",
                     "flops_per_block_executed_counters": 12540,
                     "flops_per_block_dense_generic": DENSE_GENERIC_BUILD_FLOPS,
                     "frac_dense_generic": DENSE_GENERIC_BUILD_FLOPS * T / (ms_build * 1e-3) / 1e12 / peak,
                     "algorithmic_bytes_per_launch": build_bytes_per_block(4, n, es) * T},
        # The two scans are bound by HBM: achieved algorithmic bytes (value scan: element read +
        # S (full) and v written; trajectory: element map part + S, v read, x, u written) over
        # each stage call's time, against 8 TB/s.
        "scan_hbm": {
            "value": _hbm_frac(SCAN_VALUE_BYTES * es // 8 * T, ms_scan),
            "trajectory": _hbm_frac(FORWARD_TRAJ_BYTES * es // 8 * T, ms_traj),
        },
        "stages_ms": {"build_elements": ms_build, "scan_value": ms_scan, "forward_traj": ms_traj,
                      "build_elements_forward": ms_fwd, "forward_traj_method2": ms_m2,
                      "build_elements_split": ms_split, "dense_output": ms_dense},
    }
    rec["small"] = small_leg(torch, lqt, W, dtype)
    rec["t2p16"] = t2p16_leg(torch, lqt, W, dtype)
    if not args.no_lti:
        rec["lti"] = lti_leg(torch, lqt, p, dtype, args.steps, out, T)
    if not args.no_adjoint:
        rec["adjoint"] = adjoint_leg(torch, lqt, W, max(3, args.steps // 4))
    if not args.no_nx16:
        rec["nx16"] = nx16_leg(torch, lqt, W, max(3, args.steps // 4))
    if not args.no_batched:
        rec["batched"] = batched_leg(torch, lqt, W, max(3, args.steps // 4))
    if args.copy_probe:
        a = torch.empty(args.copy_probe * 2 ** 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        rec["copy_probe_bytes"] = a.numel()
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(T, args.cpu_seconds)
    print(json.dumps(rec), flush=True)
    return 0


def lti_leg(torch, lqt, p, dtype, reps, out, T):
    """The same workload through the time-invariant path (lqt_dims.lti): shared A, C, J per
    problem and each block's b, eta as weighted sums of its samples; same outputs up to rounding."""
    dp = lqt.DeviceProblem.from_problems([p], dtype=dtype, lti=True)
    ws = lqt.workspace(dp, lqt.CALL_SOLVE)
    ws_b = lqt.workspace(dp, lqt.CALL_BUILD)
    lqt.solve(dp, out, ws)
    torch.cuda.synchronize()
    ms = _events_time(lambda: lqt.solve(dp, out, ws), reps, torch)
    ms_b = _events_time(lambda: lqt.build_elements(dp, out["elts"], ws_b), reps, torch)
    return {"workload": "same problem, time-invariant path (F, L constant, c = 0, uniform grid)",
            "ms_per_step": ms, "sub_intervals_per_s": T / (ms * 1e-3), "build_ms": ms_b}


def t2p16_leg(torch, lqt, W, dtype):
    """The same point-mass generator at T = 2^16 blocks x 4 RK4 steps (the smaller size of the
    benchmark configuration): solve time and throughput."""
    T = 2 ** 16
    p = W.point_mass(2, T, 4)
    dp = lqt.DeviceProblem.from_problems([p], dtype=dtype)
    out = lqt.solve(dp, keep_elements=True)
    ws = lqt.workspace(dp, lqt.CALL_SOLVE)
    solve = lambda: lqt.solve(dp, out, ws)
    solve()
    torch.cuda.synchronize()
    ms = _events_time(solve, 50, torch)
    return {"workload": "point-mass LQT tracking, T=65536 blocks x 4 RK4 steps on [0,10]",
            "ms_per_step": ms, "sub_intervals_per_s": T / (ms * 1e-3)}


def small_leg(torch, lqt, W, dtype):
    """Point mass with T = 64 blocks x 10 RK4 steps (the small case): solve latency, and the element
    build with whole blocks (Theorem 8) vs split blocks (two wavefronts per block)."""
    p = W.point_mass(1, 64, 10)
    dp = lqt.DeviceProblem.from_problems([p], dtype=dtype)
    out = lqt.solve(dp, keep_elements=True)
    ws, ws_b = lqt.workspace(dp, lqt.CALL_SOLVE), lqt.workspace(dp, lqt.CALL_BUILD)
    solve = lambda: lqt.solve(dp, out, ws)
    build = lambda: lqt.build_elements(dp, out["elts"], ws_b)
    split = lambda: lqt.build_elements_split(dp, out["elts"], ws_b)
    for f in (solve, build, split):
        f()
    torch.cuda.synchronize()
    return {"workload": "point-mass LQT tracking, T=64 blocks x 10 RK4 steps on [0,10]",
            "solve_ms": _events_time(solve, 200, torch), "build_ms": _events_time(build, 200, torch),
            "build_split_ms": _events_time(split, 200, torch)}


# Executed FP64 flops per block of the adjoint's RK4 kernel (k_adj_rk4, nx = 4, nu = 2, n = 4
# steps): (2 FMA + MUL + ADD + TRANS) F64 instructions per wave x 64 lanes, one block per lane,
# from the SQ counters of profiles/sq_counters_main_kernels.txt.  The same counters give 12540
# for the element build, whose own formulation counts 12496.
ADJ_RK4_FLOPS_PER_BLOCK = 44682


def adjoint_leg(torch, lqt, W, reps):
    """64 point-mass problems (seeds 5000 + i), T = 2^16, FP64: batched solve + adjoint of the
    loss sum_k |x_k - g(t_k)|^2 (gradients for Q, R, r, x0, Qf, rf)."""
    B, T, n = 64, 2 ** 16, 4
    probs = [W.point_mass(5000 + i, T, n) for i in range(B)]
    dp = lqt.DeviceProblem.from_problems(probs)
    g = torch.as_tensor(np.stack([W.tracking_targets(5, p.t) for p in probs]), device="cuda")
    ws_f, ws_b = lqt.workspace(dp, lqt.CALL_SOLVE), lqt.workspace(dp, lqt.CALL_BACKWARD)
    out = lqt.solve(dp, ws=ws_f)
    fwd = lambda: lqt.solve(dp, out, ws_f)
    bwd = lambda: lqt.backward(dp, out["S"], out["v"], out["x"], 2.0 * (out["x"] - g), ws=ws_b)
    fwd(), bwd()
    torch.cuda.synchronize()
    ms_f = _events_time(fwd, reps, torch)
    ms_b = _events_time(bwd, reps, torch)
    # The RK4 adjoint of the elements is the backward pass's dominant kernel; its flops over the
    # whole backward time bound its own fraction of the FP64 peak from below.
    rk4_tf = ADJ_RK4_FLOPS_PER_BLOCK * B * T / (ms_b * 1e-3) / 1e12
    return {"workload": f"{B} point-mass problems, T={T} blocks x {n} RK4 steps, FP64, tracking loss",
            "fwd_ms": ms_f, "bwd_ms": ms_b, "fwd_bwd_ms": ms_f + ms_b,
            "sub_intervals_per_s_fwd_bwd": B * T / ((ms_f + ms_b) * 1e-3),
            "rk4_adjoint": {"kernel": "k_adj_rk4", "flops_per_block": ADJ_RK4_FLOPS_PER_BLOCK,
                            "flops_per_block_counting": "executed FP64 instructions (SQ counters)",
                            "TFLOPs_over_bwd_ms": rk4_tf,
                            "frac_lower_bound": rk4_tf / PEAK["f64_TFLOPs"]}}


def nx16_leg(torch, lqt, W, reps):
    """Random stable time-varying LQT, nx = 16, nu = 4, T = 2^14, F(t) sampled, FP64."""
    T = 2 ** 14
    p = W.random_stable(3, nx=16, nu=4, T=T, n=4)
    dp = lqt.DeviceProblem.from_problems([p])
    ws = lqt.workspace(dp, lqt.CALL_SOLVE)
    out = lqt.solve(dp, ws=ws)
    torch.cuda.synchronize()
    ms = _events_time(lambda: lqt.solve(dp, out, ws), reps, torch)
    wsb = lqt.workspace(dp, lqt.CALL_BUILD)
    e = lqt.build_elements(dp, ws=wsb)
    builds = {}
    for name, f in (("theorem8", lqt.build_elements), ("theorem9", lqt.build_elements_forward),
                    ("split", lqt.build_elements_split)):
        f(dp, e, wsb)
        torch.cuda.synchronize()
        builds[name] = _events_time(lambda f=f: f(dp, e, wsb), reps, torch)
    e = lqt.build_elements(dp, e, wsb)
    ws2 = lqt.workspace(dp, lqt.CALL_TRAJ_METHOD2)
    x2, u2 = lqt.forward_traj_method2(dp, e, out["S"], out["v"], ws=ws2)
    m2 = lambda: lqt.forward_traj_method2(dp, e, out["S"], out["v"], x2, u2, ws=ws2)
    torch.cuda.synchronize()
    ms_m2 = _events_time(m2, reps, torch)
    d = lqt.dense_output(dp, out["S"], out["v"], out["x"], ws=wsb)
    dense = lambda: lqt.dense_output(dp, out["S"], out["v"], out["x"], out=d, ws=wsb)
    torch.cuda.synchronize()
    ms_dense = _events_time(dense, reps, torch)
    # time-invariant variant (F = F0 constant): general build vs the tabulated one
    pti = W.random_stable(3, nx=16, nu=4, T=T, n=4, time_varying=False)
    lti_ms = {}
    for name, flag in (("general", False), ("lti", True)):
        dpt = lqt.DeviceProblem.from_problems([pti], lti=flag)
        wst = lqt.workspace(dpt, lqt.CALL_BUILD)
        et = lqt.build_elements(dpt, ws=wst)
        torch.cuda.synchronize()
        lti_ms[name] = _events_time(lambda: lqt.build_elements(dpt, et, wst), reps, torch)
    return {"workload": f"random stable time-varying LQT nx=16 nu=4, T={T} x 4 RK4 steps, FP64",
            "ms": ms, "sub_intervals_per_s": T / (ms * 1e-3), "build_ms": builds,
            "method2_ms": ms_m2, "dense_output_ms": ms_dense,
            "time_invariant_build_ms": lti_ms}


def batched_leg(torch, lqt, W, reps):
    """1024 problems (nx in {2, 4, 8}, nu = nx / 2, T_i ~ U{256..8192}, FP64): the tuned plan
    captured into a HIP graph and replayed (one hipGraphLaunch), and the same plan launched
    eagerly, vs 1024 separate lqt_solve calls on one stream (all inputs and outputs resident)."""
    probs = W.batched_mix()
    bs = lqt.BatchedSolve(probs, autotune=True, graph=True)
    torch.cuda.synchronize()
    ms_plan = _events_time(bs.launch, reps, torch)
    eager_plan = lqt.BatchedSolve(probs, autotune=True)
    torch.cuda.synchronize()
    ms_eager = _events_time(eager_plan.launch, reps, torch)
    eager_plan.close()
    singles = []
    for p in probs:
        dp = lqt.DeviceProblem.from_problems([p])
        singles.append((dp, lqt.solve(dp), lqt.workspace(dp, lqt.CALL_SOLVE)))
    torch.cuda.synchronize()

    def separate():
        for dp, out, ws in singles:
            lqt.solve(dp, out, ws)

    ms_sep = _events_time(separate, max(2, reps // 2), torch)
    blocks = sum(p.T for p in probs)
    return {"workload": f"{len(probs)} problems, nx in (2, 4, 8), nu = nx/2, T_i ~ U{{256..8192}} "
                        f"(sum {blocks} blocks) x 4 RK4 steps, FP64",
            "plan_ms": ms_plan, "plan_eager_ms": ms_eager, "separate_solves_ms": ms_sep,
            "speedup": ms_sep / ms_plan,
            "sub_intervals_per_s": blocks / (ms_plan * 1e-3), "plan_config": bs.config()}


def _traffic(path, T, dtype):
    """HBM bytes per launch of the element build from a committed counter summary (key: value
    lines), or None when it was taken for another workload or an older kernel source."""
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("T") != str(T) or kv.get("dtype") != dtype or kv.get("kernel_source_sha") != _kernel_sha():
        return None
    return float(kv["hbm_bytes_per_launch"])


def _kernel_sha() -> str:
    """sha256 (first 16 hex digits) of the code of lane_math.hpp + lqt_lane.hip: every line with
    its // comment removed and surrounding blanks stripped, blank lines dropped, so edits to
    comments alone keep a counter summary valid."""
    import hashlib
    h = hashlib.sha256()
    for f in ("lane_math.hpp", "lqt_lane.hip"):
        with open(os.path.join(ROOT, "paper_2212_11744_amd", "csrc", f)) as fh:
            for line in fh:
                code = line.split("//", 1)[0].strip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


if __name__ == "__main__":
    sys.exit(main())
