"""Build the gfx950 HIP library `liblqt.so` in-tree with hipcc (no GPU needed to compile).

    python -m paper_2212_11744_amd.build [--verbose]

Each translation unit under csrc/ is compiled in parallel, then linked into one shared library
next to this file.  `--verbose` adds the compiler's per-kernel resource report (VGPRs, SGPRs,
scratch, occupancy).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "liblqt.so")
OBJ_DIR = os.path.join(HERE, "_build")

SOURCES = ["lqt_api.hip", "lqt_prep.hip", "lqt_lane.hip", "lqt_adjoint.hip", "lqt_wave.hip",
           "lqt_batched.hip"]
# Sources compiled once per build shard (-DLQT_SHARD=i): each object holds a share of the
# template instantiations, so the shards compile in parallel.  Must match kLaneShards and
# kWaveShards in csrc/lqt_internal.hpp (a mismatch fails at link time).
SHARDS = {"lqt_lane.hip": 4, "lqt_wave.hip": 8}


def units() -> list:
    """(source, shard or None, object path) of every object of the library."""
    out = []
    for src in SOURCES:
        stem = os.path.splitext(src)[0]
        n = SHARDS.get(src)
        if n is None:
            out.append((src, None, os.path.join(OBJ_DIR, stem + ".o")))
        else:
            out.extend((src, i, os.path.join(OBJ_DIR, f"{stem}.{i}.o")) for i in range(n))
    return out

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-I", INCLUDE,
    # Keep the compiler from forming packed FP32 instructions.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def _compile(unit: tuple, verbose: bool) -> str:
    src, shard, obj = unit
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    if shard is not None:
        cmd.append(f"-DLQT_SHARD={shard}")
    if verbose:
        cmd.append("-Rpass-analysis=kernel-resource-usage")
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    if verbose:
        sys.stderr.write(r.stderr)
    return obj


def build(verbose: bool = False) -> str:
    """Compile every HIP translation unit for gfx950 and link liblqt.so; returns its path."""
    os.makedirs(OBJ_DIR, exist_ok=True)
    todo = units()
    # Longest compiles first, so the pool's tail is short.
    todo.sort(key=lambda u: (u[1] is None, u[0] != "lqt_wave.hip"))
    with cf.ThreadPoolExecutor(max_workers=min(len(todo), os.cpu_count() or 1, 16)) as ex:
        list(ex.map(lambda u: _compile(u, verbose), todo))
    objs = [u[2] for u in units()]
    tmp = LIB + ".tmp"
    r = subprocess.run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


def clean() -> None:
    shutil.rmtree(OBJ_DIR, ignore_errors=True)


if __name__ == "__main__":
    print(build(verbose="--verbose" in sys.argv))
