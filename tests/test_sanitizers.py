"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The oracle (oracle/lqt_oracle.cpp) built by g++ with -fsanitize=address,undefined runs the
  oracle's pins (tests/test_oracle_pins.py) in a child Python with gcc's ASan runtime preloaded.
* The host code of the C-ABI library (argument validation, workspace layout, batched plans: the
  lqt_api, lqt_batched, lqt_prep and lqt_adjoint translation units, sanitized on the host side
  only) linked with the ordinary kernel objects runs tests/test_abi.py in a child Python with
  clang's ASan runtime preloaded.  No kernel is launched (no GPU is needed).
Any sanitizer report aborts the child, which fails the test.  The sanitized objects are cached
under paper_2212_11744_amd/_build/sanitize and rebuilt when a source is newer.
"""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2212_11744_amd", "csrc")
BUILD = os.path.join(ROOT, "paper_2212_11744_amd", "_build")
OUT = os.path.join(BUILD, "sanitize")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HOST_UNITS = ("lqt_api", "lqt_batched", "lqt_prep", "lqt_adjoint")
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _newer(target, deps):
    return os.path.exists(target) and all(os.path.getmtime(target) >= os.path.getmtime(d)
                                          for d in deps)


def _child(env_extra, args):
    env = dict(os.environ, **SAN_ENV, **env_extra)
    r = subprocess.run([sys.executable, *args], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=900)
    out = r.stdout[-4000:] + r.stderr[-4000:]
    assert r.returncode == 0, out
    assert "AddressSanitizer" not in r.stderr and "runtime error:" not in r.stderr, out
    return r.stdout


CHECK = ("import ctypes, os, sys; sys.path.insert(0, '.'); "
         "assert hasattr(ctypes.CDLL(None), '__asan_init'); "
         "import {mod}; {mod}.lib(); "
         "maps = open('/proc/self/maps').read(); assert os.environ['{var}'] in maps; print('ok')")


def test_oracle_under_asan_ubsan():
    os.makedirs(OUT, exist_ok=True)
    src = os.path.join(ROOT, "oracle", "lqt_oracle.cpp")
    so = os.path.join(OUT, "liblqt_oracle_san.so")
    if not _newer(so, [src]):
        subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-shared", "-fPIC",
                        "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                        "-fno-omit-frame-pointer", "-o", so, src], check=True)
    asan = subprocess.run(["g++", "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    env = {"LD_PRELOAD": asan, "LQT_ORACLE_LIB": so}
    assert "ok" in _child(env, ["-c", CHECK.format(mod="oracle", var="LQT_ORACLE_LIB")])
    _child(env, ["-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "tests/test_oracle_pins.py"])


def test_library_host_code_under_asan_ubsan():
    kernels = sorted(glob.glob(os.path.join(BUILD, "lqt_lane.*.o")) +
                     glob.glob(os.path.join(BUILD, "lqt_wave.*.o")))
    if len(kernels) < 12:
        pytest.skip("kernel objects not built (python -m paper_2212_11744_amd.build)")
    rt = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not rt:
        pytest.skip("clang's ASan runtime not found")
    os.makedirs(OUT, exist_ok=True)
    headers = glob.glob(os.path.join(CSRC, "*.hpp")) + [os.path.join(ROOT, "include", "lqt.h")]
    procs, objs = [], []
    for u in HOST_UNITS:
        src, obj = os.path.join(CSRC, u + ".hip"), os.path.join(OUT, u + ".o")
        objs.append(obj)
        if _newer(obj, [src, *headers]):
            continue
        # sanitizers on the host side only (each -fsanitize behind -Xarch_host)
        procs.append(subprocess.Popen(
            [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
             "-I", os.path.join(ROOT, "include"),
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
             "-Wno-unused-command-line-argument", "-c", src, "-o", obj],
            stdout=subprocess.PIPE, stderr=subprocess.PIPE))
    for p in procs:
        _, err = p.communicate()
        assert p.returncode == 0, err.decode()[-3000:]
    so = os.path.join(OUT, "liblqt_san.so")
    if not _newer(so, objs + kernels):
        subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, *kernels,
                        "-o", so], check=True)
    env = {"LD_PRELOAD": rt[-1], "LQT_LIBRARY": so}
    assert "ok" in _child(env, ["-c", CHECK.format(mod="paper_2212_11744_amd.lqt", var="LQT_LIBRARY")])
    _child(env, ["-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "tests/test_abi.py"])
