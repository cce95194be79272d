"""Test infrastructure only: the sequential FP64 CPU oracle of the parallel-in-time LQT solver.

Only `tests/`, `__graft_entry__.smoke()` and the CPU-baseline leg of `bench.py` may import this
package.  It wraps `liblqt_oracle.so` (built from `lqt_oracle.cpp` with g++) through ctypes and
shares no code with the GPU library.
"""
from .oracle import *  # noqa: F401,F403
