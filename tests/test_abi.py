"""The C-ABI library loads and exports every entry point include/lqt.h declares; host-side
argument validation rejects bad calls before anything is launched (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_2212_11744_amd import lqt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "lqt.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lqt_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    names = _declared_functions()
    assert len(names) >= 10
    L = lqt.lib()
    for n in names:
        assert hasattr(L, n), n


def test_element_count_and_version():
    assert lqt.element_count(4) == 44
    assert lqt.element_count(16) == 2 * 256 + 48
    assert lqt.lib().lqt_version() >= 100
    assert lqt.lib().lqt_status_string(lqt.LQT_EWORKSPACE).decode().startswith("workspace")
    assert lqt.lib().lqt_status_string(lqt.LQT_ENONFINITE).decode() == "non-finite output"


def _dims(**kw):
    base = dict(nx=4, nu=2, T=1024, n_steps=4, batch=1, dtype=lqt.LQT_F64, F_sampled=0, L_sampled=0,
                has_c=0)
    base.update(kw)
    return lqt.Dims(**base)


def test_workspace_sizes_grow_with_T_and_reject_invalid_dims():
    L = lqt.lib()
    s1 = L.lqt_workspace_size(ctypes.byref(_dims(T=1024)), lqt.CALL_SOLVE)
    s2 = L.lqt_workspace_size(ctypes.byref(_dims(T=4096)), lqt.CALL_SOLVE)
    assert 0 < s1 < s2
    assert L.lqt_workspace_size(ctypes.byref(_dims(T=1024, dtype=lqt.LQT_F32)), lqt.CALL_SOLVE) < s1
    for bad in (dict(T=0), dict(nx=0), dict(nu=5), dict(nx=17, nu=2), dict(n_steps=0), dict(batch=0),
                dict(dtype=7)):
        assert L.lqt_workspace_size(ctypes.byref(_dims(**bad)), lqt.CALL_SOLVE) == 0, bad


@pytest.mark.parametrize("bad,status", [
    (dict(T=0), lqt.LQT_EINVAL),
    (dict(nx=0), lqt.LQT_EINVAL),
    (dict(nu=3, nx=2), lqt.LQT_EINVAL),
    (dict(n_steps=0), lqt.LQT_EINVAL),
    (dict(dtype=3), lqt.LQT_EINVAL),
])
def test_invalid_dims_rejected_before_launch(bad, status):
    L = lqt.lib()
    d = _dims(**bad)
    p = lqt.Problem()
    st = L.lqt_build_elements(ctypes.byref(d), ctypes.byref(p), None, None, 0, None)
    assert st == status
    assert L.lqt_last_error()


def test_null_pointers_rejected_before_launch():
    L = lqt.lib()
    d = _dims()
    p = lqt.Problem()
    assert L.lqt_build_elements(ctypes.byref(d), ctypes.byref(p), None, None, 0, None) == lqt.LQT_EINVAL
    assert b"is NULL" in L.lqt_last_error()
    assert L.lqt_build_elements(ctypes.byref(d), None, None, None, 0, None) == lqt.LQT_EINVAL
    assert L.lqt_scan_value(ctypes.byref(d), None, None, None, None, None, None, 0, None) == lqt.LQT_EINVAL
    assert L.lqt_solve(None, None, None, None, None, None, None, None, 0, None) == lqt.LQT_EINVAL


def test_workspace_too_small_rejected_before_launch():
    L = lqt.lib()
    d = _dims()
    fake = 1 << 20  # never dereferenced: validation fails first
    st = L.lqt_scan_value(ctypes.byref(d), fake, fake, fake, fake, fake, fake, 16, None)
    assert st == lqt.LQT_EWORKSPACE
    st = L.lqt_scan_value(ctypes.byref(d), fake, fake, fake, fake, fake, fake + 8, 1 << 40, None)
    assert st == lqt.LQT_EWORKSPACE  # misaligned workspace


def _ragged(**kw):
    base = dict(nx=4, nu=2, n_steps=4, dtype=lqt.LQT_F64, count=3, F_sampled=0, L_sampled=0,
                has_c=0, rows=3 * 101)
    base.update(kw)
    r = lqt.Ragged()
    for k, v in base.items():
        setattr(r, k, v)
    return r


def test_batched_workspace_and_validation():
    L = lqt.lib()
    one = (lqt.Ragged * 1)(_ragged())
    n = L.lqt_batched_workspace_size(one, 1)
    assert n > 0 and n % 256 == 0
    big = (lqt.Ragged * 1)(_ragged(rows=3 * 10001))
    assert L.lqt_batched_workspace_size(big, 1) > n
    two = (lqt.Ragged * 2)(_ragged(), _ragged(nx=8, nu=4))
    assert L.lqt_batched_workspace_size(two, 2) > n
    for bad in (dict(rows=5), dict(count=0), dict(nx=17), dict(nu=5), dict(dtype=7),
                dict(rows=2 ** 31)):
        b = (lqt.Ragged * 1)(_ragged(**bad))
        assert L.lqt_batched_workspace_size(b, 1) == 0, bad
        assert L.lqt_solve_batched(b, 1, None, 0, None) == lqt.LQT_EINVAL, bad
    # Null arrays are rejected before anything is launched.
    assert L.lqt_solve_batched(one, 1, None, 0, None) == lqt.LQT_EINVAL
    assert b"is NULL" in L.lqt_last_error()
    assert L.lqt_solve_batched(None, 0, None, 0, None) == lqt.LQT_EINVAL
    h = ctypes.c_void_p()
    assert L.lqt_plan_create(one, 1, None, 0, 1, None, ctypes.byref(h)) == lqt.LQT_EINVAL
    assert not h.value
    assert L.lqt_plan_create(one, 1, None, 0, 1, None, None) == lqt.LQT_EINVAL
    assert L.lqt_plan_launch(None, None) == lqt.LQT_EINVAL
    assert L.lqt_plan_config(None) == b""
    L.lqt_plan_destroy(None)


def test_lti_flag_validation_and_workspace():
    L = lqt.lib()
    plain = L.lqt_workspace_size(ctypes.byref(_dims()), lqt.CALL_SOLVE)
    lti = L.lqt_workspace_size(ctypes.byref(_dims(lti=1)), lqt.CALL_SOLVE)
    assert lti > plain  # the response tables
    assert L.lqt_workspace_size(ctypes.byref(_dims(lti=1)), lqt.CALL_SCAN_VALUE) == \
        L.lqt_workspace_size(ctypes.byref(_dims()), lqt.CALL_SCAN_VALUE)
    for bad in (dict(F_sampled=1), dict(L_sampled=1), dict(has_c=1)):
        d = _dims(lti=1, **bad)
        assert L.lqt_workspace_size(ctypes.byref(d), lqt.CALL_SOLVE) == 0
        p = lqt.Problem()
        assert L.lqt_build_elements(ctypes.byref(d), ctypes.byref(p), None, None, 0, None) == lqt.LQT_EINVAL
        assert b"lti" in L.lqt_last_error()


def test_host_checks_of_problem_arrays():
    """Array shapes and the grid are checked on the host before anything reaches the device (the
    kernels index the arrays by the dims alone)."""
    import numpy as np
    from paper_2212_11744_amd import workloads as W
    p = W.point_mass(1, 16, 2)
    bad_r = W.point_mass(1, 16, 2)
    bad_r.r = bad_r.r[:-1]
    with pytest.raises(ValueError, match="r has shape"):
        lqt.DeviceProblem.from_problems([p, bad_r], device="cpu")
    bad_t = W.point_mass(1, 16, 2)
    bad_t.t = bad_t.t.copy()
    bad_t.t[5] = bad_t.t[4]
    with pytest.raises(ValueError, match="strictly increasing"):
        lqt.DeviceProblem.from_problems([bad_t], device="cpu")
    bad_q = W.point_mass(1, 16, 2)
    bad_q.Q = np.eye(3)
    with pytest.raises(ValueError, match="Q has shape"):
        lqt.DeviceProblem.from_problems([bad_q], device="cpu")


def test_host_checks_of_batched_members():
    from paper_2212_11744_amd import workloads as W
    good = W.point_mass(1, 16, 2)
    bad = W.point_mass(2, 20, 2)
    bad.r = bad.r[:-3]
    with pytest.raises(ValueError, match="problem 1: r has shape"):
        lqt.BatchedSolve([good, bad], device="cpu", plan=False)
