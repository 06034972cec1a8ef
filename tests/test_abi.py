"""CPU checks of the C ABI: the library loads, exports every declared entry point, and
rejects invalid problems on the host before touching the GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2510_04094_amd import nyls

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "nyls.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nyls_[a-z_]+)\s*\(", text)))


def test_header_declares_the_five_work_functions():
    names = declared_functions()
    for fn in ["nyls_features", "nyls_assemble", "nyls_solve", "nyls_newton_step", "nyls_backward"]:
        assert fn in names


def test_library_exports_every_declared_symbol():
    lib = nyls.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) == set(nyls.EXPORTS)


def problem(**kw):
    pr = nyls.Problem()
    pr.p, pr.n, pr.m, pr.uniform = 1, 100, 10, 1
    pr.t0, pr.dt = 0.0, 0.01
    pr.f = 8
    pr.r = 8
    pr.v = 8          # never dereferenced: validation fails or the test stops first
    pr.cond_d[0], pr.cond_i[0] = 0, 0
    pr.sigma, pr.gamma, pr.tau = 0.1, 1e6, 1e-12
    for k, v in kw.items():
        if k in ("cond_d", "cond_i"):
            for j, x in enumerate(v):
                getattr(pr, k)[j] = x
        else:
            setattr(pr, k, v)
    return pr


def create(pr, batch=1, mode=0):
    lib = nyls.load()
    arr = (nyls.Problem * batch)(*([pr] * batch))
    h = ctypes.c_void_p()
    rc = lib.nyls_plan_create(ctypes.cast(arr, ctypes.c_void_p), batch, mode, ctypes.byref(h))
    if rc == 0:
        lib.nyls_plan_destroy(h)
    return rc


@pytest.mark.parametrize("kw,code", [
    (dict(p=0), -4), (dict(p=5), -4),
    (dict(n=1), -5), (dict(m=1), -5), (dict(m=101), -5), (dict(n=300, m=257), -5),
    (dict(sigma=0.0), -6), (dict(gamma=-1.0), -6), (dict(tau=1.0), -6), (dict(sigma=float("nan")), -6),
    (dict(dt=0.0), -7), (dict(uniform=0), -7),
    (dict(v=None), -1),
    (dict(cond_d=[1]), -9), (dict(cond_i=[100]), -9), (dict(cond_i=[-1]), -9),
    (dict(p=2, cond_d=[0, 0], cond_i=[0, 0]), -9),
])
def test_invalid_problems_are_rejected_on_the_host(kw, code):
    assert create(problem(**kw)) == code


def test_wide_bases_only_in_fp64_mode():
    """Bases above 128 landmarks are taken by NYLS_FP64 plans only (mixed mode stops at 126)."""
    assert create(problem(n=300, m=127), mode=1) == -5
    assert create(problem(n=300, m=129), mode=1) == -5
    assert create(problem(n=300, m=129), mode=2) == -5


def test_invalid_landmarks_are_rejected():
    lib = nyls.load()
    for bad in ([0, 5, 5, 9, 10, 20, 30, 40, 50, 99], [0, 1, 2, 3, 4, 5, 6, 7, 8, 100]):
        arr = (ctypes.c_int32 * 10)(*bad)
        pr = problem()
        pr.lidx = ctypes.cast(arr, ctypes.c_void_p)
        assert create(pr) == -8


def test_bad_batch_and_mode():
    lib = nyls.load()
    pr = problem()
    arr = (nyls.Problem * 1)(pr)
    h = ctypes.c_void_p()
    assert lib.nyls_plan_create(ctypes.cast(arr, ctypes.c_void_p), 0, 0, ctypes.byref(h)) == -2
    assert lib.nyls_plan_create(ctypes.cast(arr, ctypes.c_void_p), 1, 7, ctypes.byref(h)) == -3
    assert lib.nyls_plan_create(None, 1, 0, ctypes.byref(h)) == -1


def test_work_functions_reject_null_plan():
    lib = nyls.load()
    assert lib.nyls_solve(None, 0, None, None, None, None, None, None, None) == -1
    assert lib.nyls_assemble(None, None, None, None, None) == -1
    assert lib.nyls_features(None, None, None, 0, None, None, None, None, None) == -1
    assert lib.nyls_basis(None, None, None, None, None) == -1
    assert lib.nyls_error_string(-5).decode().startswith("need 2 <= m")
