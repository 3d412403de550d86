"""Loader of libnubulb_testhooks.so (include/nubulb_testhooks.h): the stepper's arithmetic
primitives one element per thread, for tests that hold each to its definition.  Argument
marshalling only; raises if the library was not built."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnubulb_testhooks.so")
EXPORTS = ["nb_test_sincos", "nb_test_sqrt_div", "nb_test_exp3", "nb_test_rotate",
           "nb_test_last_error"]

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        # the library works on torch's device memory and streams, so it must bind to the HIP
        # runtime torch loads: import torch first (loading the library first would bring in
        # a second runtime, which then finds no device)
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        vp, i64 = C.c_void_p, C.c_int64
        L.nb_test_sincos.argtypes = [vp, i64, vp, vp, vp]
        L.nb_test_sqrt_div.argtypes = [vp, vp, i64, vp, vp, vp]
        L.nb_test_exp3.argtypes = [vp, vp, i64, vp, vp]
        L.nb_test_rotate.argtypes = [vp, vp, i64, vp, vp]
        L.nb_test_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"{what} failed ({rc}): {lib().nb_test_last_error().decode(errors='replace')}")


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def test_sincos(x):
    import torch
    s = torch.empty_like(x); c = torch.empty_like(x)
    _check(lib().nb_test_sincos(_ptr(x), x.numel(), _ptr(s), _ptr(c), _stream()), "nb_test_sincos")
    return s, c


def test_sqrt_div(a, b):
    import torch
    sq = torch.empty_like(a); dv = torch.empty_like(a)
    _check(lib().nb_test_sqrt_div(_ptr(a), _ptr(b), a.numel(), _ptr(sq), _ptr(dv), _stream()),
           "nb_test_sqrt_div")
    return sq, dv


def test_exp3(k9, psi6):
    import torch
    out = torch.empty_like(psi6)
    _check(lib().nb_test_exp3(_ptr(k9), _ptr(psi6), psi6.shape[0], _ptr(out), _stream()),
           "nb_test_exp3")
    return out


def test_rotate(x3, p3):
    import torch
    out = torch.empty_like(p3)
    _check(lib().nb_test_rotate(_ptr(x3), _ptr(p3), p3.shape[0], _ptr(out), _stream()),
           "nb_test_rotate")
    return out
