"""The C ABI library loads on the CPU, exports every symbol include/wlra.h
declares, and its host-only argument checks behave (no compute calls)."""
import ctypes
import os
import re

import pytest

from paper_1703_06303_amd import wlra

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "wlra.h")).read()
    return sorted(set(re.findall(r"\b(wlra_[a-z_]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    lib = wlra.load()
    names = _declared()
    assert set(names) == set(wlra.SYMBOLS)
    for name in names:
        assert hasattr(lib, name), name


def test_version_and_strerror():
    assert wlra.load().wlra_version() >= 100
    for code in (0, 1, 2, -1, -2, -3, -4, -5, -6, -7, -8, -9, -10):
        assert wlra.strerror(code) != "unknown status"


def _prob(**kw):
    p = wlra.Problem()
    p.m, p.n, p.k, p.r = 100, 20, 5, 8
    p.A, p.lda = 1, 100
    p.W1, p.ldw = 1, 100
    p.max_sweeps = 10
    p.X1_out, p.ldx1 = 1, 100
    for k, v in kw.items():
        setattr(p, k, v)
    return p


@pytest.mark.parametrize("kw,ok", [
    ({}, True),
    ({"k": 9}, False),                      # k > r
    ({"r": 21}, False),                     # r > min(m, n)
    ({"lda": 99}, False),                   # lda < m
    ({"ldw": 50}, False),
    ({"A": 0}, False),
    ({"X1_out": 0}, False),
    ({"max_sweeps": -1}, False),
    ({"k": 0, "X1_out": 0}, True),          # k = 0 needs no X1
    ({"k": 65, "r": 65, "n": 100}, False),  # beyond the register-tile maximum
    ({"r": 40, "n": 60}, False),            # r - k beyond the eigen block
    ({"init": 1, "X1_init": 0}, False),     # given start without a matrix
    ({"init": 1, "X1_init": 1, "ldx0": 100}, True),
    ({"X2_out": 1, "ldx2": 10}, False),
    ({"mask_out": 1, "ldm": 100, "mask_tau": 0.3}, True),
    ({"mask_out": 1, "ldm": 99, "mask_tau": 0.3}, False),      # ldm < m
    ({"mask_out": 1, "ldm": 100, "mask_tau": -0.1}, False),    # negative threshold
    ({"mask_out": 1, "ldm": 100, "mask_tau": float("nan")}, False),
    ({"V_init": 1, "v0_rows": 15, "ldv0": 15}, True),          # n - k = 15 rows
    ({"V_init": 1, "v0_rows": 16, "ldv0": 16}, False),         # more rows than n - k
    ({"V_init": 1, "v0_rows": 0, "ldv0": 1}, False),
    ({"V_init": 1, "v0_rows": 10, "ldv0": 9}, False),          # ldv0 < v0_rows
    ({"W2": 1}, True),                                         # weights are checked on the device
])
def test_validate(kw, ok):
    rc = wlra.validate(_prob(**kw), wlra.FP32)
    assert (rc == 0) == ok, (kw, rc)


def test_bad_precision_and_null():
    assert wlra.validate(_prob(), 7) == wlra.E_ARG
    assert wlra.load().wlra_validate(None, 1) == wlra.E_ARG
    assert wlra.load().wlra_solve(None, None, None) == wlra.E_ARG


def test_set_option_rejects_null_handle():
    lib = wlra.load()
    assert lib.wlra_set_option(None, wlra.OPT_EIG_MAXIT, 5) == wlra.E_ARG


def test_create_without_device():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert wlra.load().wlra_create(ctypes.byref(h), 0, None, 1, 0) == wlra.E_NODEVICE
