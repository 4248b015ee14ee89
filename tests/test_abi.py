"""The C ABI library loads and exports every symbol include/fe.h declares (CPU only).

Only host-side helpers without device work are called here.
"""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import recursion as R

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fe.h")


def declared_symbols():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(fe_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    from paper_2605_08523_amd import api
    if not os.path.exists(api.LIB_PATH):
        pytest.fail("libfe.so is not built (python -m paper_2605_08523_amd.build)")
    return api.lib()


def test_every_declared_symbol_is_exported(lib):
    syms = declared_symbols()
    assert len(syms) >= 9
    for s in syms:
        assert hasattr(lib, s), s


def test_binding_covers_the_header():
    from paper_2605_08523_amd import api
    assert set(declared_symbols()) == set(api.SIGNATURES)


def test_sp2_coeffs_match_oracle(lib):
    from paper_2605_08523_amd import api
    for mu_p in (0.1, 0.37, 0.5, 0.81):
        np.testing.assert_array_equal(api.sp2_coeffs(mu_p, 40), R.sp2_mu_coeffs(mu_p, 40))


def test_layer_count_matches_oracle(lib):
    from paper_2605_08523_amd import api
    for b in (40.0, 1500.0, 1e4):
        assert api.layer_count(b) == pytest.approx(R.layer_count(b), rel=1e-14)


def test_argument_errors_without_device(lib):
    from paper_2605_08523_amd import api
    out = np.zeros((2, 4))
    rc = lib.fe_sp2_coeffs(1.5, 2, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    assert rc == api.FE_ERR_DOMAIN
    assert b"mu'" in lib.fe_last_error()
    rc = lib.fe_expand_density(None, 4, 4, 0.0, 0.1, None, 2, 0, None, 0, 4, None, None, None, None, None)
    assert rc == api.FE_ERR_ARG
    assert lib.fe_version().startswith(b"fe-mi355x")


def test_tuner_and_plan_argument_errors_without_device(lib):
    """The tuners and batch-plan calls reject bad arguments before any device work."""
    from paper_2605_08523_amd import api
    i32 = ctypes.c_int32()
    ms = (ctypes.c_double * 3)()
    # fe_autotune_input: precision first, then the arguments of fe_expand_density
    rc = lib.fe_autotune_input(None, 4, 4, 0.0, 0.1, None, api.PREC["fp32"], ctypes.byref(i32), ms,
                               None, None)
    assert rc == api.FE_ERR_ARG and b"16-bit" in lib.fe_last_error()
    rc = lib.fe_autotune_input(None, 4, 4, 0.0, 0.1, None, api.PREC["fp16x2"], ctypes.byref(i32), ms,
                               None, None)
    assert rc == api.FE_ERR_ARG and b"workspace" in lib.fe_last_error()
    # fe_autotune: no sizes; fe_autotune_lookup: no workspace
    assert lib.fe_autotune(None, 0, api.PREC["fp16x2"], None, None, None, None) == api.FE_ERR_ARG
    assert lib.fe_autotune_lookup(128, api.PREC["fp16x2"], None, ctypes.byref(i32)) == api.FE_ERR_ARG
    assert lib.fe_autotune_clear() == api.FE_OK
    # batch plans: NULL plan, bad tile size
    assert lib.fe_batch_plan_retile(None, 64) == api.FE_ERR_ARG
    assert lib.fe_batch_plan_autotune(None, None, ctypes.byref(i32), ms) == api.FE_ERR_ARG
    assert lib.fe_batch_plan_launch(None, None) == api.FE_ERR_ARG
    assert lib.fe_batch_plan_destroy(None) == api.FE_OK
    # launch form and plan queries on a NULL plan
    assert lib.fe_batch_plan_set_launch(None, api.BATCH_LAUNCH["queue"]) == api.FE_ERR_ARG
    assert lib.fe_batch_plan_get(None, ctypes.byref(i32), None) == api.FE_ERR_ARG
    # plan creation: output pointer, precision, workspace, then an empty batch
    plan = ctypes.c_void_p()
    rc = lib.fe_batch_plan_create(None, 0, None, None, 0.0, api.PREC["fp16x2"], None, None, None)
    assert rc == api.FE_ERR_ARG and b"out" in lib.fe_last_error()
    rc = lib.fe_batch_plan_create(None, 1, None, None, 0.0, api.PREC["fp32"], None, None,
                                  ctypes.byref(plan))
    assert rc == api.FE_ERR_ARG and b"FP16x2" in lib.fe_last_error() and plan.value is None
    rc = lib.fe_batch_plan_create(None, 1, None, None, 0.0, api.PREC["fp16x2"], None, None,
                                  ctypes.byref(plan))
    assert rc == api.FE_ERR_ARG and b"workspace" in lib.fe_last_error()
    rc = lib.fe_batched_expand(None, 0, None, None, 0.0, api.PREC["fp16x2"], None, None, None)
    assert rc == api.FE_ERR_ARG
    # queue layout: tile size, queue count, sizes that are not whole tiles
    np_ = (ctypes.c_int64 * 2)(128, 192)
    L = (ctypes.c_int32 * 2)(3, 2)
    qoff = (ctypes.c_int32 * 17)()
    nitems = ctypes.c_int64()
    assert lib.fe_batch_queue_layout(2, np_, L, 96, 8, None, 0, qoff,
                                     ctypes.byref(nitems)) == api.FE_ERR_ARG
    assert lib.fe_batch_queue_layout(2, np_, L, 64, 17, None, 0, qoff,
                                     ctypes.byref(nitems)) == api.FE_ERR_ARG
    assert lib.fe_batch_queue_layout(2, np_, L, 128, 8, None, 0, qoff,
                                     ctypes.byref(nitems)) == api.FE_ERR_ARG
    assert b"multiple of the tile" in lib.fe_last_error()
    assert lib.fe_batch_queue_layout(0, np_, L, 64, 8, None, 0, qoff,
                                     ctypes.byref(nitems)) == api.FE_ERR_ARG
    # counting only (items NULL), then a buffer one item too small
    assert lib.fe_batch_queue_layout(2, np_, L, 64, 8, None, 0, qoff,
                                     ctypes.byref(nitems)) == api.FE_OK
    assert nitems.value > 0 and qoff[8] == nitems.value
    small = (ctypes.c_int32 * (4 * nitems.value))()
    assert lib.fe_batch_queue_layout(2, np_, L, 64, 8, small, nitems.value - 1, qoff,
                                     ctypes.byref(nitems)) == api.FE_ERR_ARG
