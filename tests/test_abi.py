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
    rc = lib.fe_expand_density(None, 4, 4, 0.0, 0.1, None, 2, None, 0, 4, None, None, None, None, None)
    assert rc == api.FE_ERR_ARG
    assert lib.fe_version().startswith(b"fe-mi355x")
