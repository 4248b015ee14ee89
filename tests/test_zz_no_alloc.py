"""fe_expand_density_noalloc (the entry point that allocates nothing) against fe_expand_density.

Two calls in a row through the C ABI, the second with a smaller matrix (the static scratch keeps
the first call's contents), for each precision: D and the traces must equal those of
fe_expand_density on the same input (same kernels, same schedule: bitwise), and the second
result must match the oracle's recursion to the parity bar. Sizes beyond the stated limit are
rejected before any device work.
"""
import ctypes

import numpy as np
import pytest

from oracle import recursion as R
from paper_2605_08523_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_08523_amd import api as _api
    _api.lib()
    return _api


@pytest.mark.parametrize("prec,sizes,tol", [("fp16x2", (2000, 700), 1e-5), ("bf16x2", (1500, 333), 1e-5),
                                            ("fp32", (1200, 130), 1e-5), ("fp64", (1600, 100), 1e-11)])
def test_noalloc_matches_workspace_path(api, paper_model, monkeypatch, prec, sizes, tol):
    m = paper_model
    monkeypatch.setenv("FE_SCHEDULE", "dp")   # the schedule the no-allocation path always runs
    ws = api.Workspace(max(sizes))
    for k, n in enumerate(sizes):
        H = W.random_dense(n, 600 + k)
        mu, kT = 0.05, 0.1
        Hd = torch.from_numpy(H).cuda()
        out_dtype = torch.float64 if prec == "fp64" else torch.float32
        print(f"case noalloc {prec} call {k} n={n}", flush=True)
        D1, t1, s1, i1 = api.expand_density_noalloc(Hd, mu, kT, m, prec=prec, out_dtype=out_dtype,
                                                    want_info=True)
        D0, t0, s0, i0 = api.expand_density(Hd, mu, kT, m, prec=prec, out_dtype=out_dtype, ws=ws,
                                            want_info=True)
        torch.cuda.synchronize()
        assert i1["rc"] == i0["rc"] == 0
        assert torch.equal(D1, D0), "same kernels and schedule: identical D"
        assert float(t1) == float(t0) and float(s1) == float(s0)
        assert torch.equal(D1, D1.T)
        Drec, _ = R.mlsp2_density(H, mu, kT, m.theta, m.beta0, m.mu0)
        err = np.linalg.norm(D1.double().cpu().numpy() - Drec) / n
        print(f"[noalloc {prec} n={n}] |D - D_recursion|_F/N = {err:.3e}", flush=True)
        assert err <= tol
    ws.close()


def test_noalloc_rejects_sizes_beyond_the_scratch(api, paper_model):
    m = api.make_model(paper_model.theta, paper_model.beta0, paper_model.mu0)
    lib = api.lib()
    H = torch.zeros(16, dtype=torch.float64, device="cuda")   # never read: the size check fails first
    for prec, n in (("fp16x2", 2049), ("fp32", 2305), ("fp64", 1665)):
        rc = lib.fe_expand_density_noalloc(ctypes.c_void_p(H.data_ptr()), n, n, 0.0, 0.1,
                                           ctypes.byref(m.struct), api.PREC[prec], 0, None, 0, n,
                                           None, None, None, None)
        assert rc == api.FE_ERR_WORKSPACE, (prec, n, rc)
        assert b"no-allocation scratch" in lib.fe_last_error()
