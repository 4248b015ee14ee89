"""Full-size configurations, in the launch configuration bench.py times.

* The batch of 1024 uneven matrices (N_b ~ U{64..768}), with the 40-layer model at beta0 = 1e4
  and over the benchmark's model bank: every item's status, and sampled items (the smallest, the
  largest and three seeded picks) against the oracle's eigendecomposition, element by element.
* One N = 16384 solve: the oracle's eigendecomposition would take tens of minutes, so the FP16x2
  result is checked against the FP64 expansion on the GPU (itself pinned to the oracle at smaller
  sizes) and against properties that hold at any size (exact symmetry, 0 <= sum D_ij^2 <= Tr D,
  Tr D near the 40% filling the chemical potential was placed at)."""
import numpy as np
import pytest

from oracle import fermi as F
from paper_2605_08523_amd import models
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


def test_batch1024_sampled_against_oracle(api):
    m = models.load("mlsp2_L40_b1e4_mu1third")
    items = W.batch_items(1024, 2000)
    mats = [dict(H=torch.from_numpy(it["H"]).cuda(), mu=it["mu"], kT=it["kT"]) for it in items]
    print("case batch1024 fp16x2", flush=True)
    plan = api.BatchPlan(mats, m, prec="fp16x2")
    plan.launch()
    torch.cuda.synchronize()
    assert int(np.count_nonzero(plan.status.cpu().numpy())) == 0
    ns = np.array([it["n"] for it in items])
    order = np.argsort(ns, kind="stable")
    rng = np.random.default_rng(77)
    sample = [int(order[0]), int(order[-1])] + [int(b) for b in rng.choice(1024, 3, replace=False)]
    for b in sample:
        it = items[b]
        ref = F.density(it["H"], it["mu"], it["kT"])
        Dg = plan.D[b].double().cpu().numpy()
        n = it["n"]
        fro = np.linalg.norm(Dg - ref["D"]) / n
        print(f"[batch1024 item {b}] N={n} kT={it['kT']:.3f} |dD|_F/N={fro:.3e} "
              f"|dTrD|={abs(float(plan.tr[b, 0]) - ref['trD']):.3e}", flush=True)
        assert fro <= 1e-5
        assert np.array_equal(Dg, Dg.T)
    # the same batch over the benchmark's model bank (each matrix runs its selected model)
    import bench
    bank = [models.load(x) for x in bench.BANK]
    plan.close()
    print("case batch1024 fp16x2 bank", flush=True)
    bplan = api.BatchPlan(mats, bank, prec="fp16x2", ws=plan.ws)
    bplan.launch()
    torch.cuda.synchronize()
    assert int(np.count_nonzero(bplan.status.cpu().numpy())) == 0
    assert len(set(bplan.chosen.tolist())) >= 5
    for b in sample:
        it = items[b]
        ref = F.density(it["H"], it["mu"], it["kT"])
        Dg = bplan.D[b].double().cpu().numpy()
        fro = np.linalg.norm(Dg - ref["D"]) / it["n"]
        print(f"[batch1024 bank item {b}] N={it['n']} model {bench.BANK[int(bplan.chosen[b])]} "
              f"|dD|_F/N={fro:.3e}", flush=True)
        assert fro <= 1e-5
        assert np.array_equal(Dg, Dg.T)
    bplan.close()


def test_large16384_against_fp64_expansion(api, monkeypatch):
    """Every schedule (the data-parallel one the bench's input tuner picks for this matrix, the
    two stream-K ones) against one FP64 expansion."""
    m = models.load("mlsp2_L40_b1e4_mu1third")
    c = W.config_large_banded()
    n = c["H"].shape[0]
    Hd = torch.from_numpy(c["H"]).cuda()
    del c["H"]
    lam = torch.linalg.eigvalsh(Hd).cpu().numpy()
    k = int(0.4 * n)
    mu, kT = float(0.5 * (lam[k - 1] + lam[k])), c["kT"]
    print(f"case large16384 mu={mu:.6f}", flush=True)
    ws = api.Workspace(n)
    D64, tr64, _, _ = api.expand_density(Hd, mu, kT, m, prec="fp64", ws=ws,
                                         out_dtype=torch.float64, want_info=True)
    torch.cuda.synchronize()
    for sch in ("dp", "sk2", "sk"):
        monkeypatch.setenv("FE_SCHEDULE", sch)
        print(f"case large16384 schedule {sch}", flush=True)
        D, tr, tr2, info = api.expand_density(Hd, mu, kT, m, prec="fp16x2", ws=ws, want_info=True)
        torch.cuda.synchronize()
        assert info["clamped"] == 0
        assert torch.equal(D, D.T)
        err = D.double() - D64
        fro = float(torch.linalg.norm(err).item()) / n
        print(f"[large16384 {sch}] |dD|_F/N={fro:.3e} max={float(err.abs().max()):.3e} "
              f"TrD={float(tr):.4f} (target {0.4 * n}) TrD64={float(tr64):.4f}", flush=True)
        assert fro <= 1e-5
        assert 0.0 <= float(tr2) <= float(tr) + 1e-6 * n
        assert abs(float(tr) - 0.4 * n) < 0.01 * n
        del D, err
    monkeypatch.delenv("FE_SCHEDULE")
    del D64
    # the model the benchmark's bank selects for this matrix, against its own FP64 expansion
    import bench
    bank = [models.load(x) for x in bench.BANK]
    k = api.select_model(Hd, mu, kT, bank, ws=ws)
    mb = bank[k]
    print(f"case large16384 bank model {bench.BANK[k]}", flush=True)
    assert mb.L < m.L
    D, tr, _, info = api.expand_density(Hd, mu, kT, mb, prec="fp16x2", ws=ws, want_info=True)
    D64, _, _, _ = api.expand_density(Hd, mu, kT, mb, prec="fp64", ws=ws, out_dtype=torch.float64,
                                      want_info=True)
    torch.cuda.synchronize()
    assert info["clamped"] == 0
    fro = float(torch.linalg.norm(D.double() - D64).item()) / n
    print(f"[large16384 bank {bench.BANK[k]}] |dD|_F/N={fro:.3e} TrD={float(tr):.4f}", flush=True)
    assert fro <= 1e-5
    assert abs(float(tr) - 0.4 * n) < 0.01 * n
    del D, D64
    torch.cuda.synchronize()
    ws.close()
