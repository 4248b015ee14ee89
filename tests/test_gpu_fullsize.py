"""Full-size configurations, in the launch configuration bench.py times.

* The batch of 1024 uneven matrices (N_b ~ U{64..768}), with the 40-layer model at beta0 = 1e4
  and over the benchmark's model bank: every item's status, and sampled items (the smallest, the
  largest and three seeded picks) against the oracle's eigendecomposition, element by element.
* One N = 16384 solve, against the oracle's reference values for its seeded input, stored by a
  script that calls only the oracle (its FP64 eigendecomposition takes minutes): sampled rows of D,
  D times probe vectors, Tr D, sum D_ij^2 and S."""
import numpy as np
import pytest

from oracle import fermi as F
from paper_2605_08523_amd import models
from paper_2605_08523_amd import workloads as W
from parity import within

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_08523_amd import api as _api
    _api.lib()
    return _api


# measured on MI355X for the sampled items: (||dD||_F/N, |dTr D|) with the 40-layer model, and
# ||dD||_F/N with each item's bank model, against the exact D
MEASURED_1024 = {211: (7.545e-07, 5.766e-05), 61: (1.753e-06, 1.924e-03), 649: (1.253e-06, 2.017e-04),
                 661: (4.906e-07, 1.483e-03), 804: (1.378e-06, 2.953e-03)}
MEASURED_1024_BANK = {211: 2.661e-07, 61: 5.677e-08, 649: 1.886e-07, 661: 9.318e-08, 804: 9.188e-08}


# the batch in the three-part BF16 split (single-model plan), same sample: (||dD||_F/N, |dTr D|)
MEASURED_1024_BF16X3 = {211: (4.397e-07, 1.627e-05), 61: (1.369e-06, 1.427e-03),
                        649: (1.116e-06, 1.559e-04), 661: (2.730e-07, 6.754e-04),
                        804: (8.505e-07, 1.542e-03)}


def test_batch1024_bf16x3_sampled_against_oracle(api):
    """The batch in BF16 arithmetic: the three-part split meets the bar where the two-part BF16
    split does not (beta' up to ~3700)."""
    m = models.load("mlsp2_L40_b1e4_mu1third")
    items = W.batch_items(1024, 2000)
    mats = [dict(H=torch.from_numpy(it["H"]).cuda(), mu=it["mu"], kT=it["kT"]) for it in items]
    print("case batch1024 bf16x3", flush=True)
    plan = api.BatchPlan(mats, m, prec="bf16x3")
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
        dtr = abs(float(plan.tr[b, 0]) - ref["trD"])
        print(f"[batch1024 bf16x3 item {b}] N={n} kT={it['kT']:.3f} |dD|_F/N={fro:.3e} "
              f"max|dD|={np.max(np.abs(Dg - ref['D'])):.3e} |dTrD|={dtr:.3e}", flush=True)
        within(f"batch1024 bf16x3 item {b} |dD|_F/N", fro, MEASURED_1024_BF16X3[b][0], cap=1e-5)
        within(f"batch1024 bf16x3 item {b} |dTrD|", dtr, MEASURED_1024_BF16X3[b][1])
        assert np.array_equal(Dg, Dg.T)
    plan.close()


def test_batch1024_sampled_against_oracle(api):
    m = models.load("mlsp2_L40_b1e4_mu1third")
    items = W.batch_items(1024, 2000)
    mats = [dict(H=torch.from_numpy(it["H"]).cuda(), mu=it["mu"], kT=it["kT"]) for it in items]
    print("case batch1024 fp16x2", flush=True)
    plan = api.BatchPlan(mats, m, prec="fp16x2")
    assert plan.launch_form == "queue"   # a batch that fills the GPU defaults to the queue launch
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
        dtr = abs(float(plan.tr[b, 0]) - ref["trD"])
        print(f"[batch1024 item {b}] N={n} kT={it['kT']:.3f} |dD|_F/N={fro:.3e} "
              f"max|dD|={np.max(np.abs(Dg - ref['D'])):.3e} |dTrD|={dtr:.3e}", flush=True)
        within(f"batch1024 item {b} |dD|_F/N", fro, MEASURED_1024[b][0], cap=1e-5)
        within(f"batch1024 item {b} |dTrD|", dtr, MEASURED_1024[b][1])
        assert np.array_equal(Dg, Dg.T)
    # the plan's default launch (every layer in one queue launch, as the benchmark times it)
    # against one grouped launch per layer: bitwise equal over the whole batch
    print("case batch1024 fp16x2 queue launch vs per-layer launches", flush=True)
    Dq = [d.clone() for d in plan.D]
    trq = plan.tr.clone()
    plan.set_launch("layers")
    plan.launch()
    torch.cuda.synchronize()
    assert int(np.count_nonzero(plan.status.cpu().numpy())) == 0
    assert all(torch.equal(plan.D[b], Dq[b]) for b in range(1024))
    assert torch.equal(plan.tr, trq)
    del Dq
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
              f"|dD|_F/N={fro:.3e} max|dD|={np.max(np.abs(Dg - ref['D'])):.3e}", flush=True)
        within(f"batch1024 bank item {b} |dD|_F/N", fro, MEASURED_1024_BANK[b], cap=1e-5)
        assert np.array_equal(Dg, Dg.T)
    bplan.close()


# N = 16384 solve against the oracle's stored reference, measured on MI355X: the largest |dD| over
# the sampled rows, the relative error of D v for the probe vectors, |dTr D| and |d sum D_ij^2|
# against the oracle's recursion with the same model, |dS| of the entropy expansion (theta_fermi
# reused, alpha = 0.842704); each bound is 10x its measured value
LARGE_MEASURED = {
    "dp": dict(rows_max=3.758e-06, probes_rel=1.372e-05, tr=9.908e-03, sq=1.767e-02),
    "sk2": dict(rows_max=3.758e-06, probes_rel=1.373e-05, tr=9.930e-03, sq=1.769e-02),
    "sk": dict(rows_max=3.788e-06, probes_rel=1.372e-05, tr=9.926e-03, sq=1.758e-02),
    "bank": dict(rows_max=5.307e-06, probes_rel=2.665e-05, tr=2.058e-02, sq=2.726e-02),
    "entropy": dict(S=2.052e-02),
    "theta_entropy": dict(S=1.479e-02),
}


def _compare_large(tag, D, tr, tr2, ref, prefix, V, rows):
    Dd = D.double()
    dv = (Dd @ V).cpu().numpy()
    del Dd
    drow = D[rows].double().cpu().numpy()
    e_rows = float(np.max(np.abs(drow - ref[f"{prefix}_rows"])))
    e_rows_exact = float(np.max(np.abs(drow - ref["exact_rows"])))
    e_probe = float(np.linalg.norm(dv - ref[f"{prefix}_probes"]) / np.linalg.norm(ref[f"{prefix}_probes"]))
    e_tr = abs(float(tr) - float(ref[f"{prefix}_trD"]))
    e_sq = abs(float(tr2) - float(ref[f"{prefix}_trD2"]))
    print(f"[{tag}] rows max|dD| {e_rows:.3e} (vs exact {e_rows_exact:.3e}) |dDv|/|Dv| "
          f"{e_probe:.3e} |dTrD| {e_tr:.3e} |d sum D^2| {e_sq:.3e}", flush=True)
    return dict(rows_max=max(e_rows, e_rows_exact), probes_rel=e_probe, tr=e_tr, sq=e_sq)


def _check_large(results):
    for tag, res in results:
        for k, v in res.items():
            within(f"large16384 {tag} {k}", v, LARGE_MEASURED[tag][k])


def test_large16384_against_oracle(api, monkeypatch):
    """The N = 16384 solve against the oracle's reference for this seeded input
    (tests/golden/large16384_oracle.npz, written by make_large16384.py beside it from one FP64
    eigendecomposition): eight sampled rows of D element by element, D v for four probe vectors,
    Tr D and sum D_ij^2 against the oracle's recursion with the same model (and the rows against
    the exact Fermi-Dirac D), and S from the entropy expansion. Every schedule (the data-parallel
    one the benchmark's input tuner picks for this matrix, both stream-K ones) with the 40-layer
    model, then the model the benchmark's bank selects; mu is the oracle's 40%-filling value."""
    import os
    ref = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                               "large16384_oracle.npz"))
    m = models.load("mlsp2_L40_b1e4_mu1third")
    c = W.config_large_banded()
    n = c["H"].shape[0]
    Hd = torch.from_numpy(c["H"]).cuda()
    del c["H"]
    mu, kT = float(ref["mu"]), float(ref["kT"])
    assert kT == c["kT"]
    V = torch.from_numpy(ref["V"]).cuda()
    rows = torch.from_numpy(ref["rows"]).cuda()
    ws = api.Workspace(n)
    results = []
    for sch in ("dp", "sk2", "sk"):
        monkeypatch.setenv("FE_SCHEDULE", sch)
        print(f"case large16384 schedule {sch} mu={mu:.12f}", flush=True)
        D, tr, tr2, info = api.expand_density(Hd, mu, kT, m, prec="fp16x2", ws=ws, want_info=True)
        torch.cuda.synchronize()
        assert info["clamped"] == 0 and info["beta_p"] == pytest.approx(float(
            ref["mlsp2_L40_b1e4_mu1third_beta_p"]), rel=1e-12)
        assert torch.equal(D, D.T)
        results.append((sch, _compare_large(f"large16384 {sch}", D, tr, tr2, ref,
                                            "mlsp2_L40_b1e4_mu1third", V, rows)))
        del D
    monkeypatch.delenv("FE_SCHEDULE")
    S, _ = api.expand_entropy(Hd, mu, kT, m, float(ref["alpha_reuse"]), prec="fp16x2", ws=ws)
    torch.cuda.synchronize()
    dS = abs(float(S) - float(ref["mlsp2_L40_b1e4_mu1third_S"]))
    print(f"[large16384 entropy] S={float(S):.6f} oracle recursion "
          f"{float(ref['mlsp2_L40_b1e4_mu1third_S']):.6f} exact {float(ref['exact_S']):.6f} "
          f"|dS| {dS:.3e}", flush=True)
    results.append(("entropy", dict(S=dS)))
    # the trained 40-layer entropy model (theta_entropy) against the oracle's recursion with it
    me = models.load("entropy_L40_b1e4_mu1third")
    Se, _ = api.expand_entropy(Hd, mu, kT, me, me.alpha, prec="fp16x2", ws=ws)
    torch.cuda.synchronize()
    dSe = abs(float(Se) - float(ref["entropy_L40_b1e4_mu1third_S"]))
    print(f"[large16384 theta_entropy] S={float(Se):.6f} oracle recursion "
          f"{float(ref['entropy_L40_b1e4_mu1third_S']):.6f} exact {float(ref['exact_S']):.6f} "
          f"|dS| {dSe:.3e}", flush=True)
    results.append(("theta_entropy", dict(S=dSe)))
    # the model the benchmark's bank selects for this matrix
    import bench
    bank = [models.load(x) for x in bench.BANK]
    k = api.select_model(Hd, mu, kT, bank, ws=ws)
    print(f"case large16384 bank model {bench.BANK[k]}", flush=True)
    assert bench.BANK[k] == "mlsp2_L36_b1e4_mu0p5"
    D, tr, tr2, info = api.expand_density(Hd, mu, kT, bank[k], prec="fp16x2", ws=ws, want_info=True)
    torch.cuda.synchronize()
    assert info["clamped"] == 0
    results.append(("bank", _compare_large("large16384 bank", D, tr, tr2, ref,
                                           "mlsp2_L36_b1e4_mu0p5", V, rows)))
    del D
    torch.cuda.synchronize()
    ws.close()
    _check_large(results)
