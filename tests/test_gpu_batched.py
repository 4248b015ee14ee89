"""GPU parity of the batched path (fe_batch_plan_* / fe_batched_expand) against the oracle and
against the single-matrix entry point on the same matrices."""
import numpy as np
import pytest

from oracle import fermi as F
from oracle import recursion as R
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


def uneven_batch(count, seed0, n_lo=64, n_hi=400):
    mats = []
    for b in range(count):
        rng = np.random.default_rng(seed0 + b)
        n = int(rng.integers(n_lo, n_hi + 1))
        H = W.banded_decay(n, 8.0, 2.0, seed0 + 1000 + b)
        lam = np.linalg.eigvalsh(H)
        mu = float(lam[0] + rng.uniform(0.2, 0.8) * (lam[-1] - lam[0]))
        kT = float(rng.uniform(0.05, 0.3))
        mats.append(dict(Hn=H, H=torch.from_numpy(H).cuda(), mu=mu, kT=kT))
    return mats


# measured on MI355X: ||dD||_F/N of each item against the oracle recursion
MEASURED_BATCH12 = [1.215e-07, 1.160e-07, 2.853e-07, 2.305e-07, 1.273e-07, 6.448e-08, 1.481e-07,
                    1.708e-07, 2.440e-07, 1.146e-07, 1.676e-07, 1.236e-07]


# the same with the three-part BF16 split
MEASURED_BATCH12_BF16X3 = [1.495e-07, 1.269e-07, 3.231e-07, 2.792e-07, 1.451e-07, 7.094e-08,
                           1.682e-07, 1.786e-07, 2.390e-07, 1.300e-07, 1.781e-07, 1.412e-07]


@pytest.mark.parametrize("prec", ["fp16x2", "bf16x3"])
def test_batch_matches_single_and_oracle(api, paper_model, monkeypatch, prec):
    m = paper_model
    mats = uneven_batch(12, 500)
    print(f"case batch12 {prec}", flush=True)
    plan = api.BatchPlan(mats, m, prec=prec, model_s=m, alpha=0.842704)
    plan.launch()
    torch.cuda.synchronize()
    assert plan.status.cpu().numpy().tolist() == [0] * 12
    monkeypatch.setenv("FE_SCHEDULE", "dp")
    measured = MEASURED_BATCH12 if prec == "fp16x2" else MEASURED_BATCH12_BF16X3
    for b, it in enumerate(mats):
        Db = plan.D[b]
        D1, tr1, tr21, _ = api.expand_density(it["H"], it["mu"], it["kT"], m, prec=prec)
        S1, _ = api.expand_entropy(it["H"], it["mu"], it["kT"], m, 0.842704, prec=prec)
        torch.cuda.synchronize()
        # same tiles, K-block order and epilogue arithmetic as the single-matrix data-parallel
        # kernel: D bitwise equal, and so is Tr D (an FP64 sum of FP32 values, exact in any
        # order); sum D^2 and S add FP64 values in an order that follows the workgroup's wave
        # count (eight waves here, four there), so they agree to FP64 rounding
        assert torch.equal(Db, D1), f"item {b}"
        assert float(plan.tr[b, 0]) == float(tr1)
        assert abs(float(plan.tr[b, 1]) - float(tr21)) <= 1e-12 * max(1.0, abs(float(tr21)))
        assert abs(float(plan.S[b]) - float(S1)) <= 1e-12 * max(1.0, abs(float(S1)))
        Drec, _ = R.mlsp2_density(it["Hn"], it["mu"], it["kT"], m.theta, m.beta0, m.mu0)
        n = Drec.shape[0]
        E = Db.double().cpu().numpy() - Drec
        fro = np.linalg.norm(E) / n
        print(f"[batch item {b}] N={n} |dD|_F/N={fro:.3e} max|dD|={np.max(np.abs(E)):.3e}", flush=True)
        within(f"batch item {b} {prec}", fro, measured[b], cap=1e-5)


def test_batch_status_errors_and_replay(api, paper_model):
    m = paper_model
    mats = uneven_batch(5, 700)
    lo, hi = F.gershgorin(mats[2]["Hn"])
    mats[2]["mu"] = hi + 1.0                       # outside the bounds: domain error for item 2
    plan = api.BatchPlan(mats, m, prec="bf16x2")
    outs = []
    for _ in range(3):
        plan.launch()
        torch.cuda.synchronize()
        outs.append([d.clone() for d in plan.D])
    st = plan.status.cpu().numpy().tolist()
    assert st[2] == api.FE_ERR_DOMAIN and all(s == 0 for i, s in enumerate(st) if i != 2)
    assert torch.isnan(plan.D[2]).all() and np.isnan(float(plan.tr[2, 0]))
    for b in (0, 1, 3, 4):
        assert torch.isfinite(plan.D[b]).all()
        for r in (1, 2):
            assert torch.equal(outs[0][b], outs[r][b]), "graph replays must agree"
    # a newer plan on the same workspace makes this one stale
    plan2 = api.BatchPlan(mats[:2], m, prec="bf16x2", ws=plan.ws)
    with pytest.raises(api.FeError) as e:
        plan.launch()
    assert e.value.code == api.FE_ERR_WORKSPACE
    plan2.launch()
    torch.cuda.synchronize()


MEASURED_FAMILY = [4.620e-08, 1.230e-07, 1.210e-07, 1.313e-07, 3.856e-08, 1.133e-07, 1.922e-07,
                   1.063e-07, 7.816e-08, 3.995e-08, 9.787e-08, 7.314e-08, 3.996e-08, 6.996e-08,
                   1.483e-07, 5.047e-08]


def test_batch_config_family(api):
    """Items of the uneven-batch workload family (N in [64, 768], kT in [0.01, 0.3], mu inside
    the spectrum), with a clamp warning where beta' exceeds the paper model's region."""
    from paper_2605_08523_amd import models
    m = models.load("mlsp2_L26_b1500_mu1third")
    items = W.batch_items(count=16, base_seed=2000)
    mats = [dict(Hn=it["H"], H=torch.from_numpy(it["H"]).cuda(), mu=it["mu"], kT=it["kT"]) for it in items]
    plan = api.BatchPlan(mats, m, prec="fp16x2")
    plan.launch()
    torch.cuda.synchronize()
    st = plan.status.cpu().numpy()
    for b, it in enumerate(mats):
        Drec, info = R.mlsp2_density(it["Hn"], it["mu"], it["kT"], m.theta, m.beta0, m.mu0)
        assert st[b] == (api.FE_WARN_BETA_CLAMPED if info["clamped"] else 0)
        n = Drec.shape[0]
        E = plan.D[b].double().cpu().numpy() - Drec
        fro = np.linalg.norm(E) / n
        print(f"[batch family {b}] N={n} clamped={info['clamped']} |dD|_F/N={fro:.3e} "
              f"max|dD|={np.max(np.abs(E)):.3e}", flush=True)
        within(f"batch family {b}", fro, MEASURED_FAMILY[b], cap=1e-5)


BANK = ["mlsp2_L20_b300_mu1third", "mlsp2_L22_b600_mu1third", "mlsp2_L26_b1500_mu1third",
        "mlsp2_L40_b1e4_mu1third"]
# both trained families: mu0 = 1/3 and mu0 = 1/2 (regions of validity that meet at mu' = 0.4)
BANK_MIXED = BANK + ["mlsp2_L20_b300_mu0p5", "mlsp2_L22_b600_mu0p5", "mlsp2_L24_b1500_mu0p5",
                     "mlsp2_L36_b1e4_mu0p5"]


def expected_choice(H, mu, kT, bank):
    """The selection rule written out: fewest layers whose region of validity holds (beta', mu')."""
    lo, hi = F.gershgorin(H)
    width = hi - lo
    mu_p = (hi - mu) / width
    mu_p = 1.0 - mu_p if mu_p > 0.5 else mu_p
    beta_p = width / kT
    fits = [k for k, m in enumerate(bank)
            if beta_p <= min(m.mu0 / mu_p, (1 - m.mu0) / (1 - mu_p)) * m.beta0]
    return min(fits, key=lambda k: (bank[k].L, -bank[k].beta0))


# measured on MI355X: ||dD||_F/N of each item (with its selected model) against the exact D
MEASURED_BANK = {
    "mu1third": [2.177e-07, 1.304e-07, 7.419e-08, 2.869e-07, 4.626e-07, 1.035e-07, 1.755e-07,
                 8.431e-08, 4.235e-07, 1.860e-07],
    "mixed": [2.177e-07, 1.304e-07, 1.548e-07, 7.773e-07, 5.245e-07, 1.035e-07, 1.111e-07,
              2.012e-07, 1.241e-06, 3.623e-07],
}


@pytest.mark.parametrize("bank_name", ["mu1third", "mixed"])
def test_model_bank_batch(api, monkeypatch, bank_name):
    from paper_2605_08523_amd import models
    names = BANK if bank_name == "mu1third" else BANK_MIXED
    bank = [models.load(x) for x in names]
    rng = np.random.default_rng(77)
    mats = []
    for b in range(10):
        n = int(rng.integers(64, 400))
        H = W.banded_decay(n, 8.0, 2.0, 900 + b)
        lam = np.linalg.eigvalsh(H)
        mu = float(lam[0] + rng.uniform(0.3, 0.7) * (lam[-1] - lam[0]))
        kT = float([0.3, 0.12, 0.05, 0.02, 0.01][b % 5])
        mats.append(dict(Hn=H, H=torch.from_numpy(H).cuda(), mu=mu, kT=kT))
    print(f"case model-bank batch10 fp16x2 bank {bank_name}", flush=True)
    plan = api.BatchPlan(mats, bank, prec="fp16x2", with_entropy=True, alpha=0.842704)
    plan.launch()
    torch.cuda.synchronize()
    assert plan.status.cpu().numpy().tolist() == [0] * 10
    want = [expected_choice(it["Hn"], it["mu"], it["kT"], bank) for it in mats]
    print("[bank] chosen", plan.chosen.tolist(), "expected", want, flush=True)
    assert plan.chosen.tolist() == want
    assert len(set(want)) >= 3          # the batch really mixes models
    if bank_name == "mixed":
        assert any(bank[k].mu0 == 0.5 for k in want) and any(bank[k].mu0 != 0.5 for k in want)
    monkeypatch.setenv("FE_SCHEDULE", "dp")
    for b, it in enumerate(mats):
        m = bank[int(plan.chosen[b])]
        assert api.select_model(it["H"], it["mu"], it["kT"], bank) == want[b], f"item {b}"
        D1, tr1, _, _ = api.expand_density(it["H"], it["mu"], it["kT"], m, prec="fp16x2")
        S1, _ = api.expand_entropy(it["H"], it["mu"], it["kT"], m, 0.842704, prec="fp16x2")
        torch.cuda.synchronize()
        assert torch.equal(plan.D[b], D1), f"item {b}"
        assert abs(float(plan.S[b]) - float(S1)) <= 1e-12 * max(1.0, abs(float(S1)))   # FP64 sum order
        ref = F.density(it["Hn"], it["mu"], it["kT"])
        n = it["Hn"].shape[0]
        E = plan.D[b].double().cpu().numpy() - ref["D"]
        fro = np.linalg.norm(E) / n
        print(f"[bank item {b}] N={n} kT={it['kT']} model {m.name} |dD|_F/N={fro:.3e} "
              f"max|dD|={np.max(np.abs(E)):.3e}", flush=True)
        within(f"bank {bank_name} item {b}", fro, MEASURED_BANK[bank_name][b], cap=1e-5)


MEASURED_TILE64 = [1.844e-07, 2.978e-07, 3.710e-07, 1.843e-07, 3.450e-07, 2.791e-07, 9.276e-08,
                   2.049e-07, 1.962e-07, 1.840e-07, 2.025e-07, 1.895e-07, 1.675e-07, 2.516e-07,
                   2.942e-07, 1.126e-07]


def test_batch_tile_64_and_autotune(api, paper_model):
    """64 x 64 layer tiles (fe_batch_plan_retile) against the oracle, and the tile autotuner on a
    batch of small matrices (N 64 .. 300, where 128-tile padding wastes most)."""
    m = paper_model
    rng = np.random.default_rng(91)
    mats = []
    for b in range(16):
        n = int(rng.integers(64, 300))
        H = W.banded_decay(n, 8.0, 2.0, 700 + b)
        lam = np.linalg.eigvalsh(H)
        mu = float(lam[0] + rng.uniform(0.3, 0.7) * (lam[-1] - lam[0]))
        mats.append(dict(Hn=H, H=torch.from_numpy(H).cuda(), mu=mu, kT=float(rng.uniform(0.05, 0.3))))
    plan = api.BatchPlan(mats, m, prec="fp16x2", model_s=m, alpha=0.842704)
    plan.launch()
    torch.cuda.synchronize()
    D128 = [d.clone() for d in plan.D]
    S128 = plan.S.clone()
    print("case batch16 tile 64", flush=True)
    plan.retile(64)
    plan.launch()
    torch.cuda.synchronize()
    assert plan.status.cpu().numpy().tolist() == [0] * 16
    for b, it in enumerate(mats):
        Drec, _ = R.mlsp2_density(it["Hn"], it["mu"], it["kT"], m.theta, m.beta0, m.mu0)
        n = Drec.shape[0]
        fro = np.linalg.norm(plan.D[b].double().cpu().numpy() - Drec) / n
        d = float((plan.D[b] - D128[b]).abs().max())
        print(f"[tile64 item {b}] N={n} |dD|_F/N={fro:.3e} max|D64 - D128|={d:.2e}", flush=True)
        within(f"tile64 item {b}", fro, MEASURED_TILE64[b], cap=1e-5)
        assert d == 0.0, "both tile sizes sum each element over K in the same order"
        assert torch.equal(plan.D[b], plan.D[b].T)
    assert torch.allclose(plan.S, S128, rtol=1e-5, atol=1e-6)
    tile, ms = plan.autotune()
    print(f"[batch autotune] tile {tile} ({ms})", flush=True)
    assert tile in (64, 128) and ms[tile] == min(ms.values()) and all(v > 0 for v in ms.values())
    plan.launch()
    torch.cuda.synchronize()
    assert plan.status.cpu().numpy().tolist() == [0] * 16
    for b in range(16):
        assert float((plan.D[b] - D128[b]).abs().max()) < 1e-4
    plan.close()


def test_bf16x3_plan_tiles(api, paper_model):
    """A three-part BF16 plan has the 128 x 128 tile only: the tuner times that one and keeps it,
    and a retile to 64 is refused."""
    mats = uneven_batch(3, 900)
    plan = api.BatchPlan(mats, paper_model, prec="bf16x3")
    tile, ms = plan.autotune()
    assert tile == 128 and set(ms) == {128}
    with pytest.raises(api.FeError) as e:
        plan.retile(64)
    assert e.value.code == api.FE_ERR_ARG
    plan.launch()
    torch.cuda.synchronize()
    assert plan.status.cpu().numpy().tolist() == [0] * 3


def test_batched_expand_one_shot(api, paper_model):
    """fe_batched_expand (plan, launch, wait, destroy in one call): the same D, traces, S and
    status as a captured plan of the same batch, and the oracle's D within the bar."""
    m = paper_model
    mats = uneven_batch(6, 1300)
    print("case one-shot batch6 fp16x2 with entropy", flush=True)
    D, tr, S, status = api.batched_expand(mats, m, prec="fp16x2", model_s=m, alpha=0.842704)
    assert status.cpu().numpy().tolist() == [0] * 6
    plan = api.BatchPlan(mats, m, prec="fp16x2", model_s=m, alpha=0.842704)
    plan.launch()
    torch.cuda.synchronize()
    for b, it in enumerate(mats):
        assert torch.equal(D[b], plan.D[b]), f"item {b}"
        Drec, _ = R.mlsp2_density(it["Hn"], it["mu"], it["kT"], m.theta, m.beta0, m.mu0)
        n = Drec.shape[0]
        assert np.linalg.norm(D[b].double().cpu().numpy() - Drec) / n <= 1e-5
    assert torch.equal(tr, plan.tr) and torch.equal(S, plan.S)
    plan.close()
