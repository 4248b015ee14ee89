"""GPU parity of the batch queue launch (FE_BATCH_LAUNCH_QUEUE: every layer of every matrix in one
launch, dependencies tracked per matrix on the device) against the grouped per-layer launches of
the same plan: the same per-tile arithmetic in the same order, so D, the traces and S must agree
bit for bit, on every replay. The grouped launches are themselves checked against the oracle in
test_gpu_batched.py."""
import numpy as np
import pytest

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


def uneven_batch(count, seed0, n_lo=64, n_hi=520):
    mats = []
    for b in range(count):
        rng = np.random.default_rng(seed0 + b)
        n = int(rng.integers(n_lo, n_hi + 1))
        H = W.banded_decay(n, 8.0, 2.0, seed0 + 1000 + b)
        lam = np.linalg.eigvalsh(H)
        mu = float(lam[0] + rng.uniform(0.2, 0.8) * (lam[-1] - lam[0]))
        kT = float([0.3, 0.12, 0.05, 0.02][b % 4])
        mats.append(dict(H=torch.from_numpy(H).cuda(), mu=mu, kT=kT))
    return mats


def snapshot(plan):
    return ([d.clone() for d in plan.D], plan.tr.clone(), plan.S.clone(), plan.status.clone())


def assert_same(plan, ref, what):
    D, tr, S, st = ref
    assert torch.equal(plan.status, st), what
    for b in range(plan.count):
        assert torch.equal(plan.D[b], D[b]), f"{what}: item {b}"
    assert torch.equal(plan.tr, tr), what
    assert torch.equal(plan.S, S), what


CASES = [("fp16x2", 128, "single"), ("fp16x2", 64, "single"), ("bf16x3", 128, "single"),
         ("bf16x2", 128, "single"), ("fp16x2", 128, "bank"), ("fp16x2", 64, "bank")]


@pytest.mark.parametrize("prec,tile,kind", CASES)
def test_queue_launch_bitwise_equal_to_layer_launches(api, paper_model, prec, tile, kind):
    from paper_2605_08523_amd import models
    mats = uneven_batch(24, 4100)
    print(f"case queue-launch batch24 {prec} tile {tile} {kind}", flush=True)
    if kind == "bank":
        bank = [models.load(x) for x in ("mlsp2_L20_b300_mu1third", "mlsp2_L22_b600_mu1third",
                                          "mlsp2_L26_b1500_mu1third", "mlsp2_L40_b1e4_mu1third",
                                          "mlsp2_L20_b300_mu0p5", "mlsp2_L24_b1500_mu0p5")]
        plan = api.BatchPlan(mats, bank, prec=prec, with_entropy=True, alpha=0.842704)
        assert len(set(plan.chosen.tolist())) >= 3   # layer counts differ across the batch
    else:
        plan = api.BatchPlan(mats, paper_model, prec=prec, model_s=paper_model, alpha=0.842704)
    plan.set_launch("layers")
    if tile != 128:
        plan.retile(tile)
    plan.launch()
    torch.cuda.synchronize()
    ref = snapshot(plan)
    assert min(ref[3].cpu().numpy().tolist()) >= 0   # FE_OK, or FE_WARN_BETA_CLAMPED at kT = 0.02
    assert all(bool(torch.isfinite(d).all()) for d in ref[0])
    plan.set_launch("queue")
    for rep in range(3):   # graph replays: the counters are reset inside each pass
        for d in plan.D:
            d.fill_(float("nan"))
        plan.tr.fill_(float("nan"))
        plan.S.fill_(float("nan"))
        plan.launch()
        torch.cuda.synchronize()
        assert_same(plan, ref, f"queue replay {rep}")
    plan.set_launch("layers")
    plan.launch()
    torch.cuda.synchronize()
    assert_same(plan, ref, "back to layer launches")
    plan.close()


def test_queue_launch_give_up_reports_every_matrix(api, paper_model):
    """Failure handling forced from the host: every wait of a plan built under the test hook
    expects a count no matrix reaches, gives up after a short bounded spin, and the matrices
    report FE_ERR_HIP with NaN traces; a plan built afterwards runs normally."""
    mats = uneven_batch(6, 4300, n_hi=300)
    plan = api.BatchPlan(mats, paper_model, prec="fp16x2")
    plan.set_launch("layers")
    plan.launch()
    torch.cuda.synchronize()
    ref = snapshot(plan)
    print("case queue-launch give-up (host-forced)", flush=True)
    api.debug_batch_queue_giveup(True)
    try:
        plan.set_launch("queue")
    finally:
        api.debug_batch_queue_giveup(False)
    plan.launch()
    torch.cuda.synchronize()
    assert plan.status.cpu().numpy().tolist() == [api.FE_ERR_HIP] * 6
    assert bool(torch.isnan(plan.tr).all())
    plan.set_launch("queue")   # rebuilt without the hook
    plan.launch()
    torch.cuda.synchronize()
    assert_same(plan, ref, "queue launch after the give-up test")
    plan.close()


def test_queue_launch_tiny_matrices_every_replay(api, paper_model):
    """Matrices of one 128 x 128 tile (N = 1, 2, 3) hand each layer straight to the next item of
    the same matrix, often on the same CU, whose L1 still holds the lines it read two layers
    earlier: the hand-off must invalidate it. N = 1 also sits on the recursion's unstable fixed
    point (one eigenvalue at mu), so any stale read shows up as an O(1) change of D. Bitwise equal
    to the per-layer launches on every one of eight replays."""
    from oracle import fermi as F
    mats = []
    for n in (1, 2, 3, 17, 127, 128, 129, 255, 257):
        H = W.random_dense(n, 4000 + n)
        lo, hi = F.gershgorin(H)
        mats.append(dict(H=torch.from_numpy(H).cuda(), mu=float(0.3 * lo + 0.7 * hi), kT=0.1))
    print("case queue-launch tiny matrices x8 replays", flush=True)
    plan = api.BatchPlan(mats, paper_model, prec="fp16x2")
    plan.set_launch("layers")
    plan.launch()
    torch.cuda.synchronize()
    ref = snapshot(plan)
    plan.set_launch("queue")
    for rep in range(8):
        for d in plan.D:
            d.fill_(float("nan"))
        plan.launch()
        torch.cuda.synchronize()
        assert_same(plan, ref, f"tiny matrices, queue replay {rep}")
    plan.close()


def test_autotune_chooses_tile_and_launch_form(api, paper_model):
    """fe_batch_plan_autotune times both tile sizes under both launch forms and keeps the fastest
    pair (fe_batch_plan_get reports it); the tuned plan's results equal the default plan's at the
    same tile (both launch forms are bitwise equal, the tiles agree to FP32 rounding)."""
    mats = uneven_batch(10, 4500, n_hi=300)
    plan = api.BatchPlan(mats, paper_model, prec="fp16x2")
    # a batch this small (fewer first-layer tiles than two per CU) defaults to per-layer launches
    assert plan.launch_form == "layers" and plan.tile == 128
    plan.launch()
    torch.cuda.synchronize()
    ref = snapshot(plan)
    print("case batch10 autotune (tile x launch form)", flush=True)
    tile, ms = plan.autotune()
    print(f"[batch autotune] tile {tile} launch {plan.launch_form} {ms}", flush=True)
    assert plan.tile == tile and plan.launch_form in ("queue", "layers")
    assert set(ms) == {64, 128} and ms[tile] == min(ms.values())
    plan.launch()
    torch.cuda.synchronize()
    if tile == 128:
        assert_same(plan, ref, "tuned plan")
    else:
        for b in range(plan.count):
            assert float((plan.D[b] - ref[0][b]).abs().max()) < 1e-4
    plan.close()


def test_queue_launch_beside_other_work(api, paper_model):
    """The queue launch while another stream keeps the GPU busy (FP32 products): its workgroups
    then share the CUs with the other kernels and the dispatcher's round-robin starts wherever
    that work left it; the results stay bitwise equal to the per-layer launches."""
    mats = uneven_batch(48, 4700)
    plan = api.BatchPlan(mats, paper_model, prec="fp16x2")
    plan.set_launch("layers")
    plan.launch()
    torch.cuda.synchronize()
    ref = snapshot(plan)
    plan.set_launch("queue")
    side = torch.cuda.Stream()
    a = torch.randn(2048, 2048, device="cuda")
    b = torch.randn(2048, 2048, device="cuda")
    print("case queue-launch batch48 beside FP32 products on another stream", flush=True)
    for rep in range(3):
        with torch.cuda.stream(side):
            for _ in range(20):
                a = (a @ b) * 1e-3
        plan.launch()
        torch.cuda.synchronize()
        assert_same(plan, ref, f"queue launch beside other work, replay {rep}")
    plan.close()
