"""GPU parity of the Skip-SP2 / Max-SP2 path (Sec. III.A) through the C ABI against the oracle.

Tolerances:
  * scalar model and Jacobian (FP64 on the GPU) vs the oracle's evaluation and complex-step
    Jacobian: relative 1e-10 (reverse mode vs complex step, both exact up to rounding);
  * D from the 16-bit split modes vs the oracle's FP64 matrix recursion of the same model:
    ||dD||_F/N <= 1e-5 (the accuracy bar of the expansion), D exactly symmetric, traces equal to
    those of the written D up to FP64 summation (1e-9 relative).
"""
import zlib

import numpy as np
import pytest

from oracle import fermi as F
from oracle import recursion as R
from oracle import variants as V
from paper_2605_08523_amd import workloads as W
from parity import within

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def var():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_08523_amd import api, variants
    api.lib()
    return variants


def widened_skip(theta, k, K, eps, rng):
    """The oracle's k = K = 1 embedding of an MLSP2 model, widened to k skips and K accumulators
    and perturbed by eps-sized noise on every coefficient (a generic Skip-SP2 model whose
    operands stay in the range of the trained model's)."""
    s = V.mlsp2_to_skip(theta)
    n = len(s["alpha_c"])
    alpha = np.zeros((n, k))
    alpha[:, 0] = s["alpha"][:, 0]
    beta = np.zeros((n, K))
    gamma = np.zeros((n, K))
    gamma[:, 0] = s["gamma"][:, 0]
    a0 = np.zeros(K)
    a0[0] = s["a0"][0]
    m = {"kind": "skip", "k": k, "K": K, "alpha_c": s["alpha_c"] + eps * rng.normal(size=n),
         "alpha": alpha + eps * rng.normal(size=(n, k)), "beta": beta + eps * rng.normal(size=(n, K)),
         "gamma": gamma + eps * rng.normal(size=(n, K)), "a0": a0 + eps * rng.normal(size=K),
         "omega": s["omega"] * (1 + eps * rng.normal())}
    return m


def widened_max(theta, eps, rng):
    m = V.skip_to_max(V.mlsp2_to_skip(theta))
    n = len(m["delta"])
    return {"kind": "max", "delta": m["delta"] + eps * rng.normal(size=n),
            "theta": [t + eps * rng.normal(size=t.size) for t in m["theta"]],
            "gamma": m["gamma"] + eps * rng.normal(size=n + 1), "c": m["c"] + eps * rng.normal()}


def qmodel(var, m, beta0, mu0):
    if m["kind"] == "max":
        return var.QModel("max", len(m["delta"]), V.flatten(m), beta0, mu0)
    return var.QModel("skip", len(m["alpha_c"]), V.flatten(m), beta0, mu0, m["k"], m["K"])


def test_scalar_eval_and_jacobian(var):
    from paper_2605_08523_amd import models
    base = models.load("mlsp2_L22_b600_mu1third")
    rng = np.random.default_rng(11)
    y = np.linspace(0, 1, 777)
    yd = torch.from_numpy(y).cuda()
    for m in (widened_max(base.theta[:8], 1e-2, rng), widened_skip(base.theta[:8], 2, 2, 1e-2, rng),
              widened_skip(base.theta[:8], 3, 1, 1e-2, rng)):
        qm = qmodel(var, m, base.beta0, base.mu0)
        print(f"case scalar_eval {m['kind']} P={qm.coef.size}", flush=True)
        r, JT = var.variant_eval(yd, qm)
        f = V.evaluate(y, m)
        np.testing.assert_allclose(r.cpu().numpy(), f, rtol=1e-12, atol=1e-13)
        J = V.jacobian(y, m)
        scale = np.max(np.abs(J), axis=0) + 1e-300
        err = np.max(np.abs(JT.cpu().numpy().T - J) / scale)
        print(f"[{m['kind']}] max rel Jacobian diff {err:.2e}", flush=True)
        assert err <= 1e-10


CASES = [
    ("dense300", lambda: (W.random_dense(300, 21), 0.1, 0.1)),
    ("dense384_flip", lambda: (W.random_dense(384, 22), -0.35, 0.08)),
    ("banded700", lambda: (W.banded_decay(700, 8.0, 2.0, 23), 0.3, 0.2)),
    ("anderson512", lambda: (W.anderson_cubic(8, 24), 0.0, 0.05)),
]


# measured on MI355X: (||dD||_F/N, max |dD|) against the oracle's matrix recursion
MEASURED_VARIANTS = {
    ("max", "dense300"): (6.261e-07, 2.128e-05), ("max", "dense384_flip"): (4.786e-07, 1.558e-05),
    ("max", "banded700"): (1.810e-07, 1.447e-05), ("max", "anderson512"): (1.907e-07, 4.441e-06),
    ("skip11", "dense300"): (6.104e-07, 1.991e-05), ("skip11", "dense384_flip"): (3.063e-07, 1.349e-05),
    ("skip11", "banded700"): (2.489e-07, 1.246e-05), ("skip11", "anderson512"): (1.966e-07, 4.010e-06),
    ("skip22", "dense300"): (4.866e-07, 1.881e-05), ("skip22", "dense384_flip"): (3.044e-07, 1.603e-05),
    ("skip22", "banded700"): (2.221e-07, 2.246e-05), ("skip22", "anderson512"): (1.525e-07, 3.887e-06),
}


@pytest.mark.parametrize("family", ["max", "skip11", "skip22"])
@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_density_vs_oracle(var, family, name, make):
    from paper_2605_08523_amd import models
    base = models.load("mlsp2_L22_b600_mu1third")
    rng = np.random.default_rng(zlib.crc32(f"{family}/{name}".encode()))
    if family == "max":
        m = widened_max(base.theta, 1e-4, rng)
    elif family == "skip11":
        m = widened_skip(base.theta, 1, 1, 1e-4, rng)
    else:
        m = widened_skip(base.theta, 2, 2, 1e-4, rng)
    H, mu, kT = make()
    n = H.shape[0]
    print(f"case variant {family} {name} N={n}", flush=True)
    qm = qmodel(var, m, base.beta0, base.mu0)
    Hd = torch.from_numpy(H).cuda()
    D, tr, tr2, info = var.expand_density_variant(Hd, mu, kT, qm, want_info=True)
    torch.cuda.synchronize()
    Dg = D.double().cpu().numpy()
    Dref, oinfo = V.variant_density(H, mu, kT, m, base.beta0, base.mu0)
    fro = np.linalg.norm(Dg - Dref) / n
    mx = np.max(np.abs(Dg - Dref))
    print(f"[{family} {name}] |dD|_F/N={fro:.3e} max={mx:.3e} "
          f"flipped={info['flipped']}", flush=True)
    assert info["flipped"] == int(oinfo["flipped"])
    meas = MEASURED_VARIANTS[(family, name)]
    within(f"{family} {name} |dD|_F/N", fro, meas[0], cap=1e-5)
    within(f"{family} {name} max|dD|", mx, meas[1])
    assert torch.equal(D, D.T)
    assert float(tr) == pytest.approx(np.trace(Dg), rel=1e-9, abs=1e-9)
    assert float(tr2) == pytest.approx(np.sum(Dg * Dg), rel=1e-9)


@pytest.mark.parametrize("arch", ["max", "skip"])
def test_embedding_reproduces_mlsp2(var, arch):
    """The App. C embedding of the trained model through the variant path gives the MLSP2 path's
    density matrix to the precision of the split products (both against the exact D)."""
    from paper_2605_08523_amd import api, models
    base = models.load("mlsp2_L22_b600_mu1third")
    H = W.anderson_cubic(10, 31)
    n = H.shape[0]
    mu, kT = 0.1, 0.05
    qm = var.embed_mlsp2(base, arch)
    Hd = torch.from_numpy(H).cuda()
    print(f"case embedding {arch} N={n}", flush=True)
    Dv, trv, _, _ = var.expand_density_variant(Hd, mu, kT, qm)
    Dm, trm, _, _ = api.expand_density(Hd, mu, kT, base)
    torch.cuda.synchronize()
    ex = F.density(H, mu, kT)
    exact = ex["D"]
    ev = np.linalg.norm(Dv.double().cpu().numpy() - exact) / n
    em = np.linalg.norm(Dm.double().cpu().numpy() - exact) / n
    dvm = np.linalg.norm((Dv - Dm).double().cpu().numpy()) / n
    print(f"[embed {arch}] vs exact {ev:.3e} (MLSP2 path {em:.3e}), variant - MLSP2 {dvm:.3e}", flush=True)
    meas = {"max": (5.380e-08, 7.862e-08, 2.313e-04), "skip": (5.355e-08, 7.827e-08, 1.558e-04)}[arch]
    within(f"embed {arch} vs exact", ev, meas[0], cap=1e-5)
    within(f"embed {arch} variant - MLSP2", dvm, meas[1])
    print(f"[embed {arch}] |dTrD| variant {abs(float(trv) - ex['trD']):.3e}, "
          f"MLSP2 path {abs(float(trm) - ex['trD']):.3e}", flush=True)
    within(f"embed {arch} |dTrD|", abs(float(trv) - ex["trD"]), meas[2])


def test_bf16_traces_only_and_degenerate(var):
    from paper_2605_08523_amd import models
    base = models.load("mlsp2_L22_b600_mu1third")
    rng = np.random.default_rng(5)
    m = widened_skip(base.theta, 2, 1, 1e-4, rng)
    qm = qmodel(var, m, base.beta0, base.mu0)
    H = W.random_dense(256, 41)
    Hd = torch.from_numpy(H).cuda()
    print("case bf16 skip21 dense256", flush=True)
    D, tr, _, _ = var.expand_density_variant(Hd, 0.0, 0.2, qm, prec="bf16x2")
    torch.cuda.synchronize()
    Dref, _ = V.variant_density(H, 0.0, 0.2, m, base.beta0, base.mu0)
    fro = np.linalg.norm(D.double().cpu().numpy() - Dref) / 256
    print(f"[bf16] |dD|_F/N={fro:.3e}", flush=True)
    within("bf16 skip21 dense256", fro, 2.042e-05)   # BF16 split: 16 significant bits
    # H = c I: every eigenvalue maps to the same model coordinate; D = f(y) I
    c0 = 0.25
    Hc = torch.full((96, 96), 0.0, dtype=torch.float64).fill_diagonal_(c0).cuda()
    print("case degenerate cI", flush=True)
    D2, tr2, _, info = var.expand_density_variant(Hc, 0.3, 0.1, qm, want_info=True)
    torch.cuda.synchronize()
    assert info["degenerate"] == 1
    y = np.clip(base.mu0 + (0.3 - c0) / (0.1 * base.beta0), 0, 1)
    fy = float(V.evaluate(np.array(y), m))
    d2 = D2.double().cpu().numpy()
    assert np.max(np.abs(d2 - fy * np.eye(96))) <= 1e-5
    assert float(tr2) == pytest.approx(96 * fy, rel=1e-5)


def test_errors(var):
    from paper_2605_08523_amd import api, models
    base = models.load("mlsp2_L22_b600_mu1third")
    qm = var.embed_mlsp2(base, "max")
    Hd = torch.from_numpy(W.random_dense(128, 3)).cuda()
    with pytest.raises(api.FeError) as e:
        var.expand_density_variant(Hd, 0.0, 0.1, qm, prec="fp32")
    assert e.value.code == api.FE_ERR_ARG
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(api.FeError) as e:
        var.expand_density_variant(Hd, 0.0, 0.1, qm, scratch=small)
    assert e.value.code == api.FE_ERR_WORKSPACE
    wild = var.QModel("max", 2, np.array([40.0, 1.0, 0.0, 0.0, 1.0, 0.0, 0.0, 1.0, 0.0]),
                      100.0, 1 / 3)
    with pytest.raises(api.FeError) as e:
        var.expand_density_variant(Hd, 0.0, 0.1, wild)
    assert e.value.code == api.FE_ERR_RANGE
    with pytest.raises(api.FeError) as e:
        var.expand_density_variant(Hd, 100.0, 0.1, qm, want_info=True)
    assert e.value.code == api.FE_ERR_DOMAIN


def test_trainer_from_embedding(var):
    """Max-SP2 fine-tuned from the embedding of a 10-layer MLSP2 fit at (beta = 40, mu = 0.3)
    (the setting of the paper's accuracy-versus-layers figure): the fit must not lose accuracy,
    and the extra skip connections must buy accuracy at the same layer count."""
    from paper_2605_08523_amd import api, training
    th, rep0, _ = training.train_coeffs(10, 40.0, 0.3, n_points=4096, max_iter=300, tol=1e-12)
    print(f"[mlsp2 L10] grid max err {rep0['max_err_grid']:.3e}", flush=True)
    init = var.embed_mlsp2(api.make_model(th, 40.0, 0.3), "max")
    fit, rep, _ = var.train_variant(init, 40.0, 0.3, n_points=4096, max_iter=150, tol=1e-14)
    print(f"[max-sp2 L10] grid max err {rep['max_err_grid']:.3e} after {rep['iters']} iterations",
          flush=True)
    assert rep["max_err_grid"] <= rep0["max_err_grid"] * 1.0001
    assert rep["max_err_grid"] <= 0.9 * rep0["max_err_grid"]
    # the fitted model, evaluated by the oracle, has the error the trainer reports
    y = np.linspace(0, 1, 20001)
    from oracle import training as OT
    m = V.unflatten(fit.coef, V.skip_to_max(V.mlsp2_to_skip(th)))
    err = np.max(np.abs(V.evaluate(y, m) - OT.fermi_target(y, 40.0, 0.3)))
    assert err <= rep["max_err_grid"] * 1.01


def test_full_size_tail_split(var):
    """N = 4096: 528 upper tiles of 128 on 512 workgroup slots, so the squaring runs one
    data-parallel round and splits the 16 remaining tiles along K (partials added in a fixed
    order). Property check at the headline size: the Skip-SP2 embedding equals the MLSP2 path
    (itself checked against the oracle at this size) and a second run is bitwise identical."""
    from paper_2605_08523_amd import api, models
    base = models.load("mlsp2_L22_b600_mu1third")
    c = W.config_anderson_4096()
    Hd = torch.from_numpy(c["H"]).cuda()
    qm = var.embed_mlsp2(base, "skip")
    print("case tail split skip N=4096", flush=True)
    D1, tr1, _, _ = var.expand_density_variant(Hd, c["mu"], c["kT"], qm)
    D2, _, _, _ = var.expand_density_variant(Hd, c["mu"], c["kT"], qm)
    Dm, trm, _, _ = api.expand_density(Hd, c["mu"], c["kT"], base)
    torch.cuda.synchronize()
    d = float((D1 - Dm).abs().max())
    print(f"[tail split] max |D_skip - D_mlsp2| = {d:.3e}, dTr = {abs(float(tr1) - float(trm)):.3e}",
          flush=True)
    assert torch.equal(D1, D2)
    assert d < 1e-5
    assert abs(float(tr1) - float(trm)) < 1e-5 * 4096


def test_skip_trainer_from_embedding(var):
    """Skip-SP2 with two skips (k = 2, K = 1) fine-tuned from the embedding of a 10-layer MLSP2
    fit (the extra skip weights start at zero): no accuracy lost, some gained, and the oracle
    evaluates the fitted model to the error the trainer reports."""
    from paper_2605_08523_amd import api, training
    from oracle import training as OT
    th, rep0, _ = training.train_coeffs(10, 40.0, 0.3, n_points=4096, max_iter=300, tol=1e-12)
    e11 = var.embed_mlsp2(api.make_model(th, 40.0, 0.3), "skip").coef
    L = 10
    per1, per2 = 4, 5
    c = np.zeros(per2 * L + 2)
    for i in range(L):
        a_c, a0, b, g = e11[per1 * i:per1 * (i + 1)]
        c[per2 * i:per2 * (i + 1)] = (a_c, a0, 0.0, b, g)
    c[per2 * L:] = e11[per1 * L:]
    init = var.QModel("skip", L, c, 40.0, 0.3, k=2, K=1)
    fit, rep, _ = var.train_variant(init, 40.0, 0.3, n_points=4096, max_iter=100, tol=1e-14)
    print(f"[skip-sp2 k2 L10] grid max err {rep['max_err_grid']:.3e} (MLSP2 {rep0['max_err_grid']:.3e})",
          flush=True)
    assert rep["max_err_grid"] <= rep0["max_err_grid"] * 1.0001
    assert rep["max_err_grid"] < rep0["max_err_grid"]
    like = V.unflatten(c, {"kind": "skip", "k": 2, "K": 1, "alpha_c": np.zeros(L),
                           "alpha": np.zeros((L, 2)), "beta": np.zeros((L, 1)),
                           "gamma": np.zeros((L, 1)), "a0": np.zeros(1), "omega": 0.0})
    y = np.linspace(0, 1, 20001)
    err = np.max(np.abs(V.evaluate(y, V.unflatten(fit.coef, like)) - OT.fermi_target(y, 40.0, 0.3)))
    assert err <= rep["max_err_grid"] * 1.01
