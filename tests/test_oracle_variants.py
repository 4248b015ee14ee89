"""Pins of the Skip-SP2 / Max-SP2 oracle (oracle/variants.py) against hand-derived closed forms,
textbook SP2, the eigendecomposition definition of a matrix function, finite differences and
the model-family embeddings of App. C."""
import numpy as np
import pytest

from oracle import recursion as R
from oracle import variants as V


def rand_max(n, rng, scale=0.3):
    return {"kind": "max", "delta": rng.normal(0, scale, n),
            "theta": [rng.normal(0, scale, i + 1) + (np.arange(i + 1) == i) for i in range(n)],
            "gamma": rng.normal(0, scale, n + 1), "c": float(rng.normal(0, scale))}


def rand_skip(n, k, K, rng, scale=0.2):
    return {"kind": "skip", "k": k, "K": K, "alpha_c": rng.normal(0, scale, n),
            "alpha": rng.normal(0, scale, (n, k)) + np.eye(1, k), "beta": rng.normal(0, scale, (n, K)),
            "gamma": rng.normal(0, scale, (n, K)), "a0": rng.normal(0, scale, K),
            "omega": float(1.0 + rng.normal(0, scale))}


def rand_mlsp2(n, rng):
    th = np.zeros((n, 4))
    sign = rng.choice([-1.0, 1.0], n)
    th[:, 0] = sign * rng.uniform(0.7, 1.6, n)
    th[:, 1] = np.where(sign < 0, 2.0, 0.0) + rng.normal(0, 0.1, n)
    th[:, 2] = rng.normal(0, 0.05, n)
    th[:, 3] = rng.normal(0, 0.2, n)
    return th


def sym_unit(n, rng):
    Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
    lam = rng.uniform(0, 1, n)
    return (Q * lam) @ Q.T, lam, Q


def test_max_one_layer_closed_form():
    rng = np.random.default_rng(1)
    m = rand_max(1, rng)
    y = np.linspace(-0.2, 1.2, 57)
    d0, t00 = m["delta"][0], m["theta"][0][0]
    g0, g1, c = m["gamma"][0], m["gamma"][1], m["c"]
    want = c + g0 * y + g1 * (d0 ** 2 + 2 * d0 * t00 * y + t00 ** 2 * y ** 2)
    np.testing.assert_allclose(V.max_sp2(y, m), want, rtol=1e-13, atol=1e-13)


def test_max_two_layers_polynomial_coefficients():
    """f is a quartic in y; its leading coefficient is gamma_2 theta_11^2 theta_00^4 and
    f(0) = c + gamma_1 delta_0^2 + gamma_2 (delta_1 + theta_11 delta_0^2)^2 (expanded by hand).
    The y^3 coefficient 4 gamma_2 theta_11^2 theta_00^3 delta_0 + 2 gamma_2 theta_11 theta_10
    theta_00^2 separates theta_10 from theta_11."""
    rng = np.random.default_rng(2)
    m = rand_max(2, rng, scale=0.5)
    y = np.linspace(-1, 1, 41)
    coef = np.polyfit(y, V.max_sp2(y, m), 4)
    d0, d1 = m["delta"]
    t00 = m["theta"][0][0]
    t10, t11 = m["theta"][1]
    g1, g2, c = m["gamma"][1], m["gamma"][2], m["c"]
    assert coef[0] == pytest.approx(g2 * t11 ** 2 * t00 ** 4, rel=1e-9)
    assert coef[1] == pytest.approx(4 * g2 * t11 ** 2 * t00 ** 3 * d0 + 2 * g2 * t11 * t10 * t00 ** 2,
                                    rel=1e-9)
    assert coef[4] == pytest.approx(c + g1 * d0 ** 2 + g2 * (d1 + t11 * d0 ** 2) ** 2, rel=1e-9)


def test_pure_squaring_is_power_of_two():
    n = 4
    y = np.linspace(0, 1, 33)
    m = {"kind": "max", "delta": np.zeros(n),
         "theta": [np.eye(1, i + 1, i).ravel() for i in range(n)],
         "gamma": np.eye(1, n + 1, n).ravel(), "c": 0.0}
    np.testing.assert_allclose(V.max_sp2(y, m), y ** (2 ** n), rtol=1e-14, atol=1e-300)
    s = {"kind": "skip", "k": 1, "K": 1, "alpha_c": np.zeros(n), "alpha": np.ones((n, 1)),
         "beta": np.zeros((n, 1)), "gamma": np.zeros((n, 1)), "a0": np.zeros(1), "omega": 1.0}
    np.testing.assert_allclose(V.skip_sp2(y, s), y ** (2 ** n), rtol=1e-14, atol=1e-300)


def textbook_sp2(y, mu_p, L):
    """SP2 for a known mu' (the textbook recursion): x <- x^2 or x <- 2x - x^2, whichever
    moves the image of mu' closer to mu'."""
    x, m = np.array(y, dtype=np.float64), mu_p
    for _ in range(L):
        if abs(m * m - mu_p) < abs(2 * m - m * m - mu_p):
            x, m = x * x, m * m
        else:
            x, m = 2 * x - x * x, 2 * m - m * m
    return x


def test_sp2_through_the_embeddings_is_textbook_sp2():
    y = np.linspace(0, 1, 101)
    th = R.sp2_mu_coeffs(0.37, 12)
    want = textbook_sp2(y, 0.37, 12)
    skip = V.mlsp2_to_skip(th)
    np.testing.assert_allclose(V.skip_sp2(y, skip), want, rtol=0, atol=1e-11)
    np.testing.assert_allclose(V.max_sp2(y, V.skip_to_max(skip)), want, rtol=0, atol=1e-11)


def test_mlsp2_embeds_in_skip_and_max():
    rng = np.random.default_rng(3)
    th = rand_mlsp2(9, rng)
    y = np.linspace(0, 1, 201)
    want = R.mlsp2_layers(y, th)
    skip = V.mlsp2_to_skip(th)
    assert abs(skip["gamma"][0, 0] - th[0, 3]) == 0.0       # the x_0 term survives
    np.testing.assert_allclose(V.skip_sp2(y, skip), want, rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(V.max_sp2(y, V.skip_to_max(skip)), want, rtol=1e-10, atol=1e-10)
    X, _, _ = sym_unit(12, rng)
    np.testing.assert_allclose(V.skip_sp2(X, skip), R.mlsp2_layers(X, th), atol=1e-10)


def test_paper_model_embeds():
    from paper_2605_08523_amd import models
    m = models.load("mlsp2_L26_b1500_mu1third")
    y = np.linspace(0, 1, 2001)
    want = R.mlsp2_layers(y, m.theta)
    skip = V.mlsp2_to_skip(m.theta)
    np.testing.assert_allclose(V.skip_sp2(y, skip), want, atol=1e-9)
    np.testing.assert_allclose(V.max_sp2(y, V.skip_to_max(skip)), want, atol=1e-9)


def test_skip_embeds_in_max():
    rng = np.random.default_rng(4)
    for k, K in [(1, 1), (2, 1), (2, 2), (3, 2)]:
        s = rand_skip(7, k, K, rng)
        y = np.linspace(-0.1, 1.1, 151)
        np.testing.assert_allclose(V.max_sp2(y, V.skip_to_max(s)), V.skip_sp2(y, s),
                                   rtol=1e-11, atol=1e-12)


def test_matrix_form_is_the_matrix_function():
    rng = np.random.default_rng(5)
    X, lam, Q = sym_unit(16, rng)
    for m in (rand_max(5, rng), rand_skip(5, 2, 2, rng)):
        F = V.evaluate(X, m)
        want = (Q * V.evaluate(lam, m)) @ Q.T
        np.testing.assert_allclose(F, want, atol=1e-11)
        np.testing.assert_allclose(F, F.T, atol=1e-12)


def test_parameter_counts():
    for n, k in [(10, 1), (26, 1), (8, 3)]:
        assert V.skip_param_count(n, k, 1) == (1 + k + 2) * n + 2    # the paper's (1+k+2K)n+2
    rng = np.random.default_rng(6)
    s = rand_skip(6, 2, 2, rng)
    assert V.flatten(s).size == V.skip_param_count(6, 2, 2)
    m = rand_max(6, rng)
    assert V.flatten(m).size == V.max_param_count(6) == 6 * 7 // 2 + 2 * 6 + 2
    for like in (s, m):
        back = V.unflatten(V.flatten(like), like)
        np.testing.assert_array_equal(V.flatten(back), V.flatten(like))


def test_complex_step_jacobian():
    rng = np.random.default_rng(7)
    y = np.linspace(0, 1, 23)
    for m in (rand_max(4, rng), rand_skip(4, 2, 1, rng)):
        J = V.jacobian(y, m)
        v = V.flatten(m)
        h = 1e-6
        for p in range(v.size):
            vp, vm = v.copy(), v.copy()
            vp[p] += h
            vm[p] -= h
            fd = (V.evaluate(y, V.unflatten(vp, m)) - V.evaluate(y, V.unflatten(vm, m))) / (2 * h)
            np.testing.assert_allclose(J[:, p], fd, rtol=1e-6, atol=1e-8)
    # closed forms for one Max-SP2 layer
    m = rand_max(1, rng)
    J = V.jacobian(y, m)
    z = m["delta"][0] + m["theta"][0][0] * y
    np.testing.assert_allclose(J[:, 0], 2 * m["gamma"][1] * z, rtol=1e-13)        # d/d delta_0
    np.testing.assert_allclose(J[:, 1], 2 * m["gamma"][1] * z * y, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(J[:, 2], np.ones_like(y))                           # d/dc
    np.testing.assert_allclose(J[:, 3], y, atol=0)                                 # d/d gamma_0
    np.testing.assert_allclose(J[:, 4], z * z, rtol=1e-13)                         # d/d gamma_1


@pytest.mark.parametrize("mu_frac", [0.3, 0.7])
def test_variant_density_matches_mlsp2(mu_frac):
    from oracle import fermi as F
    from paper_2605_08523_amd import models
    rng = np.random.default_rng(8)
    n = 40
    A = rng.normal(size=(n, n))
    H = (A + A.T) / (2 * np.sqrt(n)) + np.diag(rng.uniform(-1, 1, n))
    lam = np.linalg.eigvalsh(H)
    mu = float(lam[0] + mu_frac * (lam[-1] - lam[0]))
    m = models.load("mlsp2_L26_b1500_mu1third")
    D1, info = R.mlsp2_density(H, mu, 0.1, m.theta, m.beta0, m.mu0)
    D2, _ = V.variant_density(H, mu, 0.1, V.skip_to_max(V.mlsp2_to_skip(m.theta)), m.beta0, m.mu0)
    np.testing.assert_allclose(D2, D1, atol=1e-9)
    assert np.linalg.norm(D2 - F.density(H, mu, 0.1)["D"]) / n < 1e-6
