"""Pins for the plain definitions in oracle.fermi (CPU only)."""
import json
import math
import os

import numpy as np
import pytest

from oracle import fermi as F
from paper_2605_08523_amd import workloads as W

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def g(key):
    return GOLD[key]["value"]


# --- Fermi function -------------------------------------------------------

def test_fermi_half_at_mu_and_particle_hole_symmetry():
    e = np.linspace(-3, 3, 1001)
    assert F.fermi(np.array([0.7]), 0.7, 0.05)[0] == 0.5
    np.testing.assert_allclose(F.fermi(0.2 + e, 0.2, 0.3) + F.fermi(0.2 - e, 0.2, 0.3), 1.0, atol=1e-15)


def test_fermi_extremes_do_not_overflow_and_are_monotone():
    e = np.array([-1e6, -50.0, 0.0, 50.0, 1e6])
    f = F.fermi(e, 0.0, 1e-3)
    assert np.all(np.isfinite(f)) and f[0] == 1.0 and f[-1] == 0.0
    x = np.linspace(-1, 1, 10001)
    assert np.all(np.diff(F.fermi(x, 0.1, 0.02)) <= 0)


def test_fermi_small_u_taylor():
    # f(u) = 1/2 - u/4 + u^3/48 - ... (series of the logistic function)
    u = np.array([1e-3, -2e-3, 5e-4])
    np.testing.assert_allclose(F.fermi(u, 0.0, 1.0), 0.5 - u / 4 + u ** 3 / 48, atol=1e-15)


# --- entropy function -----------------------------------------------------

def test_entropy_at_mu_is_ln2_and_vanishes_far_away():
    assert abs(F.entropy_fn(np.array([0.3]), 0.3, 0.1)[0] - math.log(2)) < 1e-15
    assert F.entropy_fn(np.array([100.0]), 0.0, 0.1)[0] < 1e-300
    assert np.all(F.entropy_fn(np.linspace(-5, 5, 1001), 0.0, 0.2) >= 0)


def test_entropy_energy_form_equals_occupation_form():
    # two independent routes: s(u) in the energy variable vs -f ln f - (1-f) ln(1-f)
    e = np.linspace(-0.5, 0.5, 2001)
    s1 = F.entropy_fn(e, 0.05, 0.07)
    s2 = F.entropy_of_occupation(F.fermi(e, 0.05, 0.07))
    np.testing.assert_allclose(s1, s2, atol=2e-15)


def test_entropy_small_u_taylor():
    # s(u) = ln2 - u^2/8 + u^4/192 - ...
    u = np.array([1e-3, 3e-3])
    np.testing.assert_allclose(F.entropy_fn(u, 0.0, 1.0), math.log(2) - u ** 2 / 8 + u ** 4 / 192, atol=1e-15)


def test_table1_row1_m1_polynomial():
    """Eq. approx-s with m=1, c = 4 ln 2: max error over f and the relative Tr error (Table I row 1)."""
    f = np.linspace(0, 1, 2_000_001)
    err = np.max(np.abs(F.entropy_of_occupation(f) - 4 * math.log(2) * f * (1 - f)))
    assert abs(err - g("table1_m1_max_err")) < 1e-4          # printed to 3 digits (7.558e-2 -> 7.55e-2)
    lam = W.uniform_eigenvalues(int(g("table1_n_eigs")))
    beta, mu = g("table1_beta"), g("table1_mu")
    fo = F.fermi(lam, mu, 1 / beta)
    S = F.entropy_fn(lam, mu, 1 / beta).sum()
    Sa = (4 * math.log(2) * fo * (1 - fo)).sum()
    assert abs(abs(S - Sa) / S - g("table1_m1_rel_err")) < 5e-4


def test_alpha_ansatz_minimax_and_local():
    """Sec. III.B: alpha = 1/sqrt(2 ln 2) matches s''(mu); alpha = 0.842704 minimises the max error (1.24e-3, Table I row 4)."""
    assert abs(1 / math.sqrt(2 * math.log(2)) - g("alpha_local")) < 1e-6
    x = np.linspace(-4, 4, 1_600_001)
    kT = 0.1

    def maxerr(a):
        return np.max(np.abs(F.entropy_fn(x, 0.0, kT) - F.ansatz_entropy(x, 0.0, kT, a)))

    a0 = g("alpha_minimax")
    e0 = maxerr(a0)
    assert abs(e0 - g("table1_theta_fermi_max_err")) < 5e-6
    assert maxerr(a0 - 5e-4) > e0 and maxerr(a0 + 5e-4) > e0
    # local alpha: second derivatives at mu agree (central differences, h small)
    h = 1e-3
    al = g("alpha_local")
    d2s = (F.entropy_fn(np.array([h]), 0, 1) - 2 * math.log(2) + F.entropy_fn(np.array([-h]), 0, 1)) / h ** 2
    a = F.ansatz_entropy(np.array([-h, 0.0, h]), 0.0, 1.0, al)
    d2a = (a[0] - 2 * a[1] + a[2]) / h ** 2
    assert abs(d2s[0] - d2a) < 1e-6 and abs(d2s[0] + 0.25) < 1e-6   # s''(mu) = -1/4 in u


# --- Gershgorin -----------------------------------------------------------

def test_gershgorin_diagonal_is_exact_and_bounds_contain_spectrum():
    d = np.array([0.3, -1.2, 2.5, 0.0])
    assert F.gershgorin(np.diag(d)) == (-1.2, 2.5)
    for seed in range(5):
        H = W.random_dense(50, seed)
        lo, hi = F.gershgorin(H)
        lam = np.linalg.eigvalsh(H)
        assert lo <= lam[0] and lam[-1] <= hi
        # brute force over rows
        r = [sum(abs(H[i, j]) for j in range(50) if j != i) for i in range(50)]
        assert lo == pytest.approx(min(H[i, i] - r[i] for i in range(50)), abs=1e-13)
        assert hi == pytest.approx(max(H[i, i] + r[i] for i in range(50)), abs=1e-13)


def test_gershgorin_anderson_lattice():
    H = W.anderson_cubic(4, 3)
    d = np.diag(H)
    lo, hi = F.gershgorin(H)
    assert lo == pytest.approx(d.min() - 6) and hi == pytest.approx(d.max() + 6)
    assert np.count_nonzero(H - np.diag(d)) == 6 * 64


# --- density matrix ---------------------------------------------------------

def test_density_of_diagonal_H():
    d = np.array([-0.4, 0.1, 0.35, 0.9])
    out = F.density(np.diag(d), 0.3, 0.05)
    np.testing.assert_allclose(out["D"], np.diag(1 / (np.exp((d - 0.3) / 0.05) + 1)), atol=1e-15)


def test_density_2x2_closed_form():
    a, b, c, mu, kT = 0.3, 0.2, -0.1, 0.05, 0.08
    m, r = (a + c) / 2, math.hypot((a - c) / 2, b)
    lp, lm = m + r, m - r
    # eigenvector for lp: (b, lp - a)
    v = np.array([b, lp - a]) / math.hypot(b, lp - a)
    w = np.array([-v[1], v[0]])
    fp, fm = 1 / (math.exp((lp - mu) / kT) + 1), 1 / (math.exp((lm - mu) / kT) + 1)
    Dref = fp * np.outer(v, v) + fm * np.outer(w, w)
    out = F.density(np.array([[a, b], [b, c]]), mu, kT)
    np.testing.assert_allclose(out["D"], Dref, atol=1e-14)
    assert out["trD"] == pytest.approx(fp + fm, abs=1e-14)


def test_density_trace_commutation_affine_covariance():
    H = W.random_dense(40, 7)
    out = F.density(H, 0.1, 0.05)
    D = out["D"]
    assert out["trD"] == pytest.approx(np.trace(D), abs=1e-12)
    assert out["trD2"] == pytest.approx(np.sum(D * D), abs=1e-12)
    np.testing.assert_allclose(D @ H, H @ D, atol=1e-12)
    p, q = 2.5, -0.7
    D2 = F.density(p * H + q * np.eye(40), p * 0.1 + q, p * 0.05)["D"]
    np.testing.assert_allclose(D2, D, atol=1e-12)


def test_density_zero_temperature_is_projector():
    H, lam = W.gapped_spectrum(60, 23, 0.2, 11)
    D = F.density(H, 0.0, 1e-4)["D"]
    np.testing.assert_allclose(D @ D, D, atol=1e-12)
    assert np.trace(D) == pytest.approx(23, abs=1e-10)


def test_dD_dmu_against_finite_difference():
    H = W.random_dense(30, 5)
    mu, kT, h = 0.05, 0.1, 1e-5
    fd = (F.density(H, mu + h, kT)["D"] - F.density(H, mu - h, kT)["D"]) / (2 * h)
    np.testing.assert_allclose(F.dD_dmu(H, mu, kT), fd, atol=1e-8)


def test_mu_for_filling():
    lam = np.linalg.eigvalsh(W.random_dense(128, 0))
    mu = F.mu_for_filling(lam, 64.0, 0.1)
    assert F.fermi(lam, mu, 0.1).sum() == pytest.approx(64.0, abs=1e-9)


def test_free_energy_diagonal_closed_form():
    """Diagonal H: G = 2 sum_i [f_i (h_i - mu) - kT s_i] with f, s written out directly."""
    h = np.array([-1.3, -0.2, 0.05, 0.9, 2.0])
    mu, kT = 0.1, 0.07
    f = 1.0 / (1.0 + np.exp((h - mu) / kT))
    s = -f * np.log(f) - (1 - f) * np.log(1 - f)
    G = 2.0 * np.sum(f * (h - mu) - kT * s)
    assert F.free_energy(np.diag(h), mu, kT) == pytest.approx(G, rel=1e-13, abs=1e-14)


def test_free_energy_matrix_form_and_mu_derivative():
    """The eigenvalue form equals the matrix form 2 Tr[D (H - mu I)] - 2 kT S (Sec. III.B), and
    dG/dmu = -2 Tr D (d/dmu of f (x - mu) - kT s(x) is -f), by central differences."""
    rng = np.random.default_rng(11)
    A = rng.standard_normal((40, 40))
    H = (A + A.T) / 8.0
    mu, kT = 0.07, 0.15
    d = F.density(H, mu, kT)
    G_matrix = 2.0 * np.sum(d["D"] * H) - 2.0 * mu * d["trD"] - 2.0 * kT * d["S"]
    G = F.free_energy(H, mu, kT)
    assert G == pytest.approx(G_matrix, rel=1e-12, abs=1e-12)
    h = 1e-5
    dG = (F.free_energy(H, mu + h, kT) - F.free_energy(H, mu - h, kT)) / (2 * h)
    assert dG == pytest.approx(-2.0 * d["trD"], rel=1e-8)


def test_free_energy_zero_temperature_limit():
    """kT -> 0 with a gap at mu: G -> 2 sum_{lam < mu} (lam - mu) (the entropy term vanishes)."""
    lam = np.array([-1.0, -0.6, -0.2, 0.3, 0.8])
    H = np.diag(lam)
    G0 = 2.0 * np.sum(lam[lam < 0.0] - 0.0)
    assert F.free_energy(H, 0.0, 1e-4) == pytest.approx(G0, abs=1e-12)


def test_observable_is_twice_the_frobenius_product():
    rng = np.random.default_rng(12)
    H = rng.standard_normal((6, 6)); H = H + H.T
    A = rng.standard_normal((6, 6)); A = A + A.T
    D = F.density(H, 0.0, 0.5)["D"]
    assert F.observable(D, A) == pytest.approx(2.0 * np.trace(D @ A), rel=1e-13)
    # <H> at mu is the internal energy part of G: G = <H> - 2 mu Tr D - 2 kT S
    d = F.density(H, 0.0, 0.5)
    assert F.free_energy(H, 0.0, 0.5) == pytest.approx(
        F.observable(d["D"], H) - 2 * 0.0 * d["trD"] - 2 * 0.5 * d["S"], rel=1e-12)
