"""Seeded synthetic Hamiltonians for the Fermi-operator expansion workloads.

This module only draws matrices and scalar parameters from seeded random number
generators (``numpy.random.default_rng``). It holds none of the expansion's
arithmetic: no Fermi function, no rescaling, no recursion. Both the CPU oracle
tests and the GPU path take their inputs from here.

The paper benchmarks on random dense symmetric matrices (Sec. V.D) and on sets
of uniformly spaced eigenvalues in the unit interval (Sec. V.E, Table I). The
families below are the workloads the benchmarks and tests run on; every one is
a dense row-major float64 array.
"""
from __future__ import annotations

import numpy as np


def random_dense(n: int, seed: int) -> np.ndarray:
    """Dense symmetric H = diag(d) + (A + A^T) / (2 sqrt(n)).

    A_ij ~ N(0, 1) (drawn first, n x n), then on-site d_i ~ U[-1, 1] (drawn
    second). Spectrum roughly [-2, 2] for large n.
    """
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((n, n))
    d = rng.uniform(-1.0, 1.0, n)
    h = (a + a.T) / (2.0 * np.sqrt(n))
    h[np.diag_indices(n)] += d
    return h


def anderson_cubic(L: int, seed: int, t: float = -1.0, w: float = 1.0) -> np.ndarray:
    """3D tight-binding Hamiltonian on an L^3 periodic cubic lattice, stored dense.

    Site index n = (x*L + y)*L + z; hopping t between nearest neighbours
    (periodic boundaries); Anderson on-site disorder uniform in [-w, w].
    For L = 2 the +1 and -1 neighbours coincide and their hoppings add.
    """
    rng = np.random.default_rng(seed)
    n = L ** 3
    h = np.zeros((n, n))
    h[np.diag_indices(n)] = rng.uniform(-w, w, n)
    idx = np.arange(n)
    x, y, z = idx // (L * L), (idx // L) % L, idx % L
    for dx, dy, dz in ((1, 0, 0), (0, 1, 0), (0, 0, 1)):
        j = (((x + dx) % L) * L + (y + dy) % L) * L + (z + dz) % L
        np.add.at(h, (idx, j), t)
        np.add.at(h, (j, idx), t)
    return h


def banded_decay(n: int, xi: float, onsite: float, seed: int) -> np.ndarray:
    """Dense symmetric H with h_ij = g_ij exp(-|i-j|/xi), g_ij ~ N(0,1).

    The upper triangle of g is drawn and mirrored; the diagonal is replaced by
    on-site values uniform in [-onsite, onsite] (drawn after g).
    """
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n, n))
    d = rng.uniform(-onsite, onsite, n)
    i = np.arange(n)
    decay = np.exp(-np.abs(i[:, None] - i[None, :]) / xi)
    h = np.triu(g, 1) * decay
    h = h + h.T
    h[np.diag_indices(n)] = d
    return h


def uniform_appendix(n: int, seed: int) -> np.ndarray:
    """H = U + U^T with U_ij ~ U(0, 1): the random family of the paper's Appendix A self-test."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(0.0, 1.0, (n, n))
    return u + u.T


def gapped_spectrum(n: int, n_below: int, gap: float, seed: int):
    """Q diag(lam) Q^T with exactly ``n_below`` eigenvalues in [-1, -gap/2] and the rest in [gap/2, 1].

    Returns (H, lam). Used for the zero-temperature (projector) checks.
    """
    rng = np.random.default_rng(seed)
    lo = rng.uniform(-1.0, -gap / 2, n_below)
    hi = rng.uniform(gap / 2, 1.0, n - n_below)
    lam = np.concatenate([lo, hi])
    q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    h = (q * lam) @ q.T
    h = 0.5 * (h + h.T)
    return h, lam


def uniform_eigenvalues(n: int = 2048) -> np.ndarray:
    """n uniformly spaced normalized energies on [0, 1] (the test spectrum of Sec. V.E)."""
    return np.linspace(0.0, 1.0, n)


# ---------------------------------------------------------------------------
# The benchmark configurations
# ---------------------------------------------------------------------------

def config_small_dense(seed: int = 0):
    """N=128 dense random symmetric H (family ``random_dense``), kT=0.1.

    mu is not drawn here: the half-filling chemical potential is a property of
    the spectrum and is found by the test or benchmark that needs it.
    """
    return dict(H=random_dense(128, seed), kT=0.1, n_target=64.0, seed=seed)


def config_anderson_4096(seed: int = 1):
    """16^3 periodic Anderson lattice (N=4096), hopping -1, disorder U[-1,1], kT=0.05, mu=0."""
    return dict(H=anderson_cubic(16, seed), kT=0.05, mu=0.0, seed=seed)


def batch_items(count: int = 1024, base_seed: int = 2000, n_lo: int = 64, n_hi: int = 768,
                with_mu: bool = True):
    """The uneven batch: item b uses seed base_seed + b.

    N_b ~ U{n_lo..n_hi}; h_ij = g_ij exp(-|i-j|/8); on-site U[-2, 2];
    kT_b ~ U[0.01, 0.3]; mu_b ~ U(lambda_min, lambda_max) of the true spectrum
    (eigenvalues from LAPACK, which is plain linear algebra, not the method).
    """
    items = []
    for b in range(count):
        rng = np.random.default_rng(base_seed + b)
        n = int(rng.integers(n_lo, n_hi + 1))
        kT = float(rng.uniform(0.01, 0.3))
        u = float(rng.uniform(0.0, 1.0))
        h = banded_decay(n, 8.0, 2.0, base_seed + 100000 + b)
        item = dict(H=h, n=n, kT=kT, u=u, seed=base_seed + b)
        if with_mu:
            lam = np.linalg.eigvalsh(h)
            item["mu"] = float(lam[0] + u * (lam[-1] - lam[0]))
        items.append(item)
    return items


def config_large_banded(n: int = 16384, seed: int = 4):
    """N=16384 dense symmetric, exponential off-diagonal decay xi=32, on-site U[-1,1], kT=0.02."""
    return dict(H=banded_decay(n, 32.0, 1.0, seed), kT=0.02, filling=0.4, seed=seed)
