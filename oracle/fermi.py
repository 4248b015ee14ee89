"""Plain definitions: Fermi-Dirac occupations, entropy, and the exact density matrix.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Everything is FP64 NumPy; the eigendecomposition is LAPACK ``dsyevd`` through
``numpy.linalg.eigh``.
"""
from __future__ import annotations

import numpy as np

LN2 = float(np.log(2.0))


def fermi(e, mu: float, kT: float):
    """Fermi-Dirac occupation f(e) = 1 / (exp((e - mu)/kT) + 1) (Sec. II.A, Eq. FD_Func).

    Evaluated without overflow: for u = (e - mu)/kT >= 0 use exp(-u)/(1 + exp(-u)),
    otherwise 1/(1 + exp(u)).
    """
    u = (np.asarray(e, dtype=np.float64) - mu) / kT
    out = np.empty_like(u)
    pos = u >= 0
    ep = np.exp(-u[pos])
    out[pos] = ep / (1.0 + ep)
    out[~pos] = 1.0 / (1.0 + np.exp(u[~pos]))
    return out


def entropy_of_occupation(f):
    """s(f) = -f ln f - (1 - f) ln(1 - f) with 0 ln 0 = 0 (Sec. III.B, Eq. entropy)."""
    f = np.asarray(f, dtype=np.float64)
    out = np.zeros_like(f)
    m = (f > 0) & (f < 1)
    g = f[m]
    out[m] = -g * np.log(g) - (1.0 - g) * np.log1p(-g)
    return out


def entropy_fn(e, mu: float, kT: float):
    """Entropy function s(e) of an energy, s = -f ln f - (1-f) ln(1-f) with f = fermi(e).

    Written in u = (e - mu)/kT to avoid ln 0: with t = exp(-|u|),
    s = ln(1 + t) + |u| t / (1 + t). (Substituting f = 1/(1+e^u) into Eq. entropy.)
    """
    u = np.abs((np.asarray(e, dtype=np.float64) - mu) / kT)
    t = np.exp(-u)
    return np.log1p(t) + u * t / (1.0 + t)


def gershgorin(H: np.ndarray):
    """Spectral bounds from Gershgorin's circle theorem (Sec. IV.1; Alg. 2, first step).

    Every eigenvalue lies in some disc centred at a diagonal entry h_ii with radius
    r_i = sum_{j != i} |h_ij|, so the union of the discs' real intervals,
    [min_i (h_ii - r_i), max_i (h_ii + r_i)], holds the spectrum. Walked row by row.
    """
    H = np.asarray(H, dtype=np.float64)
    lo, hi = np.inf, -np.inf
    for i in range(H.shape[0]):
        row = H[i]
        centre = float(row[i])
        radius = float(np.sum(np.abs(row))) - abs(centre)
        lo = min(lo, centre - radius)
        hi = max(hi, centre + radius)
    return float(lo), float(hi)


def eig(H: np.ndarray):
    """FP64 eigendecomposition H = V diag(lam) V^T (LAPACK dsyevd via numpy)."""
    return np.linalg.eigh(np.asarray(H, dtype=np.float64))


def density_from_eig(lam, V, mu: float, kT: float):
    """D = V diag(f(lam)) V^T, symmetrized (Sec. II.A: D = [exp(beta(H - mu I)) + I]^-1)."""
    f = fermi(lam, mu, kT)
    D = (V * f) @ V.T
    return 0.5 * (D + D.T), f


def density(H: np.ndarray, mu: float, kT: float):
    """Exact finite-temperature density matrix and its scalars.

    Returns a dict with D, trD = sum_i f_i, trD2 = sum_ij D_ij^2 (= sum_i f_i^2),
    S = sum_i s(lambda_i) (Eq. entropy-matrix per spin channel, k_B = 1), and the
    eigenvalues.
    """
    lam, V = eig(H)
    D, f = density_from_eig(lam, V, mu, kT)
    return dict(D=D, trD=float(f.sum()), trD2=float(np.sum(f * f)),
                S=float(entropy_fn(lam, mu, kT).sum()), lam=lam, f=f)


def entropy(H: np.ndarray, mu: float, kT: float) -> float:
    """S = sum_i s(lambda_i) = -Tr[D ln D + (I - D) ln(I - D)] (Eq. entropy-matrix, k_B = 1)."""
    lam = np.linalg.eigvalsh(np.asarray(H, dtype=np.float64))
    return float(entropy_fn(lam, mu, kT).sum())


def free_energy(H: np.ndarray, mu: float, kT: float) -> float:
    """Electronic free energy with the spin factor, G = 2 Tr[g(H)] (Sec. III.B, Eq. free_energy):
    g(x) = f(x)(x - mu) - kT s(x), summed over the eigenvalues (k_B = 1, T = kT)."""
    lam = np.linalg.eigvalsh(np.asarray(H, dtype=np.float64))
    f = fermi(lam, mu, kT)
    return float(2.0 * np.sum(f * (lam - mu) - kT * entropy_fn(lam, mu, kT)))


def observable(D: np.ndarray, A: np.ndarray) -> float:
    """Expectation value <A> = 2 Tr(D A) of a symmetric observable (Sec. II.A, Eq. observables)."""
    return float(2.0 * np.sum(np.asarray(D, dtype=np.float64) * np.asarray(A, dtype=np.float64)))


def mu_for_filling(lam, n_target: float, kT: float, tol: float = 1e-12) -> float:
    """Chemical potential with sum_i f(lambda_i; mu) = n_target, by bisection.

    sum_i f is strictly increasing in mu, so bisection on [min lam - 50 kT,
    max lam + 50 kT] converges; stops when the bracket is below ``tol``.
    """
    lam = np.asarray(lam, dtype=np.float64)
    lo, hi = float(lam.min()) - 50 * kT, float(lam.max()) + 50 * kT
    while hi - lo > tol * max(1.0, abs(lo), abs(hi)):
        mid = 0.5 * (lo + hi)
        if fermi(lam, mid, kT).sum() < n_target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def dD_dmu(H: np.ndarray, mu: float, kT: float):
    """Derivative of D with respect to mu: beta D (I - D).

    From f = 1/(1 + exp(beta(e - mu))), df/dmu = beta f (1 - f) > 0, so the sign
    is positive (Sec. IV.3 prints the same expression with a leading minus; the
    derivative of an increasing function of mu is positive).
    """
    lam, V = eig(H)
    f = fermi(lam, mu, kT)
    g = f * (1.0 - f) / kT
    return (V * g) @ V.T


def ansatz_entropy(x, mu: float, kT: float, alpha: float):
    """alpha-rescaled m=1 entropy ansatz (Sec. III.B): 4 ln2 f(y)(1 - f(y)), y = alpha(x - mu) + mu."""
    y = alpha * (np.asarray(x, dtype=np.float64) - mu) + mu
    f = fermi(y, mu, kT)
    return 4.0 * LN2 * f * (1.0 - f)
