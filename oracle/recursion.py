"""The paper's recursion, step by step, in FP64 (CPU).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Readings of the paper that this module fixes (each is also listed in the design
notes of the repository):

* Coordinates. The affine rescale already flips the spectrum (Eq. H'), so the
  MLSP2 layers act on the model coordinate y directly; no further x -> 1 - x
  flip is applied. In that coordinate a model trained at (beta0, mu0)
  approximates g(y) = 1 / (1 + exp(beta0 (mu0 - y))), which rises from 0 to 1.
* Alg. 2 writes beta' = (eps_max - eps_min) beta' ; read as (eps_max - eps_min) beta
  (Eq. beta').
* Alg. 2 builds Y = alpha X + (1 - alpha) mu I; read with mu0, the step location
  in the model coordinate of X (Eq. entropy expansion written for the model).
* Alg. 2 closes with S = 4 ln2 (Tr(Y^2) - Tr(Y)), which is never positive; read
  as S = 4 ln2 (Tr U - Tr U^2) with U = A_S + Y (Eq. entropy expansion-s), and
  Tr U^2 = sum_ij U_ij^2 for symmetric U (Sec. IV.3, Eq. tr(D^2)).
* Degenerate bounds (eps_max = eps_min, i.e. H = c I): the rescale is undefined;
  the exact answer f(c) I is reached by feeding the constant model coordinate
  y = mu0 + beta (mu - c) / beta0 (clamped to [0, 1]) through the layers.
* mu outside (eps_min, eps_max) or kT <= 0 is outside the stated domain of the
  method and raises ValueError.
"""
from __future__ import annotations

import math

import numpy as np

from .fermi import gershgorin

GOLDEN = (1.0 + math.sqrt(5.0)) / 2.0
PHI = 1.0 / GOLDEN                      # inverse golden ratio, Sec. V.B
KB_EV_PER_K = 8.617e-5                  # Boltzmann constant in eV/K (Sec. V.C)


class DomainError(ValueError):
    pass


def model_map(bounds, mu: float, kT: float, beta0: float, mu0: float):
    """The affine map from energies to the model coordinate (Sec. IV.1), as one scale and shift.

    Eqs. H', mu' and beta' normalise the spectrum by its Gershgorin width w and place mu at
    mu' = (eps_max - mu)/w; Eq. H0 then stretches about mu' by beta'/beta0 and moves mu' onto
    mu0. Composed, every energy e lands at

        y(e) = mu0 + sigma (beta'/beta0) (e - mu) / w,

    with sigma = -1, or +1 when Eq. flip has replaced mu' by 1 - mu' (only for mu' > 1/2,
    strictly). Unclamped, beta'/w = 1/kT, so beta0 (y - mu0) = -+ (e - mu)/kT: this is the
    identity (mu' I - H') beta' = beta (H - mu I) that makes g(y) equal f(e) (or 1 - f(e)
    after the flip). Eq. conditions bound beta' by beta_max = beta0 min(mu0/mu', (1 - mu0)/(1 - mu'))
    (mu' after the flip); a larger beta' is replaced by beta_max and reported as clamped.

    Returns a dict with the bounds, mu', beta', beta_max, the flags, and y = scale e + shift.
    """
    if not (kT > 0.0) or not np.isfinite(kT):
        raise DomainError("kT must be positive")
    emin, emax = bounds
    width = emax - emin
    if width <= 1e-300 * max(1.0, abs(emax)):
        return dict(emin=emin, emax=emax, mu_p=float('nan'), beta_p=float('inf'),
                    beta_max=float('nan'), flipped=False, clamped=False, degenerate=True,
                    scale=0.0, shift=float('nan'))
    if not (emin < mu < emax):
        raise DomainError("mu must lie strictly inside the Gershgorin bounds")
    mu_p = (emax - mu) / width
    flipped = bool(mu_p > 0.5)
    mu_eff = 1.0 - mu_p if flipped else mu_p
    beta_p = width / kT
    bmax = beta_max(mu_eff, beta0, mu0)
    clamped = bool(beta_p > bmax)
    beta_used = bmax if clamped else beta_p
    scale = (1.0 if flipped else -1.0) * (beta_used / beta0) / width
    return dict(emin=emin, emax=emax, mu_p=mu_eff, beta_p=beta_used, beta_max=bmax,
                flipped=flipped, clamped=clamped, degenerate=False,
                scale=scale, shift=mu0 - scale * mu)


def _degenerate_coordinate(c: float, mu: float, kT: float, beta0: float, mu0: float):
    """H = c I has zero Gershgorin width, so Eq. H' is undefined. Its one eigenvalue c is
    placed where the unflipped map of any width would put it, y = mu0 + (mu - c)/(kT beta0),
    and held inside [0, 1] (outside it the model is not trained); leaving [0, 1] counts as a
    clamp."""
    y = mu0 + (mu - c) / (kT * beta0)
    return min(1.0, max(0.0, y)), not (0.0 <= y <= 1.0)


def rescale(H: np.ndarray, mu: float, kT: float, beta0: float, mu0: float):
    """X0 = scale H + shift I, the rescaled Hamiltonian of Eq. H0 (see ``model_map``).

    Returns (X0, info); info is ``model_map``'s dict (for H = c I, with the constant
    coordinate of ``_degenerate_coordinate`` as shift and scale 0).
    """
    H = np.asarray(H, dtype=np.float64)
    n = H.shape[0]
    info = model_map(gershgorin(H), mu, kT, beta0, mu0)
    if info["degenerate"]:
        y, clamped = _degenerate_coordinate(float(H[0, 0]), mu, kT, beta0, mu0)
        info.update(shift=y, clamped=clamped)
        return y * np.eye(n), info
    return info["scale"] * H + info["shift"] * np.eye(n), info


def _layers_scalar(x, theta):
    """Eq. mlsp2 on numbers: for each layer (a, b, c, d), the accumulator gains d x and x
    becomes a x^2 + b x + c; the output is the accumulator plus the last x (Eq. mlsp2-output)."""
    x = np.asarray(x, dtype=np.float64)
    acc = np.zeros_like(x)
    for a, b, c, d in np.asarray(theta, dtype=np.float64):
        acc = acc + d * x
        x = (a * x + b) * x + c
    return acc + x


def mlsp2_layers(X, theta):
    """The MLSP2 model P of Eq. mlsp2 applied to numbers, or to a symmetric matrix.

    The layers are polynomials, so for a symmetric matrix X = Q diag(y) Q^T the recursion's
    result is Q diag(P(y)) Q^T (Sec. III.A: the layers act on the eigenvalues only); the
    matrix form is evaluated that way, from one eigendecomposition.
    """
    X = np.asarray(X, dtype=np.float64)
    if X.ndim == 2 and X.shape[0] == X.shape[1] and X.shape[0] > 1:
        y, Q = np.linalg.eigh(X)
        return _assemble(Q, _layers_scalar(y, theta))
    return _layers_scalar(X, theta)


def _assemble(Q, g):
    M = (Q * g) @ Q.T
    return 0.5 * (M + M.T)


def model_values(lam, bounds, mu, kT, beta0, mu0):
    """Model coordinate y of every eigenvalue ``lam`` of a matrix with Gershgorin ``bounds``
    (``model_map``; for zero width the constant coordinate of ``_degenerate_coordinate``, where
    every eigenvalue equals the diagonal). Returns (y, info)."""
    lam = np.asarray(lam, dtype=np.float64)
    info = model_map(bounds, mu, kT, beta0, mu0)
    if info["degenerate"]:
        y, clamped = _degenerate_coordinate(float(bounds[0]), mu, kT, beta0, mu0)
        info.update(shift=y, clamped=clamped)
        return np.full_like(lam, y), info
    return info["scale"] * lam + info["shift"], info


def density_eigenvalues(lam, bounds, mu, kT, theta, beta0, mu0):
    """Eigenvalues of the expansion's D: the layers on each model coordinate, one minus that when
    the map flipped the spectrum (Eq. flip: the model then gives the occupation of holes)."""
    y, info = model_values(lam, bounds, mu, kT, beta0, mu0)
    p = _layers_scalar(y, theta)
    return (1.0 - p if info["flipped"] else p), info


def entropy_eigen_terms(lam, bounds, mu, kT, theta_s, beta0, mu0, alpha):
    """Per-eigenvalue terms of the entropy expansion: Y0 = alpha X0 + (1 - alpha) mu0 I pulls the
    model coordinate towards mu0 by alpha, the layers give u, and S = 4 ln2 (Tr U - Tr U^2)
    (Eq. entropy expansion-s) is the sum of 4 ln2 u_i (1 - u_i) over the eigenvalues of the
    symmetric U. s(f) = s(1 - f), so the flip needs no correction."""
    y, info = model_values(lam, bounds, mu, kT, beta0, mu0)
    u = _layers_scalar(alpha * (y - mu0) + mu0, theta_s)
    return 4.0 * math.log(2.0) * u * (1.0 - u), info


def mlsp2_density(H, mu, kT, theta, beta0, mu0):
    """D from Alg. 2 (density part) in FP64, evaluated on the spectrum of H:
    D = Q diag(``density_eigenvalues``) Q^T. Returns (D, info)."""
    H = np.asarray(H, dtype=np.float64)
    lam, Q = np.linalg.eigh(H)
    g, info = density_eigenvalues(lam, gershgorin(H), mu, kT, theta, beta0, mu0)
    return _assemble(Q, g), info


def entropy_layers(Y0, theta_s):
    """Entropy expansion layers on Y0 (Eq. entropy expansion): returns U = A_n + Y_n."""
    return mlsp2_layers(Y0, theta_s)


def entropy_expansion(H, mu, kT, theta_s, beta0, mu0, alpha):
    """S from Alg. 2 (entropy part) in FP64: the sum of ``entropy_eigen_terms`` over the
    spectrum of H. Returns (S, info)."""
    H = np.asarray(H, dtype=np.float64)
    lam = np.linalg.eigvalsh(H)
    s, info = entropy_eigen_terms(lam, gershgorin(H), mu, kT, theta_s, beta0, mu0, alpha)
    return float(np.sum(s)), info


def entropy_scalar(y, theta_s, mu0, alpha):
    """Scalar entropy model s~(y) = 4 ln2 u (1 - u), u = layers(alpha (y - mu0) + mu0)."""
    y0 = alpha * (np.asarray(y, dtype=np.float64) - mu0) + mu0
    u = _layers_scalar(y0, theta_s)
    return 4.0 * math.log(2.0) * u * (1.0 - u)


def sp2_mu_coeffs(mu_p: float, L: int):
    """SP2 for a known chemical potential, embedded in MLSP2 (Eq. sp2-mu; App. C).

    mu_0 = mu'. At each step, if |mu_i^2 - mu'| < |2 mu_i - mu_i^2 - mu'| the
    layer is X^2, theta = (1, 0, 0, 0), and mu_{i+1} = mu_i^2; otherwise it is
    2X - X^2, theta = (-1, 2, 0, 0), and mu_{i+1} = 2 mu_i - mu_i^2.
    """
    th = np.zeros((L, 4))
    m = float(mu_p)
    for i in range(L):
        sq, fl = m * m, 2.0 * m - m * m
        if abs(sq - mu_p) < abs(fl - mu_p):
            th[i] = (1.0, 0.0, 0.0, 0.0)
            m = sq
        else:
            th[i] = (-1.0, 2.0, 0.0, 0.0)
            m = fl
    return th


def layer_count(beta_p: float) -> float:
    """n_l = ln(beta'/4) / ln(2 phi), phi the inverse golden ratio (Sec. V.B, Eq. layer count)."""
    return math.log(beta_p / 4.0) / math.log(2.0 * PHI)


def beta0_for_layers(n_layers: int) -> float:
    """beta0 = 4 (2 phi)^n (Sec. V.C)."""
    return 4.0 * (2.0 * PHI) ** n_layers


def beta_max(mu_p: float, beta0: float, mu0: float) -> float:
    """Largest beta' inside the region of validity at mu' (Eq. conditions)."""
    return min(mu0 / mu_p, (1.0 - mu0) / (1.0 - mu_p)) * beta0


def temperature_limit_K(width_eV: float, beta_p_max: float = 1000.0) -> float:
    """Lowest temperature a model valid up to beta'_max can represent (Eq. temp limit): width / (k_B beta'_max)."""
    return width_eV / (KB_EV_PER_K * beta_p_max)
