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


def rescale(H: np.ndarray, mu: float, kT: float, beta0: float, mu0: float):
    """Affine map of H onto the model's coordinate (Sec. IV.1).

    Steps, in the paper's order:
      1. Gershgorin bounds eps_min, eps_max.
      2. H' = (eps_max I - H)/(eps_max - eps_min)      (Eq. H')
         mu' = (eps_max - mu)/(eps_max - eps_min)     (Eq. mu')
         beta' = (eps_max - eps_min) / kT            (Eq. beta')
      3. If mu' > 1/2: H' <- I - H', mu' <- 1 - mu'  (Eq. flip; strict inequality)
      4. beta_max = min(mu0/mu', (1 - mu0)/(1 - mu')) beta0 (Eq. conditions);
         beta' > beta_max is clamped to beta_max and reported.
      5. X0 = (beta'/beta0)(H' - mu' I) + mu0 I        (Eq. H0)

    Returns (X0, info). ``info`` holds the bounds, mu', beta', beta_max, the
    flip and clamp flags and the affine form X0 = scale H + shift I.
    """
    if not (kT > 0.0) or not np.isfinite(kT):
        raise DomainError("kT must be positive")
    H = np.asarray(H, dtype=np.float64)
    n = H.shape[0]
    I = np.eye(n)
    emin, emax = gershgorin(H)
    width = emax - emin
    if width <= 1e-300 * max(1.0, abs(emax)):
        # H = c I: constant model coordinate (see the module docstring).
        c = float(H[0, 0])
        y = mu0 + (mu - c) / (kT * beta0)
        clamped = not (0.0 <= y <= 1.0)
        y = min(1.0, max(0.0, y))
        info = dict(emin=emin, emax=emax, mu_p=float('nan'), beta_p=float('inf'),
                    beta_max=float('nan'), flipped=False, clamped=clamped,
                    degenerate=True, scale=0.0, shift=y)
        return y * I, info
    if not (emin < mu < emax):
        raise DomainError("mu must lie strictly inside the Gershgorin bounds")
    Hp = (emax * I - H) / width
    mu_p = (emax - mu) / width
    beta_p = width / kT
    flipped = mu_p > 0.5
    if flipped:
        Hp = I - Hp
        mu_p = 1.0 - mu_p
    beta_max = min(mu0 / mu_p, (1.0 - mu0) / (1.0 - mu_p)) * beta0
    clamped = beta_p > beta_max
    if clamped:
        beta_p = beta_max
    X0 = (Hp - mu_p * I) * (beta_p / beta0) + mu0 * I
    r = beta_p / beta0
    if flipped:
        scale, shift = r / width, r * (-emin / width - mu_p) + mu0
    else:
        scale, shift = -r / width, r * (emax / width - mu_p) + mu0
    info = dict(emin=emin, emax=emax, mu_p=mu_p, beta_p=beta_p, beta_max=beta_max,
                flipped=flipped, clamped=clamped, degenerate=False,
                scale=scale, shift=shift)
    return X0, info


def mlsp2_layers(X, theta, return_history: bool = False):
    """MLSP2 layers (Eq. mlsp2; Alg. 1 without its opening flip, see module docstring).

    For each layer (a, b, c, d) = theta_i:  A <- A + d X;  X <- a X^2 + b X + c I.
    Output A + X (Eq. mlsp2-output). Works on scalars/arrays (elementwise
    squaring) when X is not 2-D square, and on symmetric matrices (X^2 = X @ X)
    otherwise.
    """
    X = np.asarray(X, dtype=np.float64)
    matrix = X.ndim == 2 and X.shape[0] == X.shape[1]
    I = np.eye(X.shape[0]) if matrix else 1.0
    A = np.zeros_like(X)
    hist = [X]
    for a, b, c, d in np.asarray(theta, dtype=np.float64):
        A = A + d * X
        X2 = X @ X if matrix else X * X
        X = a * X2 + b * X + c * I
        hist.append(X)
    out = A + X
    return (out, hist) if return_history else out


def mlsp2_density(H, mu, kT, theta, beta0, mu0):
    """D from Alg. 2 (density part) in FP64: rescale, MLSP2 layers, undo the flip.

    Returns (D, info). If the rescale flipped the spectrum the result is I - (A + X)
    (Eq. flip).
    """
    X0, info = rescale(H, mu, kT, beta0, mu0)
    P = mlsp2_layers(X0, theta)
    n = P.shape[0]
    D = np.eye(n) - P if info["flipped"] else P
    return D, info


def entropy_layers(Y0, theta_s):
    """Entropy expansion layers on Y0 (Eq. entropy expansion): returns U = A_n + Y_n."""
    return mlsp2_layers(Y0, theta_s)


def entropy_expansion(H, mu, kT, theta_s, beta0, mu0, alpha):
    """S from Alg. 2 (entropy part) in FP64.

    Y0 = alpha X0 + (1 - alpha) mu0 I; L_S layers with Theta; U = A_S + Y;
    S = 4 ln2 (Tr U - sum_ij U_ij^2) (Eq. entropy expansion-s traced).
    The entropy is symmetric under the flip, so no flip correction is needed.
    """
    X0, info = rescale(H, mu, kT, beta0, mu0)
    n = X0.shape[0]
    Y0 = alpha * X0 + (1.0 - alpha) * mu0 * np.eye(n)
    U = entropy_layers(Y0, theta_s)
    S = 4.0 * math.log(2.0) * (np.trace(U) - np.sum(U * U))
    return float(S), info


def entropy_scalar(y, theta_s, mu0, alpha):
    """Scalar entropy model s~(y) = 4 ln2 u (1 - u), u = layers(alpha (y - mu0) + mu0)."""
    y0 = alpha * (np.asarray(y, dtype=np.float64) - mu0) + mu0
    u = mlsp2_layers(y0, theta_s)
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
