"""Training-side definitions in FP64: targets, sample points, model Jacobian.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The coefficients are fitted on scalars in the model coordinate y in [0, 1]
(Sec. III.A: the layers act on eigenvalues only). The Fermi target is
g(y) = 1 / (1 + exp(beta0 (mu0 - y))) and the entropy target is the entropy
function of that occupation (Sec. III.B). Levenberg-Marquardt minimises the
sum of squared residuals r_k = P(y_k; theta) - target(y_k) (Sec. III.C).

The fitted coefficients themselves are not unique (different optimisers and
starting points land in different minima), so the trainer's output has no
oracle value: parity unpinned for theta itself. What is checked is the
Jacobian (against central finite differences of ``forward``) and the error
level the fitted model reaches on a dense grid.
"""
from __future__ import annotations

import math

import numpy as np


def fermi_target(y, beta0: float, mu0: float):
    """g(y) = 1/(1 + exp(beta0 (mu0 - y))) evaluated without overflow."""
    u = beta0 * (mu0 - np.asarray(y, dtype=np.float64))
    out = np.empty_like(u)
    pos = u >= 0
    e = np.exp(-u[pos])
    out[pos] = e / (1.0 + e)
    out[~pos] = 1.0 / (1.0 + np.exp(u[~pos]))
    return out


def fermi_target_slope(y, beta0: float, mu0: float):
    """g'(y) = beta0 g (1 - g)."""
    g = fermi_target(y, beta0, mu0)
    return beta0 * g * (1.0 - g)


def entropy_target(y, beta0: float, mu0: float):
    """s(y) = -g ln g - (1 - g) ln(1 - g) with g = fermi_target (Eq. entropy)."""
    u = np.abs(beta0 * (mu0 - np.asarray(y, dtype=np.float64)))
    t = np.exp(-u)
    return np.log1p(t) + u * t / (1.0 + t)


def sample_points(n: int, beta0: float, mu0: float, law: str = "deriv", grid: int = 1 << 20):
    """n deterministic sample points on [0, 1] drawn as quantiles of a density (Sec. III.C).

    law = "uniform": p proportional to 1;
    law = "deriv":   p proportional to 1 + |g'|;
    law = "arclen":  p proportional to sqrt(1 + g'^2).
    The k-th point is the (k + 1/2)/n quantile of p, found on a fine grid with
    the trapezoid rule and linear interpolation of the cumulative density.
    """
    t = np.linspace(0.0, 1.0, grid + 1)
    gp = fermi_target_slope(t, beta0, mu0)
    if law == "uniform":
        p = np.ones_like(t)
    elif law == "deriv":
        p = 1.0 + np.abs(gp)
    elif law == "arclen":
        p = np.sqrt(1.0 + gp * gp)
    else:
        raise ValueError(law)
    cdf = np.concatenate([[0.0], np.cumsum(0.5 * (p[1:] + p[:-1]) * np.diff(t))])
    cdf /= cdf[-1]
    q = (np.arange(n) + 0.5) / n
    return np.interp(q, cdf, t)


def forward(y, theta, kind: str = "fermi", mu0: float = 1.0 / 3.0, alpha: float = 1.0):
    """Scalar model output.

    kind = "fermi":   P(y) = A_n + x_n with x_0 = y (Eq. mlsp2).
    kind = "entropy": 4 ln2 u (1 - u), u = A_n + x_n, x_0 = alpha (y - mu0) + mu0
                      (Eq. entropy expansion and its output layer).
    """
    y = np.asarray(y, dtype=np.float64)
    x = y if kind == "fermi" else alpha * (y - mu0) + mu0
    A = np.zeros_like(x)
    for a, b, c, d in np.asarray(theta, dtype=np.float64):
        A = A + d * x
        x = a * x * x + b * x + c
    u = A + x
    if kind == "fermi":
        return u
    return 4.0 * math.log(2.0) * u * (1.0 - u)


def jacobian(y, theta, kind: str = "fermi", mu0: float = 1.0 / 3.0, alpha: float = 1.0):
    """d output / d theta by forward-mode sensitivities (chain rule through each layer).

    Returns (out, J) with J of shape (len(y), 4L), columns ordered layer-major
    (a_0, b_0, c_0, d_0, a_1, ...). For layer i:
      dx_{i+1}/d(a_i, b_i, c_i) = (x_i^2, x_i, 1),
      dx_{i+1}/d theta_j = (2 a_i x_i + b_i) dx_i/d theta_j for earlier j,
      dA_{i+1}/d d_i = x_i,  dA_{i+1}/d theta_j = dA_i/d theta_j + d_i dx_i/d theta_j.
    """
    th = np.asarray(theta, dtype=np.float64)
    L = th.shape[0]
    y = np.asarray(y, dtype=np.float64)
    x = y.copy() if kind == "fermi" else alpha * (y - mu0) + mu0
    A = np.zeros_like(x)
    dx = np.zeros((y.size, 4 * L))
    dA = np.zeros((y.size, 4 * L))
    for i, (a, b, c, d) in enumerate(th):
        dA = dA + d * dx
        dA[:, 4 * i + 3] += x
        A = A + d * x
        slope = 2.0 * a * x + b
        dx = dx * slope[:, None]
        dx[:, 4 * i + 0] += x * x
        dx[:, 4 * i + 1] += x
        dx[:, 4 * i + 2] += 1.0
        x = a * x * x + b * x + c
    u = A + x
    du = dA + dx
    if kind == "fermi":
        return u, du
    k = 4.0 * math.log(2.0)
    return k * u * (1.0 - u), (k * (1.0 - 2.0 * u))[:, None] * du


def max_model_error(theta, beta0: float, mu0: float, kind: str = "fermi", alpha: float = 1.0,
                    n: int = 2_000_001):
    """max over a uniform grid of [0, 1] of |model - target| in FP64."""
    y = np.linspace(0.0, 1.0, n)
    tgt = fermi_target(y, beta0, mu0) if kind == "fermi" else entropy_target(y, beta0, mu0)
    return float(np.max(np.abs(forward(y, theta, kind, mu0, alpha) - tgt)))


def max_abs_state(theta, kind: str = "fermi", mu0: float = 1.0 / 3.0, alpha: float = 1.0,
                  n: int = 100001) -> float:
    """Largest |x_i| over all layer states for inputs y on a uniform grid of [0, 1].

    The split modes hold each state in 16-bit halves, so this is the operand range a model
    needs (Eq. emulated matmul)."""
    y = np.linspace(0.0, 1.0, n)
    x = y if kind == "fermi" else alpha * (y - mu0) + mu0
    m = float(np.max(np.abs(x)))
    for a, b, c, _ in np.asarray(theta, dtype=np.float64):
        x = a * x * x + b * x + c
        m = max(m, float(np.max(np.abs(x))))
    return m


def _forward_complex(y, theta, kind, mu0, alpha):
    """``forward`` with complex coefficients allowed (for the complex step)."""
    x = np.asarray(y, dtype=np.float64).astype(np.complex128)
    if kind != "fermi":
        x = alpha * (x - mu0) + mu0
    A = np.zeros_like(x)
    for a, b, c, d in np.asarray(theta):
        A = A + d * x
        x = a * x * x + b * x + c
    u = A + x
    return u if kind == "fermi" else 4.0 * math.log(2.0) * u * (1.0 - u)


def second_directional(y, theta, v, kind: str = "fermi", mu0: float = 1.0 / 3.0,
                       alpha: float = 1.0, h: float = 1e-4):
    """d^2/dt^2 of the model output at theta + t v, t = 0 (the geodesic acceleration's input in
    Levenberg-Marquardt, Sec. III.C). The first t-derivative is exact by the complex step,
    f'(t) = Im f(theta + (t + i e) v) / e; the second is its central difference with step h
    (relative error O(h^2))."""
    th = np.asarray(theta, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64).reshape(th.shape)
    e = 1e-30

    def d1(t):
        return np.imag(_forward_complex(y, th + (t + 1j * e) * v, kind, mu0, alpha)) / e
    return (d1(h) - d1(-h)) / (2.0 * h)
