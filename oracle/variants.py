"""Skip-SP2 and Max-SP2 (Sec. III.A), their matrix forms, the embeddings between the model
families (App. C) and the complex-step Jacobian of the scalar models, in FP64 on the CPU.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Models are plain dicts of numpy arrays:

* Max-SP2 with n layers (Eq. maxsp2, Alg. maxsp2-1d):
  ``{"kind": "max", "delta": (n,), "theta": [array of length i + 1 for i < n],
  "gamma": (n + 1,), "c": float}``.
  Layer i (0 <= i < n): x_{i+1} = (delta_i + sum_{j <= i} theta_{i,j} x_j)^2.
  Output: f = c + sum_{i=0}^{n} gamma_i x_i.
* Skip-SP2 with n layers, k skips, K accumulators (Sec. III.A.3):
  ``{"kind": "skip", "k": k, "K": K, "alpha_c": (n,), "alpha": (n, k), "beta": (n, K),
  "gamma": (n, K), "a0": (K,), "omega": float}``.
  Layer i: x_{i+1} = (alpha_c_i + sum_{j < k} alpha_{i,j} x_{i-j} + sum_l beta_{i,l} A_{i,l})^2,
  then A_{i+1,l} = A_{i,l} + gamma_{i,l} x_i, with A_{0,l} = a0_l.
  Output: f = omega x_n + sum_l A_{n,l}.

Readings (the paper is ambiguous or garbled here):

* x_0 is the model coordinate: the affine rescale already performs the SP2 flip
  (x_0 = 1 - x in the paper's unit-interval form), as for MLSP2.
* Max-SP2 output: Eq. maxsp2 accumulates gamma_i x_i from i = 0 and adds gamma_n x_n, while
  Alg. maxsp2-1d starts from a constant gamma_0 and adds gamma_i x_i for i >= 1. The output
  here has both a constant c and every x_i term; each printed form is a special case.
* Skip-SP2: terms x_{i-j} with i - j < 0 are absent. The accumulators start at constants a0_l
  (App. C's embedding needs a constant A_0). The printed output x_n + sum_l A_{n,l} has unit
  weight on x_n; App. C's embedding of MLSP2 needs the weight a_{n-1} there, so the weight omega
  is a parameter. With K = 1 the count (1 + k + 2K) n + 2 matches the paper's.
* App. C's map Skip-SP2 -> Max-SP2 prints alpha_{i,n-j} for j >= n - k; read with the layer
  index: theta_{i,j} gets alpha_{i,i-j} for i - k < j <= i, and sum_l beta_{i,l} gamma_{j,l}
  for j < i (A_{i,l} holds gamma_{j,l} x_j for j < i only).
"""
from __future__ import annotations

import numpy as np


def _is_matrix(X):
    return X.ndim == 2 and X.shape[0] == X.shape[1]


def _sq(Z, matrix):
    return Z @ Z if matrix else Z * Z


def max_sp2(X, model, return_history: bool = False):
    """Max-SP2 (Eq. maxsp2, Alg. maxsp2-1d) on a scalar/array (elementwise) or a symmetric
    matrix. Complex input is allowed (complex-step derivatives)."""
    X = np.asarray(X)
    matrix = _is_matrix(X)
    I = np.eye(X.shape[0]) if matrix else 1.0
    xs = [X]
    n = len(model["delta"])
    for i in range(n):
        Z = model["delta"][i] * I
        for j in range(i + 1):
            Z = Z + model["theta"][i][j] * xs[j]
        xs.append(_sq(Z, matrix))
    f = model["c"] * I
    for i in range(n + 1):
        f = f + model["gamma"][i] * xs[i]
    return (f, xs) if return_history else f


def skip_sp2(X, model):
    """Skip-SP2 (Sec. III.A.3) on a scalar/array or a symmetric matrix."""
    X = np.asarray(X)
    matrix = _is_matrix(X)
    I = np.eye(X.shape[0]) if matrix else 1.0
    k, K = model["k"], model["K"]
    n = len(model["alpha_c"])
    xs = [X]
    A = [model["a0"][l] * I for l in range(K)]
    for i in range(n):
        Z = model["alpha_c"][i] * I
        for j in range(k):
            if i - j >= 0:
                Z = Z + model["alpha"][i][j] * xs[i - j]
        for l in range(K):
            Z = Z + model["beta"][i][l] * A[l]
        x_next = _sq(Z, matrix)
        A = [A[l] + model["gamma"][i][l] * xs[i] for l in range(K)]
        xs.append(x_next)
    f = model["omega"] * xs[n]
    for l in range(K):
        f = f + A[l]
    return f


def mlsp2_to_skip(theta):
    """MLSP2 -> Skip-SP2 with k = 1, K = 1 (App. C).

    With x~_0 = x_0 and x~_{i+1} = (x_i + b_i/(2a_i))^2, the MLSP2 state is
    x_i = a_{i-1} x~_i + e_{i-1} (i >= 1), e_i = c_i - b_i^2/(4 a_i). Hence
    alpha_{0,0} = 1, alpha_c_0 = b_0/(2a_0); alpha_{i,0} = a_{i-1}, alpha_c_i = e_{i-1} + b_i/(2a_i);
    gamma_0 = d_0, gamma_i = d_i a_{i-1}; omega = a_{n-1};
    a0 = sum_{i=1}^{n-1} d_i e_{i-1} + e_{n-1}; beta = 0. Requires every a_i != 0.
    """
    th = np.asarray(theta, dtype=np.float64)
    n = th.shape[0]
    a, b, c, d = th[:, 0], th[:, 1], th[:, 2], th[:, 3]
    if np.any(a == 0.0):
        raise ValueError("the embedding needs a_i != 0 in every layer")
    e = c - b * b / (4.0 * a)
    alpha = np.zeros((n, 1))
    alpha_c = np.zeros(n)
    gamma = np.zeros((n, 1))
    alpha[0, 0] = 1.0
    alpha_c[0] = b[0] / (2.0 * a[0])
    gamma[0, 0] = d[0]
    for i in range(1, n):
        alpha[i, 0] = a[i - 1]
        alpha_c[i] = e[i - 1] + b[i] / (2.0 * a[i])
        gamma[i, 0] = d[i] * a[i - 1]
    a0 = float(np.sum(d[1:] * e[:-1]) + e[-1])
    return {"kind": "skip", "k": 1, "K": 1, "alpha_c": alpha_c, "alpha": alpha,
            "beta": np.zeros((n, 1)), "gamma": gamma, "a0": np.array([a0]), "omega": float(a[-1])}


def skip_to_max(m):
    """Skip-SP2 -> Max-SP2 (App. C, with the index reading of the module docstring).

    A_{i,l} = a0_l + sum_{j < i} gamma_{j,l} x_j, so layer i's operand is
    alpha_c_i + sum_l beta_{i,l} a0_l + sum_{j < i} (sum_l beta_{i,l} gamma_{j,l}) x_j
    + sum_{i-k < j <= i} alpha_{i,i-j} x_j; the output is
    sum_l a0_l + sum_{j < n} (sum_l gamma_{j,l}) x_j + omega x_n.
    """
    k, K = m["k"], m["K"]
    n = len(m["alpha_c"])
    beta, gamma, a0 = np.asarray(m["beta"]), np.asarray(m["gamma"]), np.asarray(m["a0"])
    delta = np.array([m["alpha_c"][i] + float(beta[i] @ a0) for i in range(n)])
    theta = []
    for i in range(n):
        row = np.zeros(i + 1)
        for j in range(i):
            row[j] += float(beta[i] @ gamma[j])
        for s in range(k):
            if i - s >= 0:
                row[i - s] += m["alpha"][i][s]
        theta.append(row)
    g = np.zeros(n + 1)
    g[:n] = gamma.sum(axis=1)
    g[n] = m["omega"]
    return {"kind": "max", "delta": delta, "theta": theta, "gamma": g, "c": float(a0.sum())}


def max_param_count(n: int) -> int:
    """delta (n) + theta (n(n+1)/2) + gamma (n+1) + c."""
    return n + n * (n + 1) // 2 + n + 2


def skip_param_count(n: int, k: int, K: int) -> int:
    """(1 + k + 2K) n per-layer coefficients + K constants a0 + omega."""
    return (1 + k + 2 * K) * n + K + 1


def flatten(model):
    """Coefficient vector in the order: per layer i [delta_i, theta_{i,0..i}] then [c, gamma_0..n]
    (Max-SP2); per layer i [alpha_c_i, alpha_{i,0..k-1}, beta_{i,1..K}, gamma_{i,1..K}] then
    [a0_1..K, omega] (Skip-SP2)."""
    out = []
    if model["kind"] == "max":
        for i in range(len(model["delta"])):
            out.append(model["delta"][i])
            out.extend(model["theta"][i])
        out.append(model["c"])
        out.extend(model["gamma"])
    else:
        for i in range(len(model["alpha_c"])):
            out.append(model["alpha_c"][i])
            out.extend(model["alpha"][i])
            out.extend(model["beta"][i])
            out.extend(model["gamma"][i])
        out.extend(model["a0"])
        out.append(model["omega"])
    return np.array(out, dtype=np.complex128 if np.iscomplexobj(np.array(out)) else np.float64)


def unflatten(v, like):
    """Inverse of flatten for a model with the structure of ``like``."""
    v = list(v)
    pos = 0

    def take(m):
        nonlocal pos
        r = v[pos:pos + m]
        pos += m
        return r

    if like["kind"] == "max":
        n = len(like["delta"])
        delta, theta = [], []
        for i in range(n):
            delta.append(take(1)[0])
            theta.append(np.array(take(i + 1)))
        c = take(1)[0]
        gamma = np.array(take(n + 1))
        return {"kind": "max", "delta": np.array(delta), "theta": theta, "gamma": gamma, "c": c}
    k, K = like["k"], like["K"]
    n = len(like["alpha_c"])
    ac, al, be, ga = [], [], [], []
    for i in range(n):
        ac.append(take(1)[0])
        al.append(take(k))
        be.append(take(K))
        ga.append(take(K))
    a0 = np.array(take(K))
    om = take(1)[0]
    return {"kind": "skip", "k": k, "K": K, "alpha_c": np.array(ac), "alpha": np.array(al),
            "beta": np.array(be), "gamma": np.array(ga), "a0": a0, "omega": om}


def evaluate(y, model):
    return max_sp2(y, model) if model["kind"] == "max" else skip_sp2(y, model)


def jacobian(y, model, h: float = 1e-30):
    """d f(y_k) / d p for every coefficient p (flatten order), by the complex step
    f'(p) = Im f(p + i h) / h, exact to rounding for these polynomial recursions."""
    y = np.asarray(y, dtype=np.float64)
    v = flatten(model).astype(np.float64)
    J = np.zeros((y.size, v.size))
    for p in range(v.size):
        w = v.astype(np.complex128)
        w[p] += 1j * h
        J[:, p] = np.imag(evaluate(y.astype(np.complex128), unflatten(w, model))) / h
    return J


def variant_density(H, mu, kT, model, beta0, mu0):
    """D for a Skip-SP2 or Max-SP2 model: the rescale of Sec. IV.1 (shared with MLSP2), the
    matrix recursion, I - f if the spectrum was flipped (Eq. flip)."""
    from .recursion import rescale
    X0, info = rescale(H, mu, kT, beta0, mu0)
    f = evaluate(X0, model)
    n = X0.shape[0]
    return (np.eye(n) - f if info["flipped"] else f), info
