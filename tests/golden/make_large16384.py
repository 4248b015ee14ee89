"""Writes ``large16384_oracle.npz``: the oracle's reference values for the N = 16384 solve.

The input is the seeded large single-solve family (exponential off-diagonal decay xi = 32,
on-site U[-1, 1], seed 4; kT = 0.02, mu for a 40% filling). One FP64 eigendecomposition by the
oracle (LAPACK dsyevd, tens of minutes on a few cores, ~10 GB of memory) gives:

* ``lam``: every eigenvalue of H;
* ``mu``: the oracle's chemical potential for Tr D = 0.4 N (bisection on the eigenvalues);
* ``bounds``: the oracle's Gershgorin bounds;
* ``exact_*``: Tr D, sum_ij D_ij^2 and S of the exact Fermi-Dirac density matrix (Sec. II.A,
  Eq. entropy-matrix), eight seeded rows of D (``rows``), and D v for four seeded probe
  vectors (``probes``, columns of V);
* ``<model>_*``: the same for the recursion of each listed model in FP64 (Alg. 2 evaluated on
  the spectrum of H), including its entropy expansion with the Fermi coefficients reused at
  alpha = 0.842704 (Sec. III.B);
* ``<entropy model>_S``: S from the entropy expansion of each listed entropy model
  (theta_entropy, its own alpha).

Only the oracle and the seeded input generator are called. Run from the repository root:
``python tests/golden/make_large16384.py``.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import fermi as F  # noqa: E402
from oracle import recursion as R  # noqa: E402
from paper_2605_08523_amd import workloads as W  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "large16384_oracle.npz")
MODELS = ("mlsp2_L40_b1e4_mu1third", "mlsp2_L36_b1e4_mu0p5")
ENTROPY_MODELS = ("entropy_L40_b1e4_mu1third",)
ALPHA_REUSE = 0.842704
N_ROWS, N_PROBES = 8, 4


def _theta(name):
    with open(os.path.join(ROOT, "paper_2605_08523_amd", "models", name + ".json")) as f:
        d = json.load(f)
    return (np.asarray(d["theta"], dtype=np.float64).reshape(-1, 4), float(d["beta0"]),
            float(d["mu0"]), float(d.get("alpha", 1.0)))


def main():
    t0 = time.time()
    c = W.config_large_banded()
    H, kT = c["H"], c["kT"]
    n = H.shape[0]
    bounds = F.gershgorin(H)
    print(f"bounds {bounds} ({time.time() - t0:.0f} s)", flush=True)
    lam, Q = F.eig(H)
    del H
    print(f"eigh done ({time.time() - t0:.0f} s)", flush=True)
    mu = F.mu_for_filling(lam, 0.4 * n, kT)
    rng = np.random.default_rng(16384)
    rows = np.sort(rng.choice(n, N_ROWS, replace=False))
    V = rng.standard_normal((n, N_PROBES))
    QtV = Q.T @ V
    Qr = Q[rows]

    def pack(prefix, g):
        return {f"{prefix}_rows": (Qr * g) @ Q.T, f"{prefix}_probes": Q @ (g[:, None] * QtV),
                f"{prefix}_trD": np.float64(np.sum(g)), f"{prefix}_trD2": np.float64(np.sum(g * g))}

    f = F.fermi(lam, mu, kT)
    out = dict(lam=lam, mu=np.float64(mu), kT=np.float64(kT), bounds=np.asarray(bounds),
               rows=rows, V=V, exact_S=np.float64(F.entropy_fn(lam, mu, kT).sum()))
    out.update(pack("exact", f))
    for name in ENTROPY_MODELS:
        theta, beta0, mu0, alpha = _theta(name)
        s, info = R.entropy_eigen_terms(lam, bounds, mu, kT, theta, beta0, mu0, alpha)
        out[f"{name}_S"] = np.float64(np.sum(s))
        out[f"{name}_clamped"] = np.int64(info["clamped"])
        print(f"{name}: S {np.sum(s):.9f} (exact {out['exact_S']:.9f})", flush=True)
    for name in MODELS:
        theta, beta0, mu0, _ = _theta(name)
        g, info = R.density_eigenvalues(lam, bounds, mu, kT, theta, beta0, mu0)
        s, _ = R.entropy_eigen_terms(lam, bounds, mu, kT, theta, beta0, mu0, ALPHA_REUSE)
        out.update(pack(name, g))
        out[f"{name}_S"] = np.float64(np.sum(s))
        out[f"{name}_beta_p"] = np.float64(info["beta_p"])
        out[f"{name}_clamped"] = np.int64(info["clamped"])
        print(f"{name}: beta' {info['beta_p']:.1f} clamped {info['clamped']} "
              f"max|g - f| {np.max(np.abs(g - f)):.3e}", flush=True)
    out["alpha_reuse"] = np.float64(ALPHA_REUSE)
    np.savez(OUT, **out)
    print(f"mu {mu:.12f} TrD {out['exact_trD']:.6f} S {out['exact_S']:.6f} -> {OUT} "
          f"({time.time() - t0:.0f} s)", flush=True)


if __name__ == "__main__":
    main()
