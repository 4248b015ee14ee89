"""Train bank models with the library's own trainer (fe_train_coeffs) and store them as JSON.

Usage (on a machine with the GPU and the built library):
    python -m paper_2605_08523_amd.models.train_bank OUTDIR SPEC ...
with SPEC one of
    L:BETA0[:MU0[:ITERS]]                    a Fermi model from the SP2 initial guess
    S:INIT:ALPHA[:ITERS]                     an entropy model (theta_entropy) from the stored
                                             Fermi model INIT (a bank name or a JSON path;
                                             same L, beta0, mu0)
e.g. ``python -m paper_2605_08523_amd.models.train_bank out 20:300 22:600``. Fermi models are
fitted to g(y) = 1/(1 + exp(beta0 (mu0 - y))) (Sec. III.C) on 8192 points sampled as quantiles of
1 + |g'|, and written as ``mlsp2_L{L}_b{beta0}_mu...``. Entropy models are fitted to
s(g(y)) = -g ln g - (1 - g) ln(1 - g) through the entropy expansion (layers on
alpha (y - mu0) + mu0, output 4 ln2 u (1 - u); Sec. III.B, Eqs. entropy expansion and -s) from
the Fermi coefficients, as the paper builds theta_entropy, and written as ``entropy_...``. The
device-measured maximum error on the trainer's check grid goes into the provenance; the oracle
re-measures every stored model in the tests.
"""
from __future__ import annotations

import os
import sys
import time


def _name(L: int, beta0: float, mu0: float) -> str:
    b = f"{beta0:g}".replace("+", "").replace("10000", "1e4")
    m = "mu1third" if abs(mu0 - 1.0 / 3.0) < 1e-12 else f"mu{mu0:g}".replace(".", "p")
    return f"mlsp2_L{L}_b{b}_{m}"


def main(argv):
    import torch
    from paper_2605_08523_amd import models, training
    if not torch.cuda.is_available():
        raise SystemExit("train_bank needs a GPU")
    torch.cuda.init()
    outdir = os.path.abspath(argv[0])
    os.makedirs(outdir, exist_ok=True)
    for spec in argv[1:]:
        parts = spec.split(":")
        if parts[0] == "S":
            _train_entropy(outdir, parts[1], float(parts[2]),
                           int(parts[3]) if len(parts) > 3 else 3000)
            continue
        L, beta0 = int(parts[0]), float(parts[1])
        mu0 = float(parts[2]) if len(parts) > 2 else 1.0 / 3.0
        iters = int(parts[3]) if len(parts) > 3 else 3000
        t0 = time.time()
        th, rep, ok = training.train_coeffs(L, beta0, mu0, n_points=8192, max_iter=iters,
                                            tol=1e-10)
        dt = time.time() - t0
        name = _name(L, beta0, mu0)
        prov = (f"Trained by fe_train_coeffs (Levenberg-Marquardt with geodesic acceleration) on "
                f"the Fermi target at beta0={beta0:g}, mu0={mu0:.6g}: 8192 sample points as "
                f"quantiles of 1+|g'|, SP2 initial guess, {rep['iters']} iterations, tol 1e-10. "
                f"Max error on the trainer's check grid (FP64, device): {rep['max_err_grid']:.3e}.")
        m = models.Model(name=name, L=L, beta0=beta0, mu0=mu0, theta=th)
        path = models.save(m, os.path.join(outdir, name + ".json"), prov,
                           extra={"max_error": rep["max_err_grid"]})
        print(f"{name}: iters={rep['iters']} grid error {rep['max_err_grid']:.3e} "
              f"({dt:.1f} s) -> {path}", flush=True)


def _train_entropy(outdir, init_name, alpha, iters):
    from paper_2605_08523_amd import models, training
    src = models.load(init_name)
    t0 = time.time()
    th, rep, ok = training.train_coeffs(src.L, src.beta0, src.mu0, target="entropy", alpha=alpha,
                                        n_points=8192, max_iter=iters, tol=1e-10,
                                        theta_init=src.theta)
    dt = time.time() - t0
    base = os.path.basename(init_name).replace(".json", "")
    name = "entropy_" + (base[len("mlsp2_"):] if base.startswith("mlsp2_") else base)
    prov = (f"Trained by fe_train_coeffs (Levenberg-Marquardt with geodesic acceleration) on the "
            f"entropy target at beta0={src.beta0:g}, mu0={src.mu0:.6g}, alpha={alpha:g}: 8192 "
            f"sample points as quantiles of 1+|g'|, initial guess the Fermi model {base}, "
            f"{rep['iters']} iterations, tol 1e-10. Max error on the trainer's check grid (FP64, "
            f"device): {rep['max_err_grid']:.3e}.")
    m = models.Model(name=name, L=src.L, beta0=src.beta0, mu0=src.mu0, theta=th, kind="entropy",
                     alpha=alpha)
    path = models.save(m, os.path.join(outdir, name + ".json"), prov,
                       extra={"max_error": rep["max_err_grid"]})
    print(f"{name}: iters={rep['iters']} grid error {rep['max_err_grid']:.3e} ({dt:.1f} s) -> "
          f"{path}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
