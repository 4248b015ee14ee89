"""Train bank models with the library's own trainer (fe_train_coeffs) and store them as JSON.

Usage (on a machine with the GPU and the built library):
    python -m paper_2605_08523_amd.models.train_bank OUTDIR L:BETA0[:MU0[:ITERS]] ...
e.g. ``python -m paper_2605_08523_amd.models.train_bank out 20:300 22:600``. Each model is fitted
to the Fermi target g(y) = 1/(1 + exp(beta0 (mu0 - y))) (Sec. III.C) on 8192 points sampled as
quantiles of 1 + |g'|, from the SP2 initial guess, and written as ``mlsp2_L{L}_b{beta0}_mu...``
with the device-measured maximum error on the trainer's check grid in its provenance. The oracle
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


if __name__ == "__main__":
    main(sys.argv[1:])
