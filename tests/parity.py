"""Parity bounds shared by the GPU tests.

* BAR: the accuracy bar of the expansion, ||D - D_ref||_F / N <= 1e-5.
* ``within``: a measured error must stay below `factor` (10) times the error measured for the
  same case on MI355X (the value is written beside each case in the tests), so that a loss of
  accuracy far below the bar (a bad tile, a dropped term, a wrong split) still fails.
* ``traces_consistent``: the FP64 traces a kernel returns against the oracle's, bounded by what
  the element-wise error allows: |Tr dD| <= sqrt(N) ||dD||_F and
  |sum D^2 - sum D_ref^2| <= 2 ||D_ref||_F ||dD||_F + ||dD||_F^2 (Cauchy-Schwarz), plus the FP64
  rounding of the sums.
"""
import numpy as np

BAR = 1e-5


def within(tag, value, measured, factor=10.0, cap=None):
    bound = factor * measured
    if cap is not None:
        bound = min(bound, cap)
    assert value <= bound, (f"{tag}: {value:.3e} above {bound:.3e} ({factor:g} x the measured "
                            f"{measured:.3e})")


def check_errors(tag, fro, mx, measured, dtr=None):
    """fro = ||dD||_F/N and mx = max |dD| against their measured values (fro_m, max_m[, dtr_m]);
    fro also against the bar."""
    within(f"{tag} |dD|_F/N", fro, measured[0], cap=BAR)
    within(f"{tag} max|dD|", mx, measured[1])
    if dtr is not None and len(measured) > 2:
        within(f"{tag} |dTrD|", dtr, measured[2])


def traces_consistent(tag, D, Dref, trD, trD2, ref_trD, ref_trD2):
    n = D.shape[0]
    e = np.linalg.norm(D - Dref)
    rnd = 1e-12 * n * n
    b_tr = np.sqrt(n) * e + rnd
    b_sq = 2.0 * np.linalg.norm(Dref) * e + e * e + rnd
    assert abs(trD - ref_trD) <= b_tr, f"{tag}: |dTrD| {abs(trD - ref_trD):.3e} > {b_tr:.3e}"
    assert abs(trD2 - ref_trD2) <= b_sq, f"{tag}: |d sum D^2| {abs(trD2 - ref_trD2):.3e} > {b_sq:.3e}"
