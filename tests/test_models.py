"""The model bank: every stored coefficient table meets its recorded error, measured by the oracle."""
import pytest

from oracle import training as T
from paper_2605_08523_amd import models


@pytest.mark.parametrize("name", models.available())
def test_model_bank_entry(name):
    m = models.load(name)
    assert m.theta.shape == (m.L, 4)
    err = T.max_model_error(m.theta, m.beta0, m.mu0, kind=m.kind, alpha=m.alpha, n=200001)
    recorded = m.meta.get("max_error", 5.960464477539063e-08)
    assert err <= 1.01 * recorded
    # inside the 16-bit operand range of the split modes
    assert T.max_abs_state(m.theta, m.kind, m.mu0, m.alpha) < 16.0


def test_table1_entropy_rows():
    """Table I rows 4 and 5 (beta = 40, mu = 1/3, 2048 uniform eigenvalues on [0, 1], FP64):
    the 26-layer Fermi model with the alpha-rescaled ansatz (theta_fermi, alpha = 0.842704)
    reproduces the printed relative entropy error, set by the ansatz (6.8e-5); the entropy model
    trained from it (theta_entropy) reaches the printed levels of row 5 or better (max error
    6.73e-8, relative error 1.4e-8). The oracle evaluates both on the scalar spectrum."""
    import json
    import os

    import numpy as np

    from oracle import recursion as R
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
    g = {k: v["value"] for k, v in gold.items() if k != "_about"}
    beta, mu, n = g["table1_beta"], g["table1_mu"], int(g["table1_n_eigs"])
    x = np.linspace(0.0, 1.0, n)
    S = T.entropy_target(x, beta, mu).sum()
    fermi = models.load("mlsp2_L26_b40_mu1third")
    ent = models.load("entropy_L26_b40_mu1third")
    assert (fermi.beta0, fermi.mu0, ent.beta0, ent.mu0) == (beta, mu, beta, mu)
    rel_f = abs(R.entropy_scalar(x, fermi.theta, mu, g["alpha_minimax"]).sum() - S) / S
    rel_e = abs(R.entropy_scalar(x, ent.theta, mu, ent.alpha).sum() - S) / S
    err_e = T.max_model_error(ent.theta, beta, mu, kind="entropy", alpha=ent.alpha, n=200001)
    print(f"[Table I] theta_fermi rel {rel_f:.3e} (printed {g['table1_theta_fermi_rel_fp64']}), "
          f"theta_entropy rel {rel_e:.3e} max {err_e:.3e} (printed "
          f"{g['table1_theta_entropy_rel_fp64']}, {g['table1_theta_entropy_max_err']})")
    assert abs(rel_f - g["table1_theta_fermi_rel_fp64"]) <= 0.05e-5    # printed to two digits
    assert err_e <= g["table1_theta_entropy_max_err"]
    assert rel_e <= g["table1_theta_entropy_rel_fp64"]
