"""The model bank: every stored coefficient table meets its recorded error, measured by the oracle."""
import pytest

from oracle import training as T
from paper_2605_08523_amd import models


@pytest.mark.parametrize("name", models.available())
def test_model_bank_entry(name):
    m = models.load(name)
    assert m.theta.shape == (m.L, 4)
    err = T.max_model_error(m.theta, m.beta0, m.mu0, n=200001)
    recorded = m.meta.get("max_error", 5.960464477539063e-08)
    assert err <= 1.01 * recorded
    # inside the 16-bit operand range of the split modes
    assert T.max_abs_state(m.theta, m.kind, m.mu0, m.alpha) < 16.0
