"""Pins for oracle.training (CPU only)."""
import math

import numpy as np
import pytest

from oracle import recursion as R
from oracle import training as T


@pytest.mark.parametrize("kind", ["fermi", "entropy"])
def test_jacobian_matches_central_differences(paper_model, kind):
    th = paper_model.theta[:10].copy()
    y = np.linspace(0.05, 0.95, 37)
    out, J = T.jacobian(y, th, kind, mu0=1 / 3, alpha=0.842704)
    np.testing.assert_allclose(out, T.forward(y, th, kind, 1 / 3, 0.842704), atol=1e-15)
    flat = th.reshape(-1)
    fd = np.zeros_like(J)
    for k in range(flat.size):
        h = 1e-6 * max(1.0, abs(flat[k]))
        p, m = flat.copy(), flat.copy()
        p[k] += h
        m[k] -= h
        fd[:, k] = (T.forward(y, p.reshape(th.shape), kind, 1 / 3, 0.842704)
                    - T.forward(y, m.reshape(th.shape), kind, 1 / 3, 0.842704)) / (2 * h)
    np.testing.assert_allclose(J, fd, rtol=1e-6, atol=1e-7)


def test_forward_matches_layers(paper_model):
    y = np.linspace(0, 1, 101)
    np.testing.assert_allclose(T.forward(y, paper_model.theta), R.mlsp2_layers(y, paper_model.theta), atol=1e-14)


def test_sample_points_laws():
    u = T.sample_points(100, 1500, 1 / 3, "uniform")
    np.testing.assert_allclose(u, (np.arange(100) + 0.5) / 100, atol=1e-9)
    n, b0, m0 = 8192, 1e4, 1 / 3
    y = T.sample_points(n, b0, m0, "deriv")
    assert np.all(np.diff(y) > 0) and y[0] > 0 and y[-1] < 1
    # mass of p ~ 1 + |g'| inside [m0 - w, m0 + w]: (2w + g(m0+w) - g(m0-w)) / (1 + g(1) - g(0))
    w = 5 / b0
    gt = lambda v: T.fermi_target(np.array([v]), b0, m0)[0]
    mass = (2 * w + gt(m0 + w) - gt(m0 - w)) / (1 + gt(1.0) - gt(0.0))
    frac = np.mean((y > m0 - w) & (y < m0 + w))
    assert abs(frac - mass) < 2 / n


def test_targets():
    y = np.linspace(0, 1, 11)
    np.testing.assert_allclose(T.fermi_target(y, 40, 0.3), 1 / (1 + np.exp(40 * (0.3 - y))), atol=1e-15)
    assert T.entropy_target(np.array([0.3]), 40, 0.3)[0] == pytest.approx(math.log(2))
