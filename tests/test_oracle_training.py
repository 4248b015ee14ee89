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


def test_sample_points_arclen_against_polyline_length():
    """law = "arclen": the points split the graph of g into equal arc lengths. Checked against
    the length of the polyline through (t, g(t)) on an independent fine grid (no derivative
    used), and against the step limit: for a sharp step at mu0 the graph is a horizontal run
    of length mu0, a unit rise, and a run of length 1 - mu0, so a quarter of the total length
    of 2 ... lies below the step (mu0 / 2 of it) and half on the rise."""
    n, b0, m0 = 4096, 300.0, 1 / 3
    y = T.sample_points(n, b0, m0, "arclen")
    assert np.all(np.diff(y) > 0) and y[0] > 0 and y[-1] < 1
    t = np.linspace(0.0, 1.0, 2_000_001)
    gt = T.fermi_target(t, b0, m0)
    seg = np.hypot(np.diff(t), np.diff(gt))
    s = np.concatenate([[0.0], np.cumsum(seg)])
    frac = np.interp(y, t, s) / s[-1]
    np.testing.assert_allclose(frac, (np.arange(n) + 0.5) / n, atol=2e-6)
    # sharp step: fractions of points below, on and above the rise
    yb = T.sample_points(8192, 1e5, m0, "arclen")
    w = 40 / 1e5
    below, rise = np.mean(yb < m0 - w), np.mean(np.abs(yb - m0) <= w)
    assert abs(below - m0 / 2) < 2e-3 and abs(rise - 0.5) < 2e-3


def test_max_abs_state_closed_forms():
    """SP2 layers (x^2 and 2x - x^2) keep [0, 1] in [0, 1] with 1 reached; a layer 2x^2 - 1
    (Chebyshev T2) maps [0, 1] onto [-1, 1]; a layer 3x maps 1 to 3."""
    sp2 = np.array([(1.0, 0.0, 0.0, 0.0), (-1.0, 2.0, 0.0, 0.0)] * 4)
    assert T.max_abs_state(sp2) == pytest.approx(1.0, abs=1e-15)
    assert T.max_abs_state(np.array([(2.0, 0.0, -1.0, 0.0)])) == pytest.approx(1.0, abs=1e-15)
    assert T.max_abs_state(np.array([(0.0, 3.0, 0.0, 0.0)])) == pytest.approx(3.0, abs=1e-15)
    # entropy kind: the first state is alpha (y - mu0) + mu0, whose largest |.| on [0, 1] is at y = 1
    assert T.max_abs_state(np.zeros((0, 4)), "entropy", 0.3, 2.0) == pytest.approx(1.7, abs=1e-15)


def test_second_directional_closed_form_and_differences(paper_model):
    """Two layers, direction only on a_0: x1 = (a0 + t) x^2 + b0 x + c0 is linear in t, so
    d^2 x2 / dt^2 = 2 a1 (x^2)^2 and the accumulator terms add d1 * 0; then the printed model
    against a plain second difference of the model output (no complex step)."""
    th = np.array([(1.3, -0.2, 0.05, 0.4), (-0.7, 1.6, 0.0, 0.0)])
    v = np.zeros_like(th)
    v[0, 0] = 1.0
    y = np.linspace(0.0, 1.0, 11)
    np.testing.assert_allclose(T.second_directional(y, th, v), 2 * th[1, 0] * y ** 4,
                               rtol=1e-7, atol=1e-9)
    th = paper_model.theta[:12]
    rng = np.random.default_rng(5)
    v = rng.standard_normal(th.shape) * 1e-2
    y = np.linspace(0.05, 0.95, 23)
    for kind in ("fermi", "entropy"):
        got = T.second_directional(y, th, v, kind, 1 / 3, 0.842704)
        h = 1e-3
        f = lambda t: T.forward(y, th + t * v, kind, 1 / 3, 0.842704)
        fd = (f(h) - 2 * f(0.0) + f(-h)) / (h * h)
        np.testing.assert_allclose(got, fd, rtol=1e-4, atol=1e-6 * np.max(np.abs(fd)))
