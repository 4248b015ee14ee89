"""Host logic of the Skip-SP2 / Max-SP2 C ABI (no GPU): coefficient counts and the MLSP2
embeddings of App. C, against the oracle's own embeddings."""
import numpy as np
import pytest

from oracle import variants as V


@pytest.fixture(scope="module")
def var():
    from paper_2605_08523_amd import api, variants
    try:
        api.lib()
    except OSError as e:   # library not built
        pytest.skip(str(e))
    return variants


def test_coef_counts(var):
    for L in (1, 5, 26, 64):
        assert var.coef_count("max", L) == V.max_param_count(L)
        for k, K in [(1, 1), (2, 1), (3, 2), (4, 4)]:
            assert var.coef_count("skip", L, k, K) == V.skip_param_count(L, k, K)


@pytest.mark.parametrize("name", ["mlsp2_L26_b1500_mu1third", "mlsp2_L22_b600_mu1third"])
def test_embedding_matches_oracle(var, name):
    from paper_2605_08523_amd import models
    m = models.load(name)
    skip = V.mlsp2_to_skip(m.theta)
    got_s = var.embed_mlsp2(m, "skip")
    np.testing.assert_allclose(got_s.coef, V.flatten(skip), rtol=1e-14, atol=1e-15)
    got_m = var.embed_mlsp2(m, "max")
    np.testing.assert_allclose(got_m.coef, V.flatten(V.skip_to_max(skip)), rtol=1e-14, atol=1e-15)
    y = np.linspace(0, 1, 501)
    from oracle import recursion as R
    np.testing.assert_allclose(V.evaluate(y, V.unflatten(got_m.coef, V.skip_to_max(skip))),
                               R.mlsp2_layers(y, m.theta), atol=1e-9)


def test_embedding_rejects_linear_layer(var):
    from paper_2605_08523_amd import api
    th = np.array([[1.0, 0.0, 0.0, 0.0], [0.0, 1.0, 0.0, 0.5]])
    with pytest.raises(api.FeError):
        var.embed_mlsp2(api.make_model(th, 100.0, 1 / 3), "skip")


def test_shape_errors(var):
    with pytest.raises(ValueError):
        var.QModel("max", 3, np.zeros(5), 100.0, 1 / 3)
    from paper_2605_08523_amd import api
    with pytest.raises(api.FeError):
        var.coef_count("skip", 3, 0, 1)
