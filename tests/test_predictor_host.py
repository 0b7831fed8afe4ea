"""Host-side pieces of the flag predictor (no GPU): feature assembly, the
feature normalizer and the precision/recall count."""
import numpy as np

from paper_1507_06767_amd import predictor as P


def test_features_layout():
    means = np.arange(2 * 3 * 4 * 4, dtype=np.float64).reshape(2, 3, 4, 4)
    bm = np.full((2, 3, 4), 1e-3)
    prev = np.full((2, 3, 4), 1e-20)        # below the floor: log10 of the floor
    f = P.features(means, bm, prev)
    assert f.shape == (2, 3, 4, 6)
    assert np.array_equal(f[..., :4], means)
    assert np.allclose(f[..., 4], np.log10(P.LOG_FLOOR)) and np.allclose(f[..., 5], -3.0)
    assert P.features(means, bm).shape == (2, 3, 4, 5)


def test_normalizer_standardises_channels():
    rng = np.random.default_rng(0)
    raw = rng.standard_normal((50, 4, 4, 4, 3)) * [1.0, 10.0, 1e-3] + [5.0, -2.0, 0.0]
    raw[..., 2] = 7.0                      # a constant channel is only shifted
    z = P.Normalizer.fit(raw)(raw)
    assert np.allclose(z[..., :2].reshape(-1, 2).mean(0), 0.0, atol=1e-12)
    assert np.allclose(z[..., :2].reshape(-1, 2).std(0), 1.0, atol=1e-12)
    assert np.allclose(z[..., 2], 0.0)


def test_flag_scores():
    true = np.array([1, 1, 1, 0, 0, 0, 0, 1], dtype=bool)
    pred = np.array([1, 1, 0, 1, 0, 0, 0, 0], dtype=bool)
    p, r = P.flag_scores(pred, true)
    assert (p, r) == (2 / 3, 2 / 4)
    assert P.flag_scores(np.zeros(4, bool), np.zeros(4, bool)) == (0.0, 0.0)


def test_learned_quantity_and_its_scale():
    """The sensor network learns the change of log10 M_b from its last input
    channel; the (rho, u) network learns log10 M_b itself, standardised with
    the training targets' mean and spread."""
    from types import SimpleNamespace
    rng = np.random.default_rng(1)
    raw = rng.standard_normal((3, 2, 2, 2, 6))
    y = rng.standard_normal((3, 2, 2, 2)) * 0.7 - 3.0
    res = SimpleNamespace(residual=True)
    assert P.FlagPredictor._target_scale(res, raw, y) == (0.0, 1.0)
    assert np.array_equal(P.FlagPredictor._learned(res, raw, y), y - raw[..., -1])
    direct = SimpleNamespace(residual=False)
    off, sc = P.FlagPredictor._target_scale(direct, raw[..., :4], y)
    z = (P.FlagPredictor._learned(direct, raw[..., :4], y) - off) * sc
    assert abs(z.mean()) < 1e-12 and abs(z.std() - 1.0) < 1e-12
