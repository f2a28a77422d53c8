"""Adaptive weighting policy (host side): one round moves weight towards
constraints with small gradient magnitude, within the clip bounds, keeping the
mean weight."""
import numpy as np

from paper_2606_06656_amd.weighting import adaptive_weights


def test_flat_constraints_gain_weight():
    mag = np.array([0.01, 0.1, 1.0, 2.0, 0.5])
    w = adaptive_weights(mag, alpha=0.5, lo=0.25, hi=4.0)
    assert np.all(np.diff(w[np.argsort(mag)]) <= 1e-6)  # weight decreases with magnitude
    assert abs(w.mean() - 1.0) < 1e-6


def test_clip_and_zero_alpha():
    mag = np.array([1e-9, 1.0, 1.0, 1.0])
    w = adaptive_weights(mag, alpha=1.0, lo=0.5, hi=2.0)
    raw = np.clip(np.mean(mag) / np.maximum(mag, 1e-3 * np.mean(mag)), 0.5, 2.0)
    np.testing.assert_allclose(w, raw * (1.0 / raw.mean()), rtol=1e-6)
    np.testing.assert_array_equal(adaptive_weights(mag, alpha=0.0), np.ones(4, np.float32))


def test_inactive_constraints_keep_weight():
    mag = np.array([0.0, 0.2, 0.8])  # the first is constant (zero gradient everywhere)
    w0 = np.array([3.0, 1.0, 1.0])
    w = adaptive_weights(mag, w0, alpha=0.5)
    assert w[0] == 3.0
    assert abs(w[1:].mean() - 1.0) < 1e-6 and w[1] > w[2]
