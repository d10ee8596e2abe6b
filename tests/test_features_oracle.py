"""Pins of the feature-channel oracle (App. B.2, Property 2 with the
transmittance as the breakable factor)."""
import numpy as np
import pytest

from oracle import features as Fo
from oracle import render as O


def ray(rng, n, F):
    w = rng.exponential(0.03, size=n)
    t1 = np.cumsum(w) + 0.2
    t0 = t1 - w
    sig = rng.lognormal(0.0, 1.5, size=n)
    sig[rng.random(n) < 0.2] = 0.0
    return sig, rng.normal(size=(n, F)), t0, t1


def test_colour_as_feature_is_the_colour():
    rng = np.random.default_rng(1)
    sig, _, t0, t1 = ray(rng, 40, 3)
    rgb = rng.random((40, 3))
    tau, phi = Fo.feature_segment(sig, rgb, t0, t1)
    ref = O.composite(sig, rgb, t0, t1)
    assert tau == pytest.approx(ref[0], rel=1e-14)
    np.testing.assert_allclose(phi, ref[1:4], rtol=1e-13)


def test_constant_density_closed_form():
    # constant sigma and feature over [0, L] in any cut: f (1 - exp(-sigma L))
    sig = np.full(7, 1.3)
    t = np.array([0.0, 0.1, 0.15, 0.4, 0.41, 0.9, 1.2, 2.0])
    f = np.tile([[2.0, -1.0, 0.5]], (7, 1))
    _, phi = Fo.feature_segment(sig, f, t[:-1], t[1:])
    np.testing.assert_allclose(phi, f[0] * (1.0 - np.exp(-1.3 * 2.0)), rtol=1e-14)


@pytest.mark.parametrize("cuts", [[5], [1, 2, 30], [10, 20, 30, 40]])
def test_any_split_merges_to_the_single_segment(cuts):
    rng = np.random.default_rng(len(cuts))
    sig, f, t0, t1 = ray(rng, 50, 6)
    edges = [0] + cuts + [50]
    seg_offsets = np.array(edges)
    tau, phi, out = Fo.render_features(sig, f, t0, t1, seg_offsets, np.array([0, len(edges) - 1]),
                                       np.arange(len(edges) - 1))
    _, whole = Fo.feature_segment(sig, f, t0, t1)
    np.testing.assert_allclose(out[0], whole, rtol=1e-12, atol=1e-15)


def test_empty_segment_and_ray_without_segments():
    tau, phi, out = Fo.render_features(np.zeros(0), np.zeros((0, 2)), np.zeros(0), np.zeros(0),
                                       np.array([0, 0]), np.array([0, 1, 1]), np.array([0]))
    assert tau.tolist() == [0.0] and phi.tolist() == [[0.0, 0.0]]
    assert out.tolist() == [[0.0, 0.0], [0.0, 0.0]]


@pytest.mark.parametrize("order", [[0, 1], [1, 0]])
def test_gradients_match_finite_differences(order):
    rng = np.random.default_rng(4)
    sig, f, t0, t1 = ray(rng, 12, 3)
    sig = sig + 0.1
    seg_offsets = np.array([0, 5, 12])
    ro = np.array([0, 2])
    ids = np.array(order)  # the merge follows the listed order
    g = rng.normal(size=(1, 3))
    gs, gf = Fo.grad_features(sig, f, t0, t1, seg_offsets, ro, ids, g)

    def loss(s, ff):
        _, _, out = Fo.render_features(s, ff, t0, t1, seg_offsets, ro, ids)
        return float((out * g).sum())
    h = 1e-6
    for i in range(12):
        e = np.zeros(12); e[i] = h
        num = (loss(sig + e, f) - loss(sig - e, f)) / (2 * h)
        assert gs[i] == pytest.approx(num, rel=1e-6, abs=1e-9)
        for c in range(3):
            E = np.zeros_like(f); E[i, c] = h
            num = (loss(sig, f + E) - loss(sig, f - E)) / (2 * h)
            assert gf[i, c] == pytest.approx(num, rel=1e-6, abs=1e-9)
