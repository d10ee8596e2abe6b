"""Pins of the breakable-integral oracle (oracle/breakable.py) against what App.
B.2 and the mathematics fix: the members the Examples subsection works out
(transmittance, volume rendering, distortion loss, computed independently by
oracle/render.py), closed forms, the Property 1 product identity, brute-force
integration of the continuous nested integral, the equivalence of any split
with the single pass, and finite differences."""
import math

import numpy as np
import pytest
import torch

from oracle import breakable as B
from oracle import render as R


def _ray(rng, n, zero_frac=0.2):
    w = rng.exponential(0.02, size=n)
    t0 = 0.1 + np.concatenate([[0.0], np.cumsum(w)[:-1]])
    t1 = t0 + w
    sig = np.exp(rng.normal(0.0, 1.5, size=n))
    sig[rng.uniform(size=n) < zero_frac] = 0.0
    return sig, t0, t1


def test_volume_rendering_member_is_the_colour_path():
    """Channels = colour: Phi is C of Eq. 1 and T the transmittance (Examples)."""
    rng = np.random.default_rng(1)
    sig, t0, t1 = _ray(rng, 40)
    rgb = rng.uniform(size=(40, 3))
    got = B.single(sig, rgb, t0, t1, [])
    ref = R.to_ray_tuple(R.composite(sig, rgb, t0, t1))
    assert got[0] == pytest.approx(ref[0], rel=1e-13)
    np.testing.assert_allclose(got[1:4], ref[1:4], rtol=1e-13)


def test_distortion_member():
    """Channels (1, m): Phi = (A, D), and 2 (Psi_(m,1) - Psi_(1,m)) is the
    distortion loss without its within-sample term (1/3) sum w^2 delta."""
    rng = np.random.default_rng(2)
    for n in (1, 2, 17, 60):
        sig, t0, t1 = _ray(rng, n)
        ch = B.midpoint_powers(t0, t1, 2)
        got = B.single(sig, ch, t0, t1, [(1, 0), (0, 1)])
        ref = R.composite(sig, np.zeros((n, 3)), t0, t1)
        delta, m, tau, alpha, T, w = R.quadrature(sig, t0, t1)
        assert got[1] == pytest.approx(ref[4], rel=1e-13, abs=1e-300)
        assert got[2] == pytest.approx(ref[5], rel=1e-13, abs=1e-300)
        L_cross = ref[6] - (w * w * delta).sum() / 3.0
        assert 2.0 * (got[3] - got[4]) == pytest.approx(L_cross, rel=1e-11, abs=1e-15)


@pytest.mark.parametrize("sigma", [0.3, 2.0, 40.0])
def test_closed_forms(sigma):
    """Psi_(1,1) = A^2 / 2 for any density; constant density gives A = 1 - e^(-sigma L)."""
    rng = np.random.default_rng(3)
    w = rng.uniform(0.001, 0.04, size=50)
    t0 = 0.2 + np.concatenate([[0.0], np.cumsum(w)[:-1]])
    t1 = t0 + w
    ch = np.ones((50, 1))
    got = B.single(np.full(50, sigma), ch, t0, t1, [(0, 0)])
    A = -math.expm1(-sigma * (t1[-1] - t0[0]))
    assert got[1] == pytest.approx(A, rel=1e-13)
    assert got[2] == pytest.approx(0.5 * A * A, rel=1e-12)
    sig, t0, t1 = _ray(rng, 33)
    got = B.single(sig, np.ones((33, 1)), t0, t1, [(0, 0)])
    assert got[2] == pytest.approx(0.5 * got[1] ** 2, rel=1e-12)


def test_property_1_product_identity():
    """Psi_(a,b) + Psi_(b,a) = Phi_a Phi_b: the product of two first-order
    members is the sum of the two nested ones."""
    rng = np.random.default_rng(4)
    sig, t0, t1 = _ray(rng, 25)
    ch = rng.normal(size=(25, 3))
    got = B.single(sig, ch, t0, t1, [(0, 2), (2, 0), (1, 1)])
    assert got[4] + got[5] == pytest.approx(got[1] * got[3], rel=1e-12, abs=1e-14)
    assert 2.0 * got[6] == pytest.approx(got[2] ** 2, rel=1e-12, abs=1e-14)


def test_nested_integral_by_brute_force():
    """The discrete Psi equals the continuous nested integral of Property 2 for
    piecewise-constant density and channels (midpoint rule on a fine grid)."""
    rng = np.random.default_rng(5)
    sig, t0, t1 = _ray(rng, 4, zero_frac=0.0)
    sig *= 8.0
    ch = rng.uniform(0.5, 2.0, size=(4, 2))
    got = B.single(sig, ch, t0, t1, [(0, 1)])
    M = 4000
    us, ws, a, b = [], [], [], []
    T = 1.0
    for i in range(4):
        h = (t1[i] - t0[i]) / M
        u = t0[i] + (np.arange(M) + 0.5) * h
        Tu = T * np.exp(-sig[i] * (u - t0[i]))
        ws.append(Tu * sig[i] * h)
        a.append(np.full(M, ch[i, 0]))
        b.append(np.full(M, ch[i, 1]))
        T *= math.exp(-sig[i] * (t1[i] - t0[i]))
    ws, a, b = np.concatenate(ws), np.concatenate(a), np.concatenate(b)
    inner = np.cumsum(ws * b) - ws * b + 0.5 * ws * b   # int_{v<u} w(v) b(v) dv at the cell midpoints
    psi = (ws * a * inner).sum()
    assert got[3] == pytest.approx(psi, rel=1e-6)
    assert got[1] == pytest.approx((ws * a).sum(), rel=1e-6)


@pytest.mark.parametrize("seed", [6, 7, 8])
def test_any_split_merges_to_the_single_pass(seed):
    rng = np.random.default_rng(seed)
    n = 45
    sig, t0, t1 = _ray(rng, n)
    ch = rng.normal(size=(n, 3))
    pairs = [(0, 1), (2, 2), (1, 0)]
    ref = B.single(sig, ch, t0, t1, pairs)
    for trial in range(4):
        k = int(rng.integers(1, 8))
        cuts = np.sort(rng.choice(np.arange(0, n + 1), size=k, replace=True))
        edges = np.concatenate([[0], cuts, [n]])
        parts = [B.segment(sig[a:b], ch[a:b], t0[a:b], t1[a:b], pairs)
                 for a, b in zip(edges[:-1], edges[1:])]
        np.testing.assert_allclose(B.merge(parts, 3, pairs), ref, rtol=1e-11, atol=1e-14)


def test_empty_segments_and_rays():
    out = B.segment(np.zeros(0), np.zeros((0, 2)), np.zeros(0), np.zeros(0), [(0, 1)])
    np.testing.assert_array_equal(out, np.zeros(4))
    np.testing.assert_array_equal(B.merge([], 2, [(0, 1)]), [1.0, 0.0, 0.0, 0.0])
    rng = np.random.default_rng(9)
    sig, t0, t1 = _ray(rng, 6)
    ch = rng.normal(size=(6, 2))
    x = B.segment(sig, ch, t0, t1, [(0, 1)])
    np.testing.assert_allclose(B.merge([out, x, out], 2, [(0, 1)]),
                               B.merge([x], 2, [(0, 1)]), rtol=1e-15)


def test_torch_twins_equal_the_plain_loops():
    rng = np.random.default_rng(10)
    sig, t0, t1 = _ray(rng, 30)
    ch = rng.normal(size=(30, 3))
    pairs = [(0, 1), (2, 0)]
    x = B._segment_t(B._t(sig), B._t(ch), B._t(t0), B._t(t1), pairs).numpy()
    np.testing.assert_allclose(x, B.segment(sig, ch, t0, t1, pairs), rtol=1e-12, atol=1e-15)
    parts = np.array([B.segment(sig[a:b], ch[a:b], t0[a:b], t1[a:b], pairs)
                      for a, b in ((0, 7), (7, 7), (7, 22), (22, 30))])
    y = B._merge_t(B._t(parts), 3, pairs).numpy()
    np.testing.assert_allclose(y, B.merge(list(parts), 3, pairs), rtol=1e-12, atol=1e-15)


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(11)
    n = 14
    sig, t0, t1 = _ray(rng, n, zero_frac=0.0)
    ch = rng.normal(size=(n, 2))
    pairs = [(0, 1), (1, 1)]
    so = np.array([0, 5, 5, 9, n])
    ro = np.array([0, 4])
    ids = np.array([0, 1, 2, 3])
    g = rng.normal(size=(1 + 2 + 2, 1))
    gseg, gs, gc = B.backward(sig, ch, t0, t1, so, ro, ids, pairs, g)

    def f(s, c):
        _, ray = B.render_rays(s, c, t0, t1, so, ro, ids, pairs)
        return float(ray[:, 0] @ g[:, 0])
    for i in range(n):
        h = 1e-6 * max(1.0, sig[i])
        sp, sm = sig.copy(), sig.copy()
        sp[i] += h
        sm[i] -= h
        assert gs[i] == pytest.approx((f(sp, ch) - f(sm, ch)) / (2 * h), rel=1e-6, abs=1e-9)
        for c in range(2):
            cp, cm = ch.copy(), ch.copy()
            cp[i, c] += 1e-6
            cm[i, c] -= 1e-6
            assert gc[i, c] == pytest.approx((f(sig, cp) - f(sig, cm)) / 2e-6, rel=1e-6, abs=1e-9)
    # the segment gradients are those of the merge alone
    seg, _ = B.render_rays(sig, ch, t0, t1, so, ro, ids, pairs)
    for k in range(4):
        for q in range(5):
            xp, xm = seg.copy(), seg.copy()
            xp[q, k] += 1e-6
            xm[q, k] -= 1e-6
            fd = (B.merge(list(xp.T), 2, pairs) - B.merge(list(xm.T), 2, pairs)) @ g[:, 0] / 2e-6
            assert gseg[q, k] == pytest.approx(fd, rel=1e-6, abs=1e-9)
