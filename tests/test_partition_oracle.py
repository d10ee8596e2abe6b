"""Pins of the partition / tag-split-pack oracle against what the paper and
geometry fix (Sec. 4.2 sample distribution, Sec. 4.4 and App. A.3 partitioning)."""
import numpy as np
import pytest

from oracle import partition as P
from oracle import render as O
from paper_2404_16221_amd import synth


def lattice(n):
    """Cell centres of an n x n x n lattice over [0, 1]^3 (float32)."""
    c = (np.arange(n, dtype=np.float64) + 0.5) / n
    g = np.stack(np.meshgrid(c, c, c, indexing="ij"), axis=-1).reshape(-1, 3)
    return g.astype(np.float32)


def leaf_counts(points, axis, plane, levels):
    cnt = np.zeros(1 << levels, np.int64)
    for x in points:
        cnt[P.box_of_point(axis, plane, levels, x)] += 1
    return cnt


def halving(m, levels):
    """Leaf counts that splitting at the rank-floor(m/2) order statistic gives."""
    if levels == 0:
        return [m]
    return halving(m // 2, levels - 1) + halving(m - m // 2, levels - 1)


@pytest.mark.parametrize("n,levels", [(1000, 3), (1001, 3), (777, 4), (5, 3)])
def test_counts_follow_the_cdf_half_plane(n, levels):
    # distinct coordinates: exactly floor(m/2) points fall below each plane
    pts = np.random.default_rng(n).normal(size=(n, 3)).astype(np.float32)
    axis, plane = P.cdf_partition(pts, levels)
    assert list(leaf_counts(pts, axis, plane, levels)) == halving(n, levels)


def test_lattice_axis_choice_and_planes():
    # 8^3 lattice: the root cuts x at the 257th coordinate (layer 4.5/8); the
    # children (0.5 x 0.875 x 0.875) prefer y over x (ratio 2.33 vs 3.5, tie
    # with z broken towards y), the grandchildren z.
    pts = lattice(8)
    axis, plane = P.cdf_partition(pts, 3)
    assert list(axis) == [0, 1, 1, 2, 2, 2, 2]
    assert plane[0] == np.float32(4.5 / 8)
    assert plane[1] == plane[2] == np.float32(4.5 / 8)
    assert all(plane[i] == np.float32(4.5 / 8) for i in range(3, 7))
    assert list(leaf_counts(pts, axis, plane, 3)) == [64] * 8


def test_elongated_cloud_splits_the_long_axis_first():
    # 8 x 1 x 1 slab: three cuts along x make eight near-cubes
    rng = np.random.default_rng(5)
    pts = (rng.random((4000, 3)) * np.array([8.0, 1.0, 1.0])).astype(np.float32)
    axis, plane = P.cdf_partition(pts, 3)
    assert list(axis) == [0] * 7
    assert sorted(np.round(plane.astype(np.float64)).tolist()) == [1, 2, 3, 4, 5, 6, 7]


def test_aspect_ratio_cases():
    assert P.aspect_ratio([2.0, 1.0, 4.0]) == 4.0
    assert P.aspect_ratio([0.0, 1.0, 1.0]) == np.inf
    assert P.aspect_ratio([0.0, 0.0, 0.0]) == 1.0


def test_grid_tree_tags_like_the_cell_formula():
    # a 2 x 2 x 2 grid over [-1, 1]^3 written as a tree (x, then y, then z at
    # 0): leaf b holds the cell with x-bit b>>2, y-bit (b>>1)&1, z-bit b&1
    axis = np.array([0, 1, 1, 2, 2, 2, 2], np.int32)
    plane = np.zeros(7, np.float32)
    x = np.random.default_rng(2).uniform(-3, 3, size=(500, 3))
    for p in x:
        bits = (p >= 0).astype(int)
        assert P.box_of_point(axis, plane, 3, p) == 4 * bits[0] + 2 * bits[1] + bits[2]
    lo, hi = P.leaf_bounds(axis, plane, 3)
    assert lo[5].tolist() == [0.0, -np.inf, 0.0] and hi[5].tolist() == [np.inf, 0.0, np.inf]


def test_hand_example_one_plane():
    # ray along +x from x = -2: crosses the plane x = 0 at t = 2 exactly
    axis, plane = np.array([0], np.int32), np.array([0.0], np.float32)
    o = np.array([[-2.0, 0.3, 0.3]], np.float32)
    d = np.array([[1.0, 0.0, 0.0]], np.float32)
    ts = np.array([0.0, 1.0, 2.0, 2.0, 2.5], np.float32)
    te = np.array([1.0, 2.0, 2.0, 2.5, 3.0], np.float32)   # one zero-width sample at 2
    out = P.tag_split_pack(o, d, ts, te, np.array([0, 5]), axis, plane, 1)
    assert out["t_start"].tolist() == [0.0, 1.0, 2.0, 2.0, 2.5]
    assert out["src"].tolist() == [0, 1, 2, 3, 4]
    assert out["seg_offsets"].tolist() == [0, 2, 5] and out["seg_box"].tolist() == [0, 1]
    # a sample across the plane is cut in two
    ts2 = np.array([1.5], np.float32)
    te2 = np.array([2.75], np.float32)
    out = P.tag_split_pack(o, d, ts2, te2, np.array([0, 1]), axis, plane, 1)
    assert out["t_start"].tolist() == [1.5, 2.0] and out["t_end"].tolist() == [2.0, 2.75]
    assert out["src"].tolist() == [0, 0] and out["seg_ids"].tolist() == [0, 1]
    # travelling the other way, the high box comes first along the ray
    o2 = np.array([[2.0, 0.3, 0.3]], np.float32)
    d2 = np.array([[-1.0, 0.0, 0.0]], np.float32)
    out = P.tag_split_pack(o2, d2, ts2, te2, np.array([0, 1]), axis, plane, 1)
    assert out["seg_box"].tolist() == [0, 1] and out["seg_ids"].tolist() == [1, 0]
    assert out["t_start"].tolist() == [2.0, 1.5] and out["t_end"].tolist() == [2.75, 2.0]


def test_ray_on_a_plane_parallel_to_it_goes_high():
    axis, plane = np.array([0], np.int32), np.array([0.0], np.float32)
    o = np.array([[0.0, -1.0, 0.0]], np.float32)
    d = np.array([[0.0, 1.0, 0.0]], np.float32)
    out = P.tag_split_pack(o, d, np.array([0.0, 1.0], np.float32), np.array([1.0, 2.0], np.float32),
                           np.array([0, 2]), axis, plane, 1)
    assert out["seg_box"].tolist() == [1] and out["seg_offsets"].tolist() == [0, 2]


def test_pieces_tile_samples_and_lie_in_their_boxes():
    rng = np.random.default_rng(7)
    o, d, ts, te, ro = synth.random_rays(7, 60, 40)
    pts = rng.normal(scale=0.6, size=(2000, 3)).astype(np.float32)
    axis, plane = P.cdf_partition(pts, 3)
    out = P.tag_split_pack(o, d, ts, te, ro, axis, plane, 3)
    src, a, b = out["src"], out["t_start"], out["t_end"]
    n_in = ts.shape[0]
    # every input sample yields pieces that tile [s, e) exactly, in t order
    seg_of_piece = np.repeat(np.arange(out["seg_box"].shape[0]), np.diff(out["seg_offsets"]))
    by_src = {}
    for k in range(src.shape[0]):
        by_src.setdefault(int(src[k]), []).append(k)
    assert sorted(by_src) == list(range(n_in))
    n_cut = 0
    for i, ks in by_src.items():
        ks = sorted(ks, key=lambda k: (a[k], b[k]))
        assert a[ks[0]] == ts[i] and b[ks[-1]] == te[i]
        for k0, k1 in zip(ks[:-1], ks[1:]):
            assert b[k0] == a[k1] and a[k0] < b[k0]
        n_cut += len(ks) - 1
    assert n_cut > 10  # the case really cuts samples
    # piece midpoints lie in their box (brute-force point tagging), away from faces
    lo, hi = P.leaf_bounds(axis, plane, 3)
    checked = 0
    for k in range(src.shape[0]):
        s = int(seg_of_piece[k])
        r = int(out["seg_ray"][s])
        m = 0.5 * (float(a[k]) + float(b[k]))
        x = o[r].astype(np.float64) + m * d[r].astype(np.float64)
        bx = int(out["seg_box"][s])
        margin = min(np.min(x - lo[bx]), np.min(hi[bx] - x))
        if margin > 1e-5:
            assert P.box_of_point(axis, plane, 3, x) == bx
            checked += 1
    assert checked > 0.9 * src.shape[0]
    # region-major, rays in order inside a box, each ray's segments front to back
    sb, sr = out["seg_box"], out["seg_ray"]
    key = sb.astype(np.int64) * (1 << 32) + sr
    assert np.all(np.diff(key) > 0)
    for r in range(o.shape[0]):
        segs = out["seg_ids"][out["ray_offsets"][r]:out["ray_offsets"][r + 1]]
        assert np.all(sr[segs] == r)
        starts = a[out["seg_offsets"][segs]]
        assert np.all(np.diff(starts) > 0) or len(segs) < 2


def test_one_box_returns_the_input():
    o, d, ts, te, ro = synth.random_rays(8, 30, 20)
    out = P.tag_split_pack(o, d, ts, te, ro, np.zeros(0, np.int32), np.zeros(0, np.float32), 0)
    assert np.array_equal(out["t_start"], ts) and np.array_equal(out["t_end"], te)
    assert np.array_equal(out["src"], np.arange(ts.shape[0]))
    nonempty = np.flatnonzero(np.diff(ro) > 0)
    assert np.array_equal(out["seg_offsets"], np.append(ro[nonempty], ro[-1]))
    assert np.array_equal(np.diff(out["ray_offsets"]), (np.diff(ro) > 0).astype(np.int64))


def test_splitting_keeps_transmittance_colour_and_opacity():
    # a piece inherits its sample's density and colour: cutting [s, e) at u
    # multiplies the transmittances exp(-sigma (u - s)) exp(-sigma (e - u)) and
    # splits the alpha-weighted colour exactly, so T, C and A of every ray
    # are unchanged (depth and distortion use piece midpoints and may move)
    o, d, ts, te, ro = synth.random_rays(9, 40, 30)
    rng = np.random.default_rng(9)
    sig = rng.lognormal(0.0, 1.5, size=ts.shape[0])
    rgb = rng.random((ts.shape[0], 3))
    pts = rng.normal(scale=0.5, size=(500, 3)).astype(np.float32)
    axis, plane = P.cdf_partition(pts, 4)
    out = P.tag_split_pack(o, d, ts, te, ro, axis, plane, 4)
    assert out["src"].shape[0] > ts.shape[0]
    split = O.render_rays_single(sig[out["src"]], rgb[out["src"]], out["t_start"], out["t_end"],
                                 out["seg_offsets"], out["ray_offsets"], out["seg_ids"])
    R = o.shape[0]
    has = np.diff(ro) > 0
    whole = O.render_rays_single(sig, rgb, ts, te, np.append(ro[:-1][has], ro[-1]),
                                 np.concatenate([[0], np.cumsum(has)]), np.arange(int(has.sum())))
    np.testing.assert_allclose(split[:5], whole[:5], rtol=1e-12, atol=1e-14)
