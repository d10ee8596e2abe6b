"""The library's host partition builder against the oracle (no GPU needed)."""
import numpy as np
import pytest

from oracle import partition as P
from paper_2404_16221_amd import _lib as xl


def clouds():
    rng = np.random.default_rng(11)
    yield "normal", rng.normal(size=(5000, 3)), 5
    yield "anisotropic", rng.normal(size=(3000, 3)) * np.array([10.0, 1.0, 0.2]), 6
    yield "ties", rng.integers(0, 4, size=(2000, 3)).astype(np.float64), 4
    yield "street", np.stack([np.linspace(-50, 50, 4096), rng.normal(scale=2.0, size=4096),
                              rng.exponential(3.0, size=4096)], axis=1), 6
    yield "few", rng.random((3, 3)), 3
    yield "one", np.array([[0.5, -1.0, 2.0]]), 2
    yield "none", np.zeros((0, 3)), 3
    yield "one box", rng.random((100, 3)), 0


@pytest.mark.parametrize("name,pts,levels", list(clouds()), ids=[c[0] for c in clouds()])
def test_partition_matches_oracle_bit_exact(name, pts, levels):
    pts = pts.astype(np.float32)
    axis, plane = xl.xl_partition_build(pts, levels)
    a_ref, p_ref = P.cdf_partition(pts, levels)
    assert np.array_equal(axis, a_ref), (axis, a_ref)
    assert np.array_equal(plane.view(np.uint32), p_ref.view(np.uint32))


def test_partition_rejects_bad_arguments():
    with pytest.raises(xl.XLError):
        xl.xl_partition_build(np.zeros((4, 3), np.float32), 7)
    bad = np.zeros((4, 3), np.float32)
    bad[2, 1] = np.nan
    with pytest.raises(xl.XLError):
        xl.xl_partition_build(bad, 2)
