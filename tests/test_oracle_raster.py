"""Pins of the oracle's rasteriser (Method, Step 2; pixel-membership
reading) against exact rational ray casting, hand-derived labels and
geometric limits."""
import os

import numpy as np
import pytest

from oracle import cartogram as oc
from synth import square_grid_map, voronoi_map
from tests.brute import brute_labels

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rast(m, N):
    return oc.rasterize(m.xy, m.ring_off, m.ring_idx, m.ring_reg, m.n_regions, N)


def test_centres_on_edges_hand_labels():
    N = 8
    m = square_grid_map(2, 1, lo=1.5 / 8, hi=5.5 / 8)
    want = np.loadtxt(os.path.join(GOLDEN, "raster_centres_n8.txt"), dtype=np.int64)
    lab, cnt, conf = _rast(m, N)
    assert conf == 0
    np.testing.assert_array_equal(lab.astype(np.int64), want)
    np.testing.assert_array_equal(cnt, np.bincount(want.ravel(), minlength=5))


@pytest.mark.parametrize("seed,R,n,N", [(11, 4, 30, 8), (12, 6, 60, 16), (13, 5, 40, 16)])
def test_voronoi_vs_rational_ray_casting(seed, R, n, N):
    m = voronoi_map(seed, R, n, fractal=True)
    lab, cnt, conf = _rast(m, N)
    want = brute_labels(m.xy, m.ring_off, m.ring_idx, m.ring_reg, N)
    np.testing.assert_array_equal(lab.astype(np.int64), want)
    assert conf == 0


def test_vertices_on_centres_vs_ray_casting():
    # a triangle and a quad sharing an edge, every vertex on a pixel centre
    N = 16
    c = lambda k: (k + 0.5) / N
    xy = np.array([[c(2), c(2)], [c(12), c(4)], [c(6), c(13)], [c(14), c(12)]])
    ring_off = np.array([0, 3, 6], np.int32)
    # shoelace-positive orientation for both rings
    ring_idx = np.array([0, 1, 2, 1, 3, 2], np.int32)
    ring_reg = np.array([1, 2], np.int32)
    for k in range(2):
        ids = ring_idx[ring_off[k]:ring_off[k + 1]]
        p, q = xy[ids], np.roll(xy[ids], -1, 0)
        assert (p[:, 0] * q[:, 1] - q[:, 0] * p[:, 1]).sum() > 0
    lab, cnt, conf = oc.rasterize(xy, ring_off, ring_idx, ring_reg, 2, N)
    want = brute_labels(xy, ring_off, ring_idx, ring_reg, N)
    np.testing.assert_array_equal(lab.astype(np.int64), want)
    assert conf == 0


def test_folded_map_contested_pixels_take_highest_id():
    # two squares sharing the edge x = 1/2; its midpoint vertex is dragged
    # past the right square's far side, so both regions claim some centres
    xy = np.array([[0.2, 0.2], [0.5, 0.2], [0.8, 0.2], [0.8, 0.8], [0.5, 0.8],
                   [0.2, 0.8], [0.9, 0.47]])
    ring_off = np.array([0, 5, 10], np.int32)
    ring_idx = np.array([0, 1, 6, 4, 5, 1, 2, 3, 4, 6], np.int32)
    ring_reg = np.array([1, 2], np.int32)
    N = 16
    lab, cnt, conf = oc.rasterize(xy, ring_off, ring_idx, ring_reg, 2, N)
    want = brute_labels(xy, ring_off, ring_idx, ring_reg, N)
    assert conf > 0
    np.testing.assert_array_equal(lab.astype(np.int64), want)
    np.testing.assert_array_equal(cnt, np.bincount(want.ravel(), minlength=3))


def test_grid_outline_partition():
    N = 64
    m = square_grid_map(3, 4, lo=0.25, hi=0.75)
    lab, cnt, conf = _rast(m, N)
    assert conf == 0
    inside = np.zeros((N, N), bool)
    inside[16:48, 16:48] = True          # centres (p + 1/2)/64 inside [1/4, 3/4)
    assert np.all(lab[inside] > 0) and np.all(lab[~inside] == 0)
    assert cnt[1:].sum() == 32 * 32 and cnt.sum() == N * N


def test_counts_converge_to_shoelace_areas():
    m = voronoi_map(21, 12, 400, fractal=True)
    A = oc.region_areas(m.xy, m.ring_off, m.ring_idx, m.ring_reg, m.n_regions)
    errs = []
    for N in (64, 256, 1024):
        _, cnt, conf = _rast(m, N)
        assert conf == 0
        errs.append(np.abs(cnt[1:] / N**2 - A[1:]).max())
    assert errs[2] < errs[1] < errs[0]
    assert errs[2] < 2e-3
