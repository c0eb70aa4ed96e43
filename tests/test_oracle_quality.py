"""Pins of the oracle's geographic-distortion measures (Background,
"Quality Measures"): hand-built label images with known adjacencies and
overlaps, brute-force translation search against the FFT search, exact
centroids of simple polygons, and rotations whose relative position error
is known in closed form."""
import math

import numpy as np
import pytest

from oracle import cartogram as oc
from oracle import quality as oq
from synth import PlanarMap, square_grid_map, voronoi_map


def test_adjacency_of_a_grid_map():
    # 3 x 3 squares: 6 horizontal and 6 vertical neighbour pairs; corners
    # touching only at a point are not neighbours
    m = square_grid_map(3, 4)
    lab, _, _ = oc.rasterize(m.xy, m.ring_off, m.ring_idx, m.ring_reg, m.n_regions, 64)
    E = oq.adjacency(lab)
    assert len(E) == 12
    ids = lab[lab > 0]
    assert set(np.unique(ids)) == set(range(1, 10))
    # regions sharing a side have centres one square apart
    cx = {v: np.argwhere(lab == v).mean(0) for v in range(1, 10)}
    for u, v in E:
        d = np.abs(cx[u] - cx[v])
        assert min(d) < 1 and 8 < max(d) < 24
    assert oq.topology_distortion(lab, lab) == (0.0, 12, 12, 12)


def test_topology_distortion_by_hand():
    a = np.array([[1, 1, 2, 2, 3, 3],
                  [1, 1, 2, 2, 3, 3]])              # E = {(1,2), (2,3)}
    b = np.array([[1, 1, 0, 2, 2, 0],
                  [3, 3, 0, 0, 0, 0]])              # E = {(1,3)}; 1 and 2 separated by background
    tau, nm, nc, common = oq.topology_distortion(a, b)
    assert (nm, nc, common) == (2, 1, 0) and tau == 1.0
    c = np.array([[1, 2, 0, 3],
                  [1, 1, 1, 3]])                    # E = {(1,2), (1,3)}
    tau, nm, nc, common = oq.topology_distortion(a, c)
    assert (nm, nc, common) == (2, 2, 1) and tau == pytest.approx(2 / 3, abs=1e-15)
    assert oq.topology_distortion(np.zeros((4, 4), int), np.zeros((4, 4), int))[0] == 0.0


def _square(n, side, y0, x0):
    z = np.zeros((n, n), bool)
    z[y0:y0 + side, x0:x0 + side] = True
    return z


def test_overlap_closed_forms():
    a = _square(32, 3, 2, 5)
    b = _square(32, 6, 20, 11)
    # a square fits inside the doubled square: best overlap 9,
    # distortion (9 + 36 - 18) / (9 + 36 - 9) = 3/4
    assert oq.best_overlap_bruteforce(a, b) == 9 == oq.best_overlap(a, b)
    assert oq.shape_ratio(9, 36, 9) == 0.75
    # a translated copy overlaps itself completely: distortion 0
    c = np.roll(np.roll(a, 7, 0), -3, 1)
    assert oq.best_overlap(a, c) == 9 and oq.shape_ratio(9, 9, 9) == 0.0
    # an L of three unit squares against a 2 x 2 square: best overlap 3
    L = np.zeros((8, 8), bool)
    L[1, 1] = L[2, 1] = L[2, 2] = True
    assert oq.best_overlap_bruteforce(L, _square(8, 2, 4, 4)) == 3 == oq.best_overlap(L, _square(8, 2, 4, 4))
    assert oq.shape_ratio(3, 4, 3) == pytest.approx(1 / 4, abs=1e-16)
    # empty sets
    z = np.zeros((8, 8), bool)
    assert oq.best_overlap(z, L) == 0 and oq.shape_ratio(0, 3, 0) == 1.0 and oq.shape_ratio(0, 0, 0) == 0.0


def test_fft_search_equals_brute_force_on_random_shapes():
    rng = np.random.default_rng(3)
    for _ in range(12):
        a = rng.random((rng.integers(3, 14), rng.integers(3, 14))) < 0.5
        b = rng.random((rng.integers(3, 14), rng.integers(3, 14))) < 0.5
        A = np.zeros((24, 24), bool)
        B = np.zeros((24, 24), bool)
        A[2:2 + a.shape[0], 5:5 + a.shape[1]] = a
        B[9:9 + b.shape[0], 1:1 + b.shape[1]] = b
        assert oq.best_overlap(A, B) == oq.best_overlap_bruteforce(A, B)


def test_shape_distortion_of_a_small_deformed_map():
    m = voronoi_map(31, 7, 200, fractal=True)
    s = np.exp(np.random.default_rng(31).normal(0, 1, 7))
    r = oc.run(m, s, 64, fixed_iters=6)
    lm, _, _ = oc.rasterize(m.xy, m.ring_off, m.ring_idx, m.ring_reg, 7, 64)
    lc, _, _ = oc.rasterize(r.xy, m.ring_off, m.ring_idx, m.ring_reg, 7, 64)
    H, hm, hx, best = oq.shape_distortion(lm, lc, 7)
    Hb, _, _, bestb = oq.shape_distortion(lm, lc, 7, brute=True)
    assert np.array_equal(best, bestb) and np.array_equal(H, Hb)
    assert 0 < hm <= hx < 1 and H[0] == 0
    H0, hm0, hx0, _ = oq.shape_distortion(lm, lm, 7)
    assert hm0 == 0 and hx0 == 0


def test_barycenters_of_simple_polygons():
    # region 1: unit-area-scaled rectangle; region 2: triangle; region 3:
    # an L made of two rings (two rectangles)
    xy = np.array([[0.1, 0.1], [0.5, 0.1], [0.5, 0.3], [0.1, 0.3],
                   [0.6, 0.6], [0.9, 0.6], [0.6, 0.9],
                   [0.1, 0.5], [0.3, 0.5], [0.3, 0.9], [0.1, 0.9],
                   [0.3, 0.7], [0.5, 0.7], [0.5, 0.9]])
    ring_off = np.array([0, 4, 7, 11, 15], np.int32)
    ring_idx = np.array([0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 11, 12, 13, 9], np.int32)
    ring_reg = np.array([1, 2, 3, 3], np.int32)
    b = oq.barycenters(xy, ring_off, ring_idx, ring_reg, 3)
    assert np.allclose(b[1], (0.3, 0.2), atol=1e-15)
    assert np.allclose(b[2], (0.7, 0.7), atol=1e-15)
    # L: 0.2 x 0.4 at centre (0.2, 0.7) plus 0.2 x 0.2 at (0.4, 0.8)
    assert np.allclose(b[3], ((0.08 * 0.2 + 0.04 * 0.4) / 0.12, (0.08 * 0.7 + 0.04 * 0.8) / 0.12), atol=1e-15)


def _rot(b, th, c=(0.5, 0.5)):
    out = b.copy()
    d = b[1:] - c
    out[1:, 0] = c[0] + math.cos(th) * d[:, 0] - math.sin(th) * d[:, 1]
    out[1:, 1] = c[1] + math.sin(th) * d[:, 0] + math.cos(th) * d[:, 1]
    return out


def test_relative_position_error_closed_forms():
    rng = np.random.default_rng(7)
    b = np.zeros((13, 2))
    b[1:] = rng.random((12, 2))
    assert oq.relative_position_error(b, b) == 0.0
    # a similarity without rotation keeps every direction
    sim = b.copy()
    sim[1:] = 0.3 + 0.5 * b[1:]
    assert oq.relative_position_error(b, sim) < 1e-15
    # a rotation by theta turns every vector by theta: R = theta / pi
    for th in (0.3, math.pi / 2, 2.5):
        assert oq.relative_position_error(b, _rot(b, th)) == pytest.approx(th / math.pi, abs=1e-13)
    # two regions swapping a horizontal for a vertical offset: both
    # ordered pairs turn by pi/2, R = (2 * pi/2) / (pi * 2 * 1) = 1/2
    bm = np.array([[0, 0], [0.2, 0.5], [0.8, 0.5]])
    bc = np.array([[0, 0], [0.5, 0.2], [0.5, 0.8]])
    assert oq.relative_position_error(bm, bc) == pytest.approx(0.5, abs=1e-15)


def test_quality_of_the_map_itself_is_zero():
    m = voronoi_map(1000, 32, 2000, fractal=False)
    q = oq.quality(m, m.xy, m.xy, 128)
    assert q["tau"] == 0.0 and q["shape_mean"] == 0.0 and q["shape_max"] == 0.0 and q["rel_pos"] == 0.0
    assert q["adj_map"] == q["adj_cart"] == q["adj_common"] > 32
