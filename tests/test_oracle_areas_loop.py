"""Pins of the oracle's areas and cartographic errors (Background,
"Quality Measures"), its iteration and stopping rule (Method, Steps 2-7)
and the direct / cumulative series (Method, "Coherence of Dynamic
Cartograms")."""
import numpy as np
import pytest

from oracle import cartogram as oc
from synth import lognormal_values, random_walk_series, square_grid_map, voronoi_map
from tests.brute import segments_cross


def test_areas_exact_on_dyadic_shapes():
    xy = np.array([[0.125, 0.25], [0.625, 0.25], [0.625, 0.75], [0.125, 0.75],   # rect 0.5 x 0.5
                   [0.75, 0.125], [0.875, 0.125], [0.75, 0.5]])                  # right triangle
    ring_off = np.array([0, 4, 7])
    ring_idx = np.array([0, 1, 2, 3, 4, 5, 6])
    A = oc.region_areas(xy, ring_off, ring_idx, np.array([1, 2]), 2)
    assert A[1] == 0.25 and A[2] == 0.5 * 0.125 * 0.375 and A[0] == 1 - A[1] - A[2]


def test_cartographic_errors_hand_example():
    # areas 0.3 and 0.1 with equal values: w = 0.2 each
    eps, xi = oc.cartographic_errors(np.array([0.6, 0.3, 0.1]), np.array([1.0, 1.0]))
    assert abs(xi - 0.5) < 1e-15 and abs(eps - (1 / 3 + 1 / 2) / 2) < 1e-15


def test_voronoi_cells_tile_the_placed_square():
    m = voronoi_map(5, 40, 3000, fractal=True)
    A = oc.region_areas(m.xy, m.ring_off, m.ring_idx, m.ring_reg, m.n_regions)
    assert abs(A[1:].sum() - 0.81) < 1e-2      # the fractal outline moves area in and out
    assert np.all(A[1:] > 0)
    m2 = voronoi_map(5, 40, 3000, fractal=False)
    A2 = oc.region_areas(m2.xy, m2.ring_off, m2.ring_idx, m2.ring_reg, m2.n_regions)
    assert abs(A2[1:].sum() - 0.81) < 1e-6


def test_density_mass_balance():
    N = 64
    m = voronoi_map(8, 10, 300, fractal=True)
    s = lognormal_values(8, 10, 1.0)
    lab, cnt, conf = oc.rasterize(m.xy, m.ring_off, m.ring_idx, m.ring_reg, m.n_regions, N)
    lut, d0 = oc.density_lut(cnt, s, b=1.1)
    im = oc.integral_images(oc.density_texture(lab, lut))
    have = cnt[1:] > 0
    assert abs(d0 - s[have].sum() / cnt[1:].sum()) < 1e-15
    assert abs(im.C - (s[have].sum() + 1.1 * d0 * cnt[0])) < 1e-9 * im.C


def test_converges_and_keeps_topology():
    m = square_grid_map(3, 6)
    s = lognormal_values(0, 9, 0.25)
    res = oc.run(m, s, 256)
    assert res.status == oc.STATUS_CONVERGED and res.xi < 0.01 and res.iters < 80
    h = np.array(res.xi_history)
    assert h[-1] < 0.05 * h[0]
    assert np.all(oc.ring_areas(res.xy, m.ring_off, m.ring_idx) > 0)
    assert segments_cross(res.xy, m.ring_off, m.ring_idx) == 0


def test_pixel_count_floor_and_polygon_source():
    # pixel counts quantise small regions: at 64^2 the error stalls above 1%,
    # while densities from polygon areas keep converging (area-source reading)
    m = square_grid_map(3, 6)
    s = lognormal_values(0, 9, 0.25)
    pix = oc.run(m, s, 64, max_iters=120)
    poly = oc.run(m, s, 64, max_iters=120, area_source="polygon")
    assert pix.xi > 0.01 and poly.xi < 0.01 and poly.status == oc.STATUS_CONVERGED


def test_stopping_rule_semantics():
    m = square_grid_map(2, 2)
    s = lognormal_values(1, 4, 1.0)
    r = oc.run(m, s, 32, tol=1.0)
    assert r.iters == 0 and r.status == oc.STATUS_CONVERGED
    r = oc.run(m, s, 32, max_iters=3)
    assert r.iters == 3 and r.status == oc.STATUS_MAXITER and len(r.xi_history) == 4
    r = oc.run(m, s, 32, patience=0)
    assert r.iters == 0 and r.status == oc.STATUS_STALLED
    r = oc.run(m, s, 32, fixed_iters=5)
    assert r.iters == 5


def test_series_direct_cumulative_frames():
    m = square_grid_map(2, 3)
    S = random_walk_series(4, 4, 3, sigma0=0.5, step_sigma=0.1)
    kw = dict(max_iters=6)
    direct, _ = oc.run_series(m, S, 32, mode="direct", **kw)
    for t in range(3):
        single = oc.run(m, S[t], 32, **kw)
        assert np.array_equal(single.xy, direct[t].xy)
    cum, frames = oc.run_series(m, S, 32, mode="cumulative", frames_per_step=4, **kw)
    assert np.array_equal(cum[0].xy, direct[0].xy)
    again = oc.run(m, S[1], 32, xy0=cum[0].xy, **kw)
    assert np.array_equal(again.xy, cum[1].xy)
    assert len(frames) == 2 and frames[0].shape == (3,) + m.xy.shape
    np.testing.assert_allclose(frames[0][1], 0.5 * (cum[0].xy + cum[1].xy), atol=1e-15)
