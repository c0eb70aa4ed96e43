"""Pins of the oracle's eight-anchor map and DET (Background, eqs.(2),
(3); Method, Steps 1, 5, 6) against hand-derived values, a closed form
and exact symmetries."""
import os

import numpy as np
import pytest

from oracle import cartogram as oc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(kind):
    rows = []
    for line in open(os.path.join(GOLDEN, "det_worked_values.txt")):
        parts = line.split()
        if parts and parts[0] == kind:
            rows.append([float(v) for v in parts[1:]])
    return rows


def t0_closed_form(x, y):
    """Uniform-density map: quadrant areas are products, wedge areas are
    squares minus the parts cut off by the domain border (derived from the
    wedge geometry, m(z) = max(z, 0)^2)."""
    m = lambda z: np.maximum(z, 0.0) ** 2
    a, b, g, dl = x * y, x * (1 - y), (1 - x) * (1 - y), (1 - x) * y
    at = y**2 - 0.5 * m(y - x) - 0.5 * m(x + y - 1)
    bt = x**2 - 0.5 * m(x - y) - 0.5 * m(x + y - 1)
    gt = (1 - y) ** 2 - 0.5 * m(1 - x - y) - 0.5 * m(x - y)
    dt = (1 - x) ** 2 - 0.5 * m(1 - x - y) - 0.5 * m(y - x)
    lowx = y < x
    low = x + y < 1
    q1 = (np.where(lowx, 1.0, 1 - y + x), np.where(lowx, 1 + y - x, 1.0))
    q3 = (np.where(lowx, x - y, 0.0), np.where(lowx, 0.0, y - x))
    q2 = (np.where(low, x + y, 1.0), np.where(low, 0.0, x + y - 1))
    q4 = (np.where(low, 0.0, x + y - 1), np.where(low, x + y, 1.0))
    tx = a * q1[0] + b * q2[0] + g * q3[0] + dl * q4[0] + at * x + bt + gt * x
    ty = a * q1[1] + b * q2[1] + g * q3[1] + dl * q4[1] + at + bt * y + dt * y
    return tx / 2, ty / 2


@pytest.mark.parametrize("N", [8, 64])
def test_uniform_map_worked_values(N):
    tx, ty = oc.t_uniform(N)
    for x, y, ex, ey in _golden("t0"):
        i, j = int(round(x * N)), int(round(y * N))
        assert abs(tx[j, i] - ex) < 1e-14 and abs(ty[j, i] - ey) < 1e-14


@pytest.mark.parametrize("N", [16, 128])
def test_uniform_map_closed_form(N):
    tx, ty = oc.t_uniform(N)
    jj, ii = np.mgrid[0:N + 1, 0:N + 1]
    cx, cy = t0_closed_form(ii / N, jj / N)
    assert np.abs(tx - cx).max() < 1e-13 and np.abs(ty - cy).max() < 1e-13


@pytest.mark.parametrize("N", [8, 32])
def test_heavy_quadrant_displacement(N):
    for a, ex, ey in _golden("quad"):
        d = np.ones((N, N))
        d[: N // 2, : N // 2] = a
        Dx, Dy = oc.displacement(oc.integral_images(d))
        assert abs(Dx[N // 2, N // 2] - ex) < 1e-14 and abs(Dy[N // 2, N // 2] - ey) < 1e-14


@pytest.mark.parametrize("c", [1.0, 3.7, 1e-3])
def test_uniform_density_is_a_fixed_point(c):
    Dx, Dy = oc.displacement(oc.integral_images(np.full((32, 32), c)))
    assert np.abs(Dx).max() < 1e-14 and np.abs(Dy).max() < 1e-14


def test_border_invariance_and_symmetries():
    N = 32
    d = np.random.default_rng(3).lognormal(0, 1, (N, N))
    Dx, Dy = oc.displacement(oc.integral_images(d))
    assert np.abs(Dx[:, 0]).max() < 1e-14 and np.abs(Dx[:, N]).max() < 1e-14
    assert np.abs(Dy[0, :]).max() < 1e-14 and np.abs(Dy[N, :]).max() < 1e-14
    fx, fy = oc.displacement(oc.integral_images(d[:, ::-1]))        # mirror x
    np.testing.assert_allclose(fx, -Dx[:, ::-1], atol=1e-13)
    np.testing.assert_allclose(fy, Dy[:, ::-1], atol=1e-13)
    gx, gy = oc.displacement(oc.integral_images(d[::-1, :]))        # mirror y
    np.testing.assert_allclose(gx, Dx[::-1, :], atol=1e-13)
    np.testing.assert_allclose(gy, -Dy[::-1, :], atol=1e-13)
    tx, ty = oc.displacement(oc.integral_images(d.T))               # transpose
    np.testing.assert_allclose(tx, Dy.T, atol=1e-13)
    np.testing.assert_allclose(ty, Dx.T, atol=1e-13)


def test_move_points_bilinear():
    N = 16
    jj, ii = np.mgrid[0:N + 1, 0:N + 1]
    # a bilinear field is reproduced exactly; nodes get their own value
    Fx = 0.01 * (ii / N) * (jj / N) - 0.003 * (ii / N)
    Fy = 0.002 + 0.004 * (jj / N)
    rng = np.random.default_rng(0)
    pts = np.concatenate([rng.random((50, 2)) * 0.9 + 0.05,
                          np.stack([ii.ravel() / N, jj.ravel() / N], 1)])
    out = oc.move_points(pts, Fx, Fy)
    ex = np.clip(pts[:, 0] + 0.01 * pts[:, 0] * pts[:, 1] - 0.003 * pts[:, 0], 0, 1)
    ey = np.clip(pts[:, 1] + 0.002 + 0.004 * pts[:, 1], 0, 1)
    assert np.abs(out[:, 0] - ex).max() < 1e-15 and np.abs(out[:, 1] - ey).max() < 1e-15


def test_warm_start_move_reproduces_affine_fields_and_extends_constantly():
    G = 8
    grid = oc.tracer_grid(G).reshape(G, G, 2)
    assert np.allclose(grid[0, 0], [0.5 / G, 0.5 / G]) and np.allclose(grid[0, 1], [1.5 / G, 0.5 / G])
    # affine field sampled at the centres
    field = np.stack([0.02 * grid[..., 0] - 0.01 * grid[..., 1] + 0.003,
                      -0.015 * grid[..., 0] + 0.01], axis=-1)
    rng = np.random.default_rng(4)
    inner = 0.5 / G + (1 - 1.0 / G) * rng.random((200, 2))
    want = inner + np.stack([0.02 * inner[:, 0] - 0.01 * inner[:, 1] + 0.003,
                             -0.015 * inner[:, 0] + 0.01], axis=1)
    assert np.allclose(oc.warm_start_move(inner, field), want, atol=1e-15)
    # beyond the outermost centres the field is held constant (corner value)
    corner = np.array([[0.01, 0.02]])
    assert np.allclose(oc.warm_start_move(corner, field), corner + field[0, 0], atol=1e-15)
    # clamped to the unit square
    big = np.full((G, G, 2), 5.0)
    assert np.array_equal(oc.warm_start_move(inner, big), np.ones_like(inner))
    # a single cell is a constant shift
    assert np.allclose(oc.warm_start_move(inner, np.array([[[0.01, -0.02]]])), inner + [0.01, -0.02])


def test_log_density_mean_is_zero_in_linear_space():
    from synth import voronoi_map, lognormal_values
    m = voronoi_map(1000, 32, 2000, fractal=False)
    s = lognormal_values(1000, 32, 1.0)
    labels, counts, _ = oc.rasterize(m.xy, m.ring_off, m.ring_idx, m.ring_reg, m.n_regions, 64)
    ld = oc.log_density(labels, counts, s, b=1.0)
    assert abs(np.exp(ld).mean() - 1.0) < 1e-12
    # background pixels carry log(BDV / mean), region pixels log(s/o / mean)
    lut, d0 = oc.density_lut(counts, s, 1.0)
    mean = (lut[labels]).mean()
    assert np.allclose(ld[labels == 0], np.log(d0 / mean))
