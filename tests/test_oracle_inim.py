"""Pins of the oracle's integral images (Background, "Integral Images",
eq.(1); node-based and tilted-wedge readings) against direct sums and
pixel-by-pixel clipping of the summation areas."""
import numpy as np
import pytest

from oracle import cartogram as oc
from tests.brute import rect_mass, wedge_mass


def _dyadic(N, seed):
    rng = np.random.default_rng(seed)
    return rng.integers(0, 64, size=(N, N)) / 8.0


@pytest.mark.parametrize("N", [4, 8])
def test_axis_aligned_vs_direct_sums(N):
    d = _dyadic(N, N)
    im = oc.integral_images(d)
    a, b, g, dl, *_ = oc.eight_inims(im)
    for j in range(N + 1):
        for i in range(N + 1):
            assert im.S[j, i] == rect_mass(d, 0, i, 0, j)           # alpha: top-left
            assert b[j, i] == rect_mass(d, 0, i, j, N)               # beta: bottom-left
            assert g[j, i] == rect_mass(d, i, N, j, N)               # gamma: bottom-right
            assert dl[j, i] == rect_mass(d, i, N, 0, j)              # delta: top-right


@pytest.mark.parametrize("N,seed", [(5, 1), (6, 2), (8, 3)])
def test_tilted_vs_wedge_clipping(N, seed):
    d = np.random.default_rng(seed).random((N, N))
    im = oc.integral_images(d)
    a, b, g, dl, at, bt, gt, dt = oc.eight_inims(im)
    for j in range(N + 1):
        for i in range(N + 1):
            assert abs(at[j, i] - wedge_mass(d, i, j, 'top')) < 1e-12
            assert abs(bt[j, i] - wedge_mass(d, i, j, 'left')) < 1e-12
            assert abs(gt[j, i] - wedge_mass(d, i, j, 'bottom')) < 1e-12
            assert abs(dt[j, i] - wedge_mass(d, i, j, 'right')) < 1e-12


def test_partition_and_marginal_ends():
    N = 32
    d = np.random.default_rng(5).random((N, N))
    im = oc.integral_images(d)
    ims = oc.eight_inims(im)
    C = d.sum()
    assert abs(im.C - C) < 1e-10
    assert abs(sum(ims[:4]) - C).max() < 1e-10       # eq.(1), axis-aligned
    assert abs(sum(ims[4:]) - C).max() < 1e-10       # eq.(1), tilted
    assert min(x.min() for x in ims) > -1e-10         # every summation area is non-negative
    assert im.HA[0] == 0 and abs(im.HA[2 * N] - C) < 1e-10
    assert im.HB[0] == 0 and abs(im.HB[2 * N] - C) < 1e-10
    # HA[s] + mass(x'+y' >= s) = C and monotone marginals
    assert np.all(np.diff(im.HA) >= -1e-12) and np.all(np.diff(im.HB) >= -1e-12)


def test_flip_and_transpose_relations():
    N = 16
    d = np.random.default_rng(7).random((N, N))
    a, b, g, dl, at, bt, gt, dt = oc.eight_inims(oc.integral_images(d))
    # mirror x -> 1-x: top/bottom wedges mirror, left <-> right
    f = oc.eight_inims(oc.integral_images(d[:, ::-1]))
    np.testing.assert_allclose(f[4], at[:, ::-1], atol=1e-10)
    np.testing.assert_allclose(f[5], dt[:, ::-1], atol=1e-10)
    np.testing.assert_allclose(f[7], bt[:, ::-1], atol=1e-10)
    np.testing.assert_allclose(f[6], gt[:, ::-1], atol=1e-10)
    # transpose (swap x and y): top <-> left, bottom <-> right
    t = oc.eight_inims(oc.integral_images(d.T))
    np.testing.assert_allclose(t[4], bt.T, atol=1e-10)
    np.testing.assert_allclose(t[5], at.T, atol=1e-10)
    np.testing.assert_allclose(t[6], dt.T, atol=1e-10)
    np.testing.assert_allclose(t[7], gt.T, atol=1e-10)
