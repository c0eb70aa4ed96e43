"""Pins of the oracle's time-varying forms (Method, "Coherence of Dynamic
Cartograms" and "Interactive Steering"): the background mass of eq.(4)
by hand values and by its defining property (the map's share of the
domain follows the prescribed area fraction once the density is
equalised), its reduction to the plain background density, and
value-interpolated transition frames against single runs."""
import numpy as np
import pytest

from oracle import cartogram as oc
from synth import lognormal_values, square_grid_map, voronoi_map


def test_background_mass_hand_values():
    # totals 2, 5, 8 over two regions; A_min = 0.2, A_max = 0.8:
    # w = 0, 1/2, 1 -> A_i = 0.2, 0.5, 0.8 -> M_b = M (1 - A) / A = 8, 5, 2
    S = np.array([[1.5, 0.5], [4.0, 1.0], [2.0, 6.0]])
    Mb, A = oc.background_masses(S, 0.2, 0.8)
    assert np.allclose(A, [0.2, 0.5, 0.8], atol=1e-15)
    assert np.allclose(Mb, [8.0, 5.0, 2.0], rtol=1e-14)
    Mi = S.sum(1)
    assert np.allclose(Mi / (Mi + Mb), A, atol=1e-15)
    # extremes over steps 1..2 only: step 0 lies below the range, w clamps to 0
    Mb, A = oc.background_masses(S, 0.2, 0.8, 1, 2)
    assert np.allclose(A, [0.2, 0.2, 0.8], atol=1e-15)
    # constant total: w = 1, the map keeps A_max of the domain
    Mb, A = oc.background_masses(np.ones((3, 4)), 0.3, 0.9)
    assert np.allclose(A, 0.9) and np.allclose(Mb, 4 * 0.1 / 0.9, rtol=1e-14)
    # evaluation at in-between totals
    Mb, A = oc.background_masses(S, 0.2, 0.8, at=[3.5])
    assert A[0] == pytest.approx(0.35, abs=1e-15) and Mb[0] == pytest.approx(3.5 * 0.65 / 0.35, rel=1e-14)


def test_background_mass_of_the_plain_density_gives_the_plain_iteration():
    m = voronoi_map(1000, 32, 2000, fractal=False)
    s = lognormal_values(1000, 32, 1.0)
    N = 128
    lab, cnt, _ = oc.rasterize(m.xy, m.ring_off, m.ring_idx, m.ring_reg, 32, N)
    b = 1.03
    lut, d0 = oc.density_lut(cnt, s, b)
    lut2, _ = oc.density_lut(cnt, s, b, bg_mass=d0 * cnt[0])
    assert lut2[0] == pytest.approx(lut[0], rel=1e-15) and np.array_equal(lut[1:], lut2[1:])
    # no background pixel: the mass has nowhere to go, the plain BDV is kept
    c0 = cnt.copy()
    c0[0] = 0
    assert oc.density_lut(c0, s, b, bg_mass=5.0)[0][0] == b * oc.density_lut(c0, s, b)[1]


def test_map_area_follows_the_prescribed_fraction():
    # equalised density: the map's share of the domain is M_i / (M_i + M_b) = A_i(t)
    m = square_grid_map(3, 8)
    rng = np.random.default_rng(5)
    s0 = np.exp(rng.normal(0, 0.5, 9))
    S = np.stack([s0, 3 * s0 * np.exp(rng.normal(0, 0.1, 9))])
    out, _ = oc.run_series(m, S, 128, mode="direct", area_fraction=(0.3, 0.7), fixed_iters=20)
    fr = [oc.region_areas(r.xy, m.ring_off, m.ring_idx, m.ring_reg, 9)[1:].sum() for r in out]
    assert abs(fr[0] - 0.3) < 0.002 and abs(fr[1] - 0.7) < 0.002
    # the plain background density keeps the map near its original share (0.25)
    plain, _ = oc.run_series(m, S, 128, mode="direct", fixed_iters=20)
    fp = [oc.region_areas(r.xy, m.ring_off, m.ring_idx, m.ring_reg, 9)[1:].sum() for r in plain]
    assert all(abs(f - 0.25) < 0.02 for f in fp)


@pytest.mark.parametrize("mode", ["direct", "cumulative"])
def test_value_frames_are_cartograms_of_interpolated_values(mode):
    m = square_grid_map(2, 4)
    rng = np.random.default_rng(9)
    S = np.exp(rng.normal(0, 0.6, (3, 4)))
    K = 4
    kw = dict(fixed_iters=3)
    out, frames = oc.run_series(m, S, 64, mode=mode, frames_per_step=K, frame_mode="values", **kw)
    assert len(out) == 3 and len(frames) == 2 and frames[0].shape == (K - 1, m.n_vertices, 2)
    # frame 2 of transition 1 -> 2 (values 1/2 s_1 + 1/2 s_2)
    mid = 0.5 * S[1] + 0.5 * S[2]
    start = m.xy if mode == "direct" else frames[1][0]
    want = oc.run(m, mid, 64, xy0=start, **kw).xy
    assert np.array_equal(frames[1][1], want)
    if mode == "direct":
        # the steps equal a series without frames
        plain, _ = oc.run_series(m, S, 64, mode="direct", **kw)
        assert all(np.array_equal(a.xy, b.xy) for a, b in zip(out, plain))
    else:
        # step 1 starts from the last frame of transition 0 -> 1
        want1 = oc.run(m, S[1], 64, xy0=frames[0][-1], **kw).xy
        assert np.array_equal(out[1].xy, want1)
