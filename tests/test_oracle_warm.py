"""Pins of the oracle's graded warm start (`warm_start_choose`): maps and
fields built by hand so that every trial step's areas, max area error and
fold status follow from the geometry, in dyadic coordinates where the
comparison has to be exact.

The rule being pinned: the trial steps alpha = 1, 3/4, 1/2, 1/4 are
tried in that order; a step whose moved map has a pixel centre claimed by
two regions is rejected; among the others the lowest max area error wins
if it is strictly below the plain start's; on a tie the earlier step is
kept; otherwise alpha = 0 and the plain start is returned.
"""
import numpy as np

from oracle import cartogram as oc
from synth import PlanarMap


def _two_rects(e: float) -> PlanarMap:
    """Regions 1 = [1/4, e] x [1/4, 3/4] and 2 = [e, 3/4] x [1/4, 3/4],
    sharing the edge x = e (vertices 1 and 2)."""
    xy = np.array([[0.25, 0.25], [e, 0.25], [e, 0.75], [0.25, 0.75], [0.75, 0.25], [0.75, 0.75]])
    return PlanarMap(xy=xy, ring_off=np.array([0, 4, 8], np.int32),
                     ring_idx=np.array([0, 1, 2, 3, 1, 4, 5, 2], np.int32),
                     ring_reg=np.array([1, 2], np.int32), n_regions=2)


def _column_field(G: int, cols, d) -> np.ndarray:
    f = np.zeros((G, G, 2))
    for i in cols:
        f[:, i] = d
    return f


def test_tie_keeps_the_earlier_step():
    # equal values: desired areas are 1/8 each.  The shared edge starts at
    # x = 25/64 (max area error 7/16) and the field moves it by alpha/8: the
    # step 1 overshoots to 33/64 and the step 3/4 undershoots to 31/64 by
    # the same 1/64, so both have max area error exactly 1/16 (every
    # coordinate and area here is dyadic, so the comparison is exact)
    m = _two_rects(25 / 64)
    s = np.array([1.0, 1.0])
    # G = 16: x = 25/64 falls between the centres of columns 5 and 6 and
    # x = 1/4, 3/4 between columns 3, 4 and 11, 12, so only the shared edge moves
    field = _column_field(16, (5, 6), (0.125, 0.0))
    xi_plain = oc.cartographic_errors(oc.region_areas(m.xy, m.ring_off, m.ring_idx, m.ring_reg, 2), s)[1]
    assert xi_plain == 0.4375
    for alpha, xi in ((1.0, 0.0625), (0.75, 0.0625), (0.5, 0.1875), (0.25, 0.3125)):
        moved = oc.warm_start_move(m.xy, alpha * field)
        assert moved[1, 0] == 25 / 64 + alpha / 8 and np.array_equal(moved[[0, 3, 4, 5]], m.xy[[0, 3, 4, 5]])
        A = oc.region_areas(moved, m.ring_off, m.ring_idx, m.ring_reg, 2)
        assert oc.cartographic_errors(A, s)[1] == xi
    alpha, xy = oc.warm_start_choose(m, s, 64, m.xy, field)
    assert alpha == 1.0
    assert xy[1, 0] == 33 / 64 and xy[2, 0] == 33 / 64


def test_lowest_error_wins():
    # values 3 : 5 (desired areas 3/32 and 5/32): the edge must move from
    # x = 1/2 to 7/16, i.e. by -1/16 = alpha * (-1/8) at alpha = 1/2
    m = _two_rects(0.5)
    s = np.array([3.0, 5.0])
    field = _column_field(16, (7, 8), (-0.125, 0.0))     # x = 1/2 lies between the centres of columns 7 and 8
    alpha, xy = oc.warm_start_choose(m, s, 64, m.xy, field)
    assert alpha == 0.5
    assert xy[1, 0] == 0.4375 and xy[2, 0] == 0.4375
    A = oc.region_areas(xy, m.ring_off, m.ring_idx, m.ring_reg, 2)
    assert A[1] == 3 / 32 and A[2] == 5 / 32


def test_field_that_helps_nothing_gives_the_plain_start():
    m = _two_rects(25 / 64)
    s = np.array([1.0, 1.0])
    # a translation of the whole map by 1/16 leaves every area (exactly) unchanged
    shift = np.zeros((16, 16, 2))
    shift[..., 0] = 0.0625
    alpha, xy = oc.warm_start_choose(m, s, 64, m.xy, shift)
    assert alpha == 0.0 and np.array_equal(xy, m.xy)
    # a field that moves the shared edge the wrong way makes every step worse
    wrong = _column_field(16, (5, 6), (-0.0625, 0.0))
    alpha, xy = oc.warm_start_choose(m, s, 64, m.xy, wrong)
    assert alpha == 0.0 and np.array_equal(xy, m.xy)


def _three_rects_with_spike() -> PlanarMap:
    """Regions 1 = [0.2, 0.4], 2 = [0.4, 0.6], 3 = [0.6, 0.8] (x) times
    [0.2, 0.8] (y); the edge between 1 and 2 has a middle vertex (0.4, 0.5)
    (id 2) that a field can push towards region 3."""
    xy = np.array([[0.2, 0.2], [0.4, 0.2], [0.4, 0.5], [0.4, 0.8], [0.2, 0.8],
                   [0.6, 0.2], [0.6, 0.8], [0.8, 0.2], [0.8, 0.8]])
    ring_idx = np.array([0, 1, 2, 3, 4,
                         1, 5, 6, 3, 2,
                         5, 7, 8, 6], np.int32)
    return PlanarMap(xy=xy, ring_off=np.array([0, 5, 10, 14], np.int32), ring_idx=ring_idx,
                     ring_reg=np.array([1, 2, 3], np.int32), n_regions=3)


def test_folding_step_is_rejected_even_with_the_lowest_error():
    m = _three_rects_with_spike()
    # G = 20: the spike vertex (0.4, 0.5) sits between the centres of
    # columns 7, 8 and rows 9, 10; no other vertex touches those cells
    field = np.zeros((20, 20, 2))
    field[9:11, 7:9] = (0.25, 0.0)
    # pushing the spike by t moves the triangle area 0.5 * 0.6 * t from
    # region 2 to region 1; the values are the areas at t = 1/4, so the
    # step alpha = 1 has zero area error -- but its tip passes x = 0.6 and
    # covers pixel centres of region 3 (at N = 64 e.g. the centre
    # (38.5, 31.5) / 64 lies right of x = 0.6 and left of the spike edge
    # from (0.4, 0.2) to (0.65, 0.5)): a fold
    s = np.array([0.12 + 0.3 * 0.25, 0.12 - 0.3 * 0.25, 0.12])
    full = oc.warm_start_move(m.xy, field)
    assert np.allclose(full[2], (0.65, 0.5)) and np.array_equal(np.delete(full, 2, 0), np.delete(m.xy, 2, 0))
    assert oc.cartographic_errors(oc.region_areas(full, m.ring_off, m.ring_idx, m.ring_reg, 3), s)[1] < 1e-12
    px, py = 38.5 / 64, 31.5 / 64
    x_edge = 0.4 + 0.25 * (py - 0.2) / 0.3
    assert 0.6 < px < x_edge
    lab, _, conflicts = oc.rasterize(full, m.ring_off, m.ring_idx, m.ring_reg, 3, 64)
    assert conflicts > 0 and lab[31, 38] == 3          # claimed by all three; the highest id is kept
    # the other steps do not fold; by hand, their max area errors are
    # 0.01875/0.06375 (3/4), 0.0375/0.0825 (1/2), 0.05625/0.10125 (1/4)
    # against 0.075/0.12 for the plain start: alpha = 3/4 wins
    alpha, xy = oc.warm_start_choose(m, s, 64, m.xy, field)
    assert alpha == 0.75
    assert np.allclose(xy[2], (0.4 + 0.75 * 0.25, 0.5))
    for a, want in ((0.75, 0.01875 / 0.06375), (0.5, 0.0375 / 0.0825), (0.25, 0.05625 / 0.10125)):
        xi = oc.cartographic_errors(oc.region_areas(oc.warm_start_move(m.xy, a * field), m.ring_off, m.ring_idx,
                                                    m.ring_reg, 3), s)[1]
        assert abs(xi - want) < 1e-12, (a, xi, want)
