"""Failure handling through the C ABI, every condition forced from the host
so that each kernel still runs to its normal end: invalid topology is
rejected before anything is launched, values that define no density end
the step with CG_STATUS_ERROR before any iteration, and the iteration cap
ends a run with CG_STATUS_MAXITER."""
import ctypes as C

import numpy as np
import pytest

from synth import lognormal_values, square_grid_map, voronoi_map

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2604_13880_amd import binding as B
    c = B.Context(0)
    yield c
    c.close()


def test_edge_in_three_rings_is_rejected(ctx):
    from paper_2604_13880_amd import binding as B
    # three triangles on the edge 0-1: that edge has three owners
    ring_off = np.array([0, 3, 6, 9], np.int32)
    ring_idx = np.array([0, 1, 2, 1, 0, 3, 0, 1, 4], np.int32)
    ring_reg = np.array([1, 2, 3], np.int32)
    h = C.c_void_p()
    rc = B.lib().cg_map_build(ctx.handle, 5, 3, 3, ring_off.ctypes.data_as(C.c_void_p),
                              ring_idx.ctypes.data_as(C.c_void_p), ring_reg.ctypes.data_as(C.c_void_p),
                              C.byref(h))
    assert rc == -1 and not h.value
    assert "more than two rings" in B.lib().cg_last_error(ctx.handle).decode()
    with pytest.raises(B.CartogramError):
        ctx.map_build(ring_off, ring_idx, ring_reg, 5, 3)


@pytest.mark.parametrize("bad", ["index", "region", "short_ring"])
def test_bad_ring_tables_are_rejected(ctx, bad):
    from paper_2604_13880_amd import binding as B
    m = square_grid_map(2, 2)
    ro, ri, rr = m.ring_off.copy(), m.ring_idx.copy(), m.ring_reg.copy()
    if bad == "index":
        ri[3] = m.n_vertices
    elif bad == "region":
        rr[1] = m.n_regions + 1
    else:
        ro[1] = 2          # the first ring keeps two vertices
    with pytest.raises(B.CartogramError):
        ctx.map_build(ro, ri, rr, m.n_vertices, m.n_regions)


@pytest.mark.parametrize("kind", ["nan", "inf", "negative", "zero"])
def test_values_without_a_density_end_with_an_error(ctx, kind):
    from paper_2604_13880_amd import binding as B
    m = voronoi_map(1000, 32, 2000, fractal=False)
    s = lognormal_values(1000, 32, 1.0).astype(np.float32)
    if kind == "nan":
        s[5] = np.nan
    elif kind == "inf":
        s[0] = np.inf
    elif kind == "negative":
        s[31] = -1.0
    else:
        s[:] = 0.0
    gm = ctx.map_from(m)
    good = lognormal_values(1001, 32, 1.0).astype(np.float32)
    res = ctx.step_series([dict(map=gm, xy0=m.xy32(), N=256, values=np.stack([good, s]))])[0]
    assert res["status"][1] == B.STATUS_ERROR and res["iters"][1] == 0
    assert res["flags"][1] & B.FLAG_BADVALUES
    # nothing moved: the step's output is its starting map
    assert np.array_equal(res["xy"][1].cpu().numpy(), m.xy32())
    # the good step of the same batch is unaffected
    assert res["status"][0] != B.STATUS_ERROR and res["iters"][0] > 0
    assert not res["flags"][0] & B.FLAG_BADVALUES


def test_iteration_cap_of_one(ctx):
    from paper_2604_13880_amd import binding as B
    m = voronoi_map(1000, 32, 2000, fractal=False)
    s = lognormal_values(1000, 32, 1.0).astype(np.float32)
    gm = ctx.map_from(m)
    r = ctx.step_series([dict(map=gm, xy0=m.xy32(), N=256, values=s, max_iters=1)])[0]
    assert r["status"][0] == B.STATUS_MAXITER and r["iters"][0] == 1
    r0 = ctx.step_series([dict(map=gm, xy0=m.xy32(), N=256, values=s, max_iters=0)])[0]
    assert r0["status"][0] == B.STATUS_MAXITER and r0["iters"][0] == 0
    assert np.array_equal(r0["xy"][0].cpu().numpy(), m.xy32())


def test_bad_series_arguments_are_rejected_before_launch(ctx):
    from paper_2604_13880_amd import binding as B
    m = square_grid_map(2, 2)
    gm = ctx.map_from(m)
    s = np.ones(m.n_regions, np.float32)
    for kw in (dict(N=100), dict(N=8), dict(precision=7), dict(mode=3), dict(tol=0.0), dict(shape=-1.0),
               dict(area_source=5), dict(max_iters=-1)):
        d = dict(map=gm, xy0=m.xy32(), N=64, values=s)
        d.update(kw)
        with pytest.raises(B.CartogramError):
            ctx.step_series([d])


def test_map_destroyed_after_its_context():
    """A map freed after its context leaves no device error behind: the next
    context's launches run (regression: the map read its device through the
    freed context)."""
    from paper_2604_13880_amd import binding as B
    m = square_grid_map(2, 2)
    c1 = B.Context(0)
    gm = c1.map_from(m)
    c1.close()
    del gm
    import gc
    gc.collect()
    c2 = B.Context(0)
    g2 = c2.map_from(m)
    r = c2.step_series([dict(map=g2, xy0=m.xy32(), N=64, values=np.ones(4, np.float32), fixed_iters=1)])[0]
    assert r["iters"][0] == 1
    c2.close()
