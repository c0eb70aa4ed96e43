"""GPU parity: every C-ABI call against the FP64 oracle on the same seeded
inputs (labels and counts bit-exact; floating point within bounds derived
from the storage and accumulation precision of each mode)."""
import os
import sys

import numpy as np
import pytest

from oracle import cartogram as oc
from synth import lognormal_values, square_grid_map, voronoi_map

pytestmark = pytest.mark.gpu

# |S - S_oracle| / C and |T - T_oracle| / C bounds per accumulation mode
INIM_TOL = {0: 3e-6, 1: 3e-7, 2: 1e-12, 3: 3e-7}
SHAPES = [(64, 16), (128, 16), (128, 32), (256, 32), (256, 64)]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_2604_13880_amd import binding as B
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = B.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


def _np(t):
    return t.detach().cpu().numpy()


def _labels_np(t):
    return _np(t).view(np.uint16)


MAPS = {
    "grid_n8": (lambda: square_grid_map(2, 1, lo=1.5 / 8, hi=5.5 / 8), 16),
    "vor5_n16": (lambda: voronoi_map(12, 6, 60, fractal=True), 16),
    "c1_n256": (lambda: voronoi_map(1000, 32, 2000, fractal=False), 256),
    "c1_n64": (lambda: voronoi_map(1001, 32, 2000, fractal=False), 64),
    "frac_n512": (lambda: voronoi_map(1500, 60, 12000, fractal=True), 512),
    "c2_n1024": (lambda: voronoi_map(2000, 100, 50000, fractal=True), 1024),
    "c3_n2048": (lambda: voronoi_map(3000, 200, 200000, fractal=True), 2048),
}


@pytest.mark.parametrize("name", list(MAPS))
def test_rasterize_bit_exact(ctx, name):
    make, N = MAPS[name]
    m = make()
    say("rasterize", name, "N", N, "n", m.n_vertices)
    gm = ctx.map_from(m)
    lab, cnt, cont = ctx.rasterize(gm, m.xy32(), N)
    want, wcnt, wconf = oc.rasterize(m.xy, m.ring_off, m.ring_idx, m.ring_reg, m.n_regions, N)
    got = _labels_np(lab)
    assert int(_np(cont)[0]) == wconf
    np.testing.assert_array_equal(got, want)
    np.testing.assert_array_equal(_np(cnt), wcnt)


def test_rasterize_folded_map_and_ragged_sizes(ctx):
    # folded map: contested pixels take the highest id on both sides
    xy = np.array([[0.2, 0.2], [0.5, 0.2], [0.8, 0.2], [0.8, 0.8], [0.5, 0.8], [0.2, 0.8], [0.9, 0.47]])
    ring_off = np.array([0, 5, 10], np.int32)
    ring_idx = np.array([0, 1, 6, 4, 5, 1, 2, 3, 4, 6], np.int32)
    ring_reg = np.array([1, 2], np.int32)
    gm = ctx.map_build(ring_off, ring_idx, ring_reg, 7, 2)
    for N in (16, 128):
        say("folded N", N)
        lab, cnt, cont = ctx.rasterize(gm, xy.astype(np.float32), N)
        want, wcnt, wconf = oc.rasterize(xy.astype(np.float32).astype(np.float64), ring_off, ring_idx, ring_reg, 2, N)
        assert wconf > 0 and int(_np(cont)[0]) == wconf
        np.testing.assert_array_equal(_labels_np(lab), want)
        np.testing.assert_array_equal(_np(cnt), wcnt)


@pytest.mark.parametrize("noise", [0.0, 0.004])
def test_rasterize_many_crossings_per_pixel(ctx, noise):
    """A fractal map of ~5000 vertices on a 64^2 texture: most rows have
    several crossings in one pixel (groups of coincident crossings); with
    vertex noise the map folds, so some groups hold more than one claim
    and the exact per-region claim sets decide.  Labels, counts and the
    contested-pixel count bit for bit."""
    m = voronoi_map(1700, 40, 5000, fractal=True)
    rng = np.random.default_rng(17)
    xy = np.clip(m.xy + noise * rng.standard_normal(m.xy.shape), 0.0, 1.0).astype(np.float32)
    gm = ctx.map_from(m)
    for N in (64, 128):
        lab, cnt, cont = ctx.rasterize(gm, xy, N)
        want, wcnt, wconf = oc.rasterize(xy.astype(np.float64), m.ring_off, m.ring_idx, m.ring_reg, m.n_regions, N)
        say("noise", noise, "N", N, "contested", wconf)
        if noise > 0:
            assert wconf > 0
        assert int(_np(cont)[0]) == wconf
        np.testing.assert_array_equal(_labels_np(lab), want)
        np.testing.assert_array_equal(_np(cnt), wcnt)


def test_rasterize_deformed_map(ctx):
    # a map after several oracle iterations (vertices off any grid)
    m = voronoi_map(1002, 32, 2000, fractal=False)
    s = lognormal_values(1002, 32, 1.0)
    res = oc.run(m, s, 256, fixed_iters=12, state_dtype=np.float32)
    xy32 = res.xy.astype(np.float32)
    gm = ctx.map_from(m)
    for N in (256, 1024):
        say("deformed N", N)
        lab, cnt, cont = ctx.rasterize(gm, xy32, N)
        want, wcnt, wconf = oc.rasterize(xy32.astype(np.float64), m.ring_off, m.ring_idx, m.ring_reg, m.n_regions, N)
        np.testing.assert_array_equal(_labels_np(lab), want)
        np.testing.assert_array_equal(_np(cnt), wcnt)


def _cmp_inim(im, ref, prec, N):
    S = _np(im.S)[:, : N + 1].astype(np.float64)
    T = _np(im.T)[:, : N + 1].astype(np.float64)
    HA = _np(im.HA).astype(np.float64)
    HB = _np(im.HB).astype(np.float64)
    C = ref.C
    tol = INIM_TOL[prec]
    eS = np.abs(S - ref.S).max() / C
    eT = np.abs(T - ref.T).max() / C
    eA = np.abs(HA - ref.HA).max() / C
    eB = np.abs(HB - ref.HB).max() / C
    say(f"  prec {prec} N {N}: S {eS:.2e} T {eT:.2e} HA {eA:.2e} HB {eB:.2e}")
    assert eS <= tol and eT <= tol and eA <= tol and eB <= tol


@pytest.mark.parametrize("N", [16, 32, 64, 256, 1024, 2048])
@pytest.mark.parametrize("prec", [0, 1, 2, 3])
def test_integral_image_dense(ctx, N, prec):
    d = np.random.default_rng(N + 17 * prec).lognormal(0, 1, (N, N)).astype(np.float32)
    say("inim dense", N, prec)
    im = ctx.integral_image(N, density=d, precision=prec)
    ref = oc.integral_images(d.astype(np.float64))
    _cmp_inim(im, ref, prec, N)


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("N", [16, 128, 1024])
def test_integral_image_every_tile_shape(ctx, shape, N):
    d = np.random.default_rng(N + shape[0] + shape[1]).lognormal(0, 1, (N, N)).astype(np.float32)
    ctx.set_tile_shape(N, 3, N * N, *shape)
    say("inim shape", shape, "N", N)
    im = ctx.integral_image(N, density=d, precision=3)
    _cmp_inim(im, oc.integral_images(d.astype(np.float64)), 3, N)


def test_autotune_picks_a_supported_shape(ctx, tmp_path):
    cache = str(tmp_path / "tiles.txt")
    shape = ctx.autotune(512, 3, 2, cache)
    assert tuple(shape) in SHAPES
    again = ctx.autotune(512, 3, 2, cache)      # read back from the cache file
    assert tuple(again) == tuple(shape)
    assert len(open(cache).read().strip().splitlines()) == 1


@pytest.mark.parametrize("prec", [0, 1, 2, 3])
def test_integral_image_labels(ctx, prec):
    m = voronoi_map(2000, 100, 50000, fractal=True)
    N = 1024
    lab, cnt, _ = oc.rasterize(m.xy, m.ring_off, m.ring_idx, m.ring_reg, m.n_regions, N)
    s = lognormal_values(2000, 100, 1.5)
    lut, _ = oc.density_lut(cnt, s)
    lut32 = (lut / lut.mean()).astype(np.float32)
    say("inim labels", prec)
    im = ctx.integral_image(N, labels=lab, lut=lut32, precision=prec)
    ref = oc.integral_images(lut32.astype(np.float64)[lab.astype(np.int64)])
    _cmp_inim(im, ref, prec, N)


@pytest.mark.parametrize("N", [16, 256, 1024])
def test_map_points_from_oracle_tables(ctx, N):
    import torch
    d = np.random.default_rng(N).lognormal(0, 1, (N, N))
    ref = oc.integral_images(d)
    im = ctx.inim_alloc(N, 2)
    im.S.zero_()
    im.T.zero_()
    im.S[:, : N + 1] = torch.from_numpy(ref.S).cuda()
    im.T[:, : N + 1] = torch.from_numpy(ref.T).cuda()
    im.HA.copy_(torch.from_numpy(ref.HA))
    im.HB.copy_(torch.from_numpy(ref.HB))
    rng = np.random.default_rng(N + 1)
    pts = np.concatenate([rng.random((5000, 2)), [[0, 0], [1, 1], [1, 0], [0.5, 1.0], [1.0, 0.25]],
                          np.stack(np.meshgrid(np.arange(N + 1) / N, [0.5]), -1).reshape(-1, 2)]).astype(np.float32)
    say("map from oracle tables", N)
    out = _np(ctx.map_points(im, pts, torch.empty((len(pts), 2), dtype=torch.float32, device="cuda")))
    Dx, Dy = oc.displacement(ref)
    want = oc.move_points(pts.astype(np.float64), Dx, Dy)
    err = np.abs(out - want).max()
    say("  max err", err)
    assert err <= 1.2e-7      # float32 rounding of the result (positions in [0, 1])


@pytest.mark.parametrize("prec", [0, 1, 2, 3])
def test_one_iteration_matches_oracle(ctx, prec):
    # rasterise, density, integral images and move on the GPU for one step
    import torch
    m = voronoi_map(1000, 32, 2000, fractal=False)
    s = lognormal_values(1000, 32, 1.0)
    N = 256
    gm = ctx.map_from(m)
    say("one iteration", prec)
    r = ctx.step_series([dict(map=gm, xy0=m.xy32(), N=N, values=s.astype(np.float32), fixed_iters=1,
                              precision=prec)])[0]
    got = _np(r["xy"])[0].astype(np.float64)
    want, _ = oc.iterate_once(m.xy32().astype(np.float64), m, s.astype(np.float32).astype(np.float64), N)
    err = np.abs(got - want).max()
    say("  max err", err, "iters", r["iters"], "status", r["status"])
    assert r["iters"][0] == 1
    assert err <= 1e-6


def test_region_areas(ctx):
    m = voronoi_map(2000, 100, 50000, fractal=True)
    s = lognormal_values(2000, 100, 1.5).astype(np.float32)
    gm = ctx.map_from(m)
    say("areas")
    areas, ex = ctx.region_areas(gm, m.xy32(), s)
    A = oc.region_areas(m.xy32().astype(np.float64), m.ring_off, m.ring_idx, m.ring_reg, m.n_regions)
    eps, xi = oc.cartographic_errors(A, s.astype(np.float64))
    got = _np(areas)
    assert np.abs(got[1:] - A[1:]).max() <= 1e-12 * np.abs(A[1:]).max()
    assert abs(got[0] - A[0]) <= 1e-12
    e = _np(ex)
    assert abs(e[0] - eps) <= 1e-12 and abs(e[1] - xi) <= 1e-12


# ---------------------------------------------------------------------------
# whole iterations and series


def _run1(ctx, gm, xy, N, s, prec=1, **kw):
    r = ctx.step_series([dict(map=gm, xy0=xy, N=N, values=s, fixed_iters=1, precision=prec, **kw)])[0]
    return _np(r["xy"])[0], r


def test_per_iteration_parity_256(ctx):
    """The small workload (32 regions, ~2k vertices, 256^2, 20 iterations): every
    iteration replayed from the GPU's own state -- labels bit-exact and
    moved positions within 1e-6 of the oracle's step."""
    m = voronoi_map(1000, 32, 2000, fractal=False)
    s = lognormal_values(1000, 32, 1.0).astype(np.float32)
    N = 256
    gm = ctx.map_from(m)
    xy = m.xy32()
    worst = 0.0
    for it in range(20):
        lab, cnt, _ = ctx.rasterize(gm, xy, N)
        nxt, r = _run1(ctx, gm, xy, N, s)
        want, info = oc.iterate_once(xy.astype(np.float64), m, s.astype(np.float64), N)
        np.testing.assert_array_equal(_labels_np(lab), info["labels"])
        np.testing.assert_array_equal(_np(cnt), info["counts"])
        err = np.abs(nxt.astype(np.float64) - want).max()
        worst = max(worst, err)
        assert err <= 1e-6, (it, err)
        xy = nxt
    say("per-iteration worst", worst)


@pytest.mark.parametrize("prec", [1, 2, 3])
def test_end_to_end_256(ctx, prec):
    """20 iterations on the GPU against the FP64 oracle with a float32
    state: positions within 1e-5 of the domain width."""
    m = voronoi_map(1000, 32, 2000, fractal=False)
    s = lognormal_values(1000, 32, 1.0).astype(np.float32)
    N = 256
    gm = ctx.map_from(m)
    r = ctx.step_series([dict(map=gm, xy0=m.xy32(), N=N, values=s, fixed_iters=20, precision=prec)])[0]
    got = _np(r["xy"])[0].astype(np.float64)
    ref = oc.run(m, s.astype(np.float64), N, fixed_iters=20, state_dtype=np.float32)
    err = np.abs(got - ref.xy).max()
    say("end-to-end", prec, "err", err, "xi gpu", r["xi"][0], "xi oracle", ref.xi)
    assert r["iters"][0] == 20
    assert err <= 1e-5
    assert abs(r["xi"][0] - ref.xi) <= 1e-5


def test_batched_equals_unbatched_and_cumulative(ctx):
    from synth import random_walk_series
    m = voronoi_map(1003, 24, 1500, fractal=True)
    S = random_walk_series(1003, 24, 4).astype(np.float32)
    N = 128
    gm = ctx.map_from(m)
    kw = dict(map=gm, xy0=m.xy32(), N=N, precision=1, fixed_iters=6)
    batch = ctx.step_series([dict(values=S, **kw)])[0]
    for t in range(4):
        single = ctx.step_series([dict(values=S[t], **kw)])[0]
        assert np.array_equal(_np(single["xy"])[0], _np(batch["xy"])[t])
    cum = ctx.step_series([dict(values=S, mode=1, frames=5, **kw)])[0]
    assert np.array_equal(_np(cum["xy"])[0], _np(batch["xy"])[0])
    for t in range(1, 4):
        kw2 = dict(kw)
        kw2["xy0"] = _np(cum["xy"])[t - 1]
        again = ctx.step_series([dict(values=S[t], **kw2)])[0]
        assert np.array_equal(_np(again["xy"])[0], _np(cum["xy"])[t])
    fr = _np(cum["frames"])
    xy = _np(cum["xy"])
    assert fr.shape == (3, 4) + xy.shape[1:]
    for t in range(3):
        for k in range(1, 5):
            w = np.float32(k / 5)
            np.testing.assert_allclose(fr[t, k - 1], xy[t] + w * (xy[t + 1] - xy[t]), atol=2e-7)


def test_tracer_points_follow_the_map(ctx):
    m = square_grid_map(3, 6)
    s = lognormal_values(7, 9, 0.5).astype(np.float32)
    N = 128
    g = np.stack(np.meshgrid((np.arange(33) + 0.5) / 33, (np.arange(33) + 0.5) / 33), -1).reshape(-1, 2).astype(np.float32)
    gm = ctx.map_from(m)
    r = ctx.step_series([dict(map=gm, xy0=m.xy32(), N=N, values=s, fixed_iters=5, precision=2, extra=g)])[0]
    ref = oc.run(m, s.astype(np.float64), N, fixed_iters=5, state_dtype=np.float32, extra=g)
    e1 = np.abs(_np(r["xy"])[0] - ref.xy).max()
    e2 = np.abs(_np(r["extra_xy"])[0] - ref.extra).max()
    say("tracer", e1, e2)
    assert e1 <= 1e-5 and e2 <= 1e-5


def test_stopping_rule_matches_oracle(ctx):
    m = square_grid_map(3, 6)
    s = lognormal_values(0, 9, 0.25).astype(np.float32)
    N = 256
    gm = ctx.map_from(m)
    r = ctx.step_series([dict(map=gm, xy0=m.xy32(), N=N, values=s, precision=1)])[0]
    ref = oc.run(m, s.astype(np.float64), N, state_dtype=np.float32)
    say("stop", r["iters"], r["status"], ref.iters, ref.status)
    assert r["status"][0] == ref.status == oc.STATUS_CONVERGED
    assert abs(int(r["iters"][0]) - ref.iters) <= 1
    for kw, status in ((dict(tol=1.0), 0), (dict(max_iters=3), 2), (dict(patience=0), 1)):
        r = ctx.step_series([dict(map=gm, xy0=m.xy32(), N=N, values=s, precision=1, **kw)])[0]
        o = oc.run(m, s.astype(np.float64), N, state_dtype=np.float32, **kw)
        assert r["status"][0] == status == o.status and r["iters"][0] == o.iters


def test_stopping_rule_same_for_every_graph_length(ctx):
    """For launches of single-edge emit blocks the stopping rule of an
    iteration runs in the next iteration's emit pass, and in a launch of
    its own after the last iteration of each graph.  The decision must not
    depend on where a graph ends: graphs of 32, 5 and 1 iterations and
    eager launches give the same iteration count, status, errors and
    positions, bit for bit, whether the run ends by the tolerance, the cap,
    a stall, fixed_iters or already at the start."""
    m = voronoi_map(1003, 24, 3000, fractal=True)
    s = lognormal_values(1003, 24, 0.8).astype(np.float32)
    N = 256
    gm = ctx.map_from(m)
    cases = [dict(), dict(max_iters=13), dict(patience=2), dict(fixed_iters=7), dict(fixed_iters=33),
             dict(tol=1.0)]
    for kw in cases:
        runs = []
        for gi in (32, 5, 1, -3):
            r = ctx.step_series([dict(map=gm, xy0=m.xy32(), N=N, values=s, precision=1, **kw)], graph_iters=gi)[0]
            runs.append((int(r["iters"][0]), int(r["status"][0]), float(r["xi"][0]), float(r["eps"][0]),
                         _np(r["xy"])[0].copy()))
        say("rule", kw, [(a, b, c) for a, b, c, _, _ in runs])
        for other in runs[1:]:
            assert other[:4] == runs[0][:4], (kw, other[:4], runs[0][:4])
            assert np.array_equal(other[4], runs[0][4]), kw
    o = oc.run(m, s.astype(np.float64), N, state_dtype=np.float32, max_iters=13)
    r = ctx.step_series([dict(map=gm, xy0=m.xy32(), N=N, values=s, precision=1, max_iters=13)], graph_iters=5)[0]
    assert int(r["iters"][0]) == o.iters and int(r["status"][0]) == o.status


def test_polygon_area_source_iteration(ctx):
    m = voronoi_map(1004, 20, 1200, fractal=True)
    s = lognormal_values(1004, 20, 1.0).astype(np.float32)
    N = 128
    gm = ctx.map_from(m)
    nxt, r = _run1(ctx, gm, m.xy32(), N, s, prec=2, area_source=1)
    want, _ = oc.iterate_once(m.xy32().astype(np.float64), m, s.astype(np.float64), N, area_source="polygon")
    assert np.abs(nxt - want).max() <= 1e-6


def test_shape_parameter(ctx):
    m = voronoi_map(1005, 20, 1200, fractal=True)
    s = lognormal_values(1005, 20, 1.0).astype(np.float32)
    N = 128
    gm = ctx.map_from(m)
    for b in (0.95, 1.05):
        nxt, r = _run1(ctx, gm, m.xy32(), N, s, prec=2, shape=b)
        want, _ = oc.iterate_once(m.xy32().astype(np.float64), m, s.astype(np.float64), N, b=b)
        assert np.abs(nxt - want).max() <= 1e-6


@pytest.mark.parametrize("shape", [(128, 32), (256, 32), (128, 16)])
@pytest.mark.parametrize("prec", [0, 1, 2, 3])
def test_integral_image_labels_2048(ctx, prec, shape):
    # (128, 16) at 2048^2: the tile-row prefix table (128 x 17) exceeds the
    # carry pass's LDS table, so the separate row-carry pass runs
    """Labels + LUT at 2048^2 (the size of the batched series) for every accumulation mode."""
    m = voronoi_map(3000, 200, 200000, fractal=True)
    N = 2048
    lab, cnt, _ = oc.rasterize(m.xy, m.ring_off, m.ring_idx, m.ring_reg, m.n_regions, N)
    s = lognormal_values(3000, 200, 1.0)
    lut, _ = oc.density_lut(cnt, s)
    lut32 = (lut / lut.mean()).astype(np.float32)
    ctx.set_tile_shape(N, prec, N * N, *shape)
    say("inim labels 2048", prec, shape)
    im = ctx.integral_image(N, labels=lab, lut=lut32, precision=prec)
    ref = oc.integral_images(lut32.astype(np.float64)[lab.astype(np.int64)])
    S = _np(im.S)[:, : N + 1].astype(np.float64)
    err = np.abs(S - ref.S)
    j, i = np.unravel_index(np.argmax(err), err.shape)
    say("  worst S at row", j, "col", i, "err/C", err[j, i] / ref.C)
    _cmp_inim(im, ref, prec, N)


def test_uneven_batch_equals_single_runs_and_oracle(ctx):
    """Independent cartograms of different sizes in one call (one launch
    per kernel per iteration for all of them, each with its own stopping
    rule) give exactly the results of one call per cartogram under the
    same tile shape, and one batched iteration matches the oracle."""
    import torch
    specs = [(4100, 16, 64, 0.5, 40), (4101, 40, 256, 1.0, 25), (4102, 24, 128, 2.0, 60), (4103, 70, 512, 1.5, 33),
             (4104, 16, 16, 0.8, 12), (4105, 33, 256, 1.2, 47)]
    maps, descs = [], []
    for seed, R, N, sig, cap in specs:
        m = voronoi_map(seed, R, 40 * R, fractal=True)
        s = lognormal_values(seed, R, sig).astype(np.float32)
        maps.append((m, s, N))
        descs.append(dict(map=ctx.map_from(m), xy0=m.xy32(), N=N, values=s, precision=1, max_iters=cap, patience=16))
    px = sum(N * N for _, _, N in maps)
    for N in {N for _, _, N in maps}:
        ctx.set_tile_shape(N, 1, N * N, 64, 16)
    ctx.set_tile_shape(512, 1, px, 64, 16)
    say("uneven batch of", len(maps))
    batch = ctx.step_series(descs)
    iters = [int(r["iters"][0]) for r in batch]
    assert len(set(iters)) > 1          # the instances stop at different iterations
    for k, d in enumerate(descs):
        single = ctx.step_series([d])[0]
        assert torch.equal(single["xy"], batch[k]["xy"]), k
        assert single["iters"][0] == batch[k]["iters"][0] and single["status"][0] == batch[k]["status"][0]
        assert single["xi"][0] == batch[k]["xi"][0]
    one = ctx.step_series([dict(d, fixed_iters=1) for d in descs])
    for k, (m, s, N) in enumerate(maps):
        want, _ = oc.iterate_once(m.xy32().astype(np.float64), m, s.astype(np.float64), N)
        err = np.abs(_np(one[k]["xy"])[0].astype(np.float64) - want).max()
        assert err <= 1e-6, (k, err)


def _comb_map(teeth: int):
    """One region whose upper side is a square wave of `teeth` teeth between
    y = 0.4 and 0.6: every row in that band is crossed 2 * teeth times."""
    from synth import PlanarMap
    pts = [(0.1, 0.1), (0.9, 0.1), (0.9, 0.4)]
    dx = 0.8 / teeth
    for i in range(teeth):
        x0 = 0.9 - i * dx
        pts += [(x0, 0.6), (x0 - dx / 2, 0.6), (x0 - dx / 2, 0.4)]
        if i + 1 < teeth:
            pts.append((x0 - dx, 0.4))
    pts.append((0.1, 0.4))
    xy = np.asarray(pts, dtype=np.float32).astype(np.float64)
    ring = np.arange(len(pts), dtype=np.int32)
    a = 0.5 * np.sum(xy[ring, 0] * np.roll(xy[ring, 1], -1) - np.roll(xy[ring, 0], -1) * xy[ring, 1])
    if a < 0:
        ring = ring[::-1].copy()
    return PlanarMap(xy=xy, ring_off=np.array([0, len(pts)], dtype=np.int32), ring_idx=ring,
                     ring_reg=np.array([1], dtype=np.int32), n_regions=1)


def test_row_bucket_overflow_is_reported(ctx):
    """A row crossed more often than its bucket holds (256 crossings) makes
    the series report CG_FLAG_OVERFLOW and end with CG_STATUS_ERROR; a map
    just under the limit runs normally."""
    from paper_2604_13880_amd import binding as B
    for teeth, over in ((150, True), (100, False)):
        m = _comb_map(teeth)
        gm = ctx.map_from(m)
        r = ctx.step_series([dict(map=gm, xy0=m.xy32(), N=256, values=np.array([1.0], np.float32),
                                  fixed_iters=2)])[0]
        flagged = bool(r["flags"][0] & B.FLAG_OVERFLOW)
        assert flagged == over, (teeth, r["flags"][0])
        assert (r["status"][0] == B.STATUS_ERROR) == over


def _folded_comb_map(teeth: int):
    """The comb of `_comb_map` plus a second region, the rectangle
    [0.3, 0.7] x [0.45, 0.55], laid over the teeth without sharing an edge:
    the pixel centres inside both are claimed by two regions (a folded
    map; they take the highest id), in rows crossed 2 * teeth + 2 times."""
    from synth import PlanarMap
    c = _comb_map(teeth)
    n = c.xy.shape[0]
    rect = np.array([[0.3, 0.45], [0.7, 0.45], [0.7, 0.55], [0.3, 0.55]], dtype=np.float32).astype(np.float64)
    ring2 = np.arange(n, n + 4, dtype=np.int32)
    return PlanarMap(xy=np.concatenate([c.xy, rect]), ring_off=np.array([0, n, n + 4], dtype=np.int32),
                     ring_idx=np.concatenate([c.ring_idx, ring2]), ring_reg=np.array([1, 2], dtype=np.int32),
                     n_regions=2)


@pytest.mark.parametrize("case", ["comb40", "comb100", "folded_comb40", "folded_comb100"])
def test_rows_beyond_64_crossings_bit_exact(ctx, case):
    """Rows crossed more than 64 times take the fill kernel's serial walk of
    the claim set: labels, counts and the contested count match the oracle
    bit for bit (80 and 200 crossings per row; the folded combs add rows
    where two regions claim the same runs)."""
    teeth = int(case.rsplit("comb", 1)[1])
    m = _folded_comb_map(teeth) if case.startswith("folded") else _comb_map(teeth)
    gm = ctx.map_from(m)
    for N in (256, 512):
        say("long rows", case, "N", N)
        lab, cnt, cont = ctx.rasterize(gm, m.xy32(), N)
        want, wcnt, wconf = oc.rasterize(m.xy32().astype(np.float64), m.ring_off, m.ring_idx, m.ring_reg,
                                         m.n_regions, N)
        rows = [q for q in range(N) if 0.4 * N < q + 0.5 < 0.6 * N]
        assert len(rows) > 0
        np.testing.assert_array_equal(_labels_np(lab), want)
        np.testing.assert_array_equal(_np(cnt), wcnt)
        assert int(_np(cont)[0]) == wconf
        assert (wconf > 0) == case.startswith("folded")


def test_whole_run_1024_replays_match_oracle(ctx):
    """Map 2000 of the 1024^2 workload (100 fractal regions, ~50k
    vertices, compensated FP32) iterated on the GPU to 64, 256 and 511
    iterations, the regime the benchmark runs (strongly deformed maps,
    more crossings per row); from the GPU's own state at each point one
    more iteration is replayed through the oracle: labels, counts and the
    contested count bit-exact, moved positions within 1e-6."""
    m = voronoi_map(2000, 100, 50000, fractal=True)
    s = lognormal_values(2000, 100, 1.5).astype(np.float32)
    N = 1024
    gm = ctx.map_from(m)
    xy = m.xy32()
    done = 0
    for k in (64, 256, 511):
        r = ctx.step_series([dict(map=gm, xy0=xy, N=N, values=s, precision=1, fixed_iters=k - done)])[0]
        assert int(r["iters"][0]) == k - done and int(r["flags"][0]) & 2 == 0
        xy = _np(r["xy"])[0]
        done = k
        lab, cnt, cont = ctx.rasterize(gm, xy, N)
        nxt, _ = _run1(ctx, gm, xy, N, s, prec=1)
        want, info = oc.iterate_once(xy.astype(np.float64), m, s.astype(np.float64), N)
        same = int((_labels_np(lab) == info["labels"]).sum())
        err = np.abs(nxt.astype(np.float64) - want).max()
        say(f"  after {k} iterations: labels equal {same}/{N * N}, contested {int(_np(cont)[0])}, max |dxy| {err:.2e}")
        np.testing.assert_array_equal(_labels_np(lab), info["labels"])
        np.testing.assert_array_equal(_np(cnt), info["counts"])
        assert int(_np(cont)[0]) == info["conflicts"]
        assert err <= 1e-6, (k, err)


def test_large_batch_with_separate_density_pass(ctx):
    """A batch whose LUT work (tiles x LUT entries) exceeds what the reduce
    pass builds itself runs Step 3 as its own launch: one iteration still
    matches the oracle, and a single (fused) run of the same map to rounding."""
    import torch
    m = voronoi_map(4200, 300, 30000, fractal=False)
    N, n = 1024, 8
    vals = [lognormal_values(4200 + k, 300, 1.0).astype(np.float32) for k in range(n)]
    gm = ctx.map_from(m)
    descs = [dict(map=gm, xy0=m.xy32(), N=N, values=v, fixed_iters=1) for v in vals]
    ctx.set_tile_shape(N, 1, n * N * N, 128, 16)      # 8 x 512 tiles x 301 entries > 2^20
    ctx.set_tile_shape(N, 1, N * N, 128, 16)
    say("large batch, separate density pass")
    batch = ctx.step_series(descs)
    single = ctx.step_series([descs[0]])[0]
    assert np.abs(_np(single["xy"]) - _np(batch[0]["xy"])).max() <= 1e-6
    for k in (0, 5):
        want, _ = oc.iterate_once(m.xy32().astype(np.float64), m, vals[k].astype(np.float64), N)
        err = np.abs(_np(batch[k]["xy"])[0].astype(np.float64) - want).max()
        assert err <= 1e-6, (k, err)



def test_large_batch_emits_several_edges_per_thread(ctx):
    """A batch of more than 8192 blocks of 256 edges (2M edges) runs the
    rasteriser's emit pass with several edges per thread: one iteration of
    its first and last instances matches the oracle and a single run of the
    same map (one edge per thread) to rounding."""
    m = voronoi_map(2000, 100, 50000, fractal=True)
    N, n = 1024, 48
    vals = [lognormal_values(4400 + k, 100, 1.5).astype(np.float32) for k in range(n)]
    gm = ctx.map_from(m)
    assert n * ((gm.n_edges + 255) // 256) > 8192 and (gm.n_edges + 255) // 256 <= 8192
    descs = [dict(map=gm, xy0=m.xy32(), N=N, values=v, fixed_iters=1) for v in vals]
    ctx.set_tile_shape(N, 1, n * N * N, 128, 16)
    ctx.set_tile_shape(N, 1, N * N, 128, 16)
    say("large batch, several edges per emit thread")
    batch = ctx.step_series(descs)
    for k in (0, n - 1):
        single = ctx.step_series([descs[k]])[0]
        assert np.abs(_np(single["xy"]) - _np(batch[k]["xy"])).max() <= 1e-6
        want, _ = oc.iterate_once(m.xy32().astype(np.float64), m, vals[k].astype(np.float64), N)
        err = np.abs(_np(batch[k]["xy"])[0].astype(np.float64) - want).max()
        assert err <= 1e-6, (k, err)


def test_series_at_full_size_matches_oracle(ctx):
    """The 64-step 2048^2 series as the benchmark runs it (one instance per
    step in one batch, FP64-accumulated integral images, 256x64 tiles, four
    edges per emit thread): one iteration of sampled steps matches the
    oracle."""
    from paper_2604_13880_amd import binding as B
    from synth import random_walk_series
    m = voronoi_map(3000, 200, 200000, fractal=True)
    S = random_walk_series(3000, 200, 64).astype(np.float32)
    N, T = 2048, 64
    gm = ctx.map_from(m)
    assert T * ((gm.n_edges + 255) // 256) > 8192
    ctx.set_tile_shape(N, B.F64ACC, T * N * N, 256, 64)
    say("series 64 x 2048^2, one iteration")
    r = ctx.step_series([dict(map=gm, xy0=m.xy32(), N=N, values=S, precision=B.F64ACC, fixed_iters=1)])[0]
    xy = _np(r["xy"])
    assert xy.shape[0] == T
    for t in (0, 31, 63):
        want, _ = oc.iterate_once(m.xy32().astype(np.float64), m, S[t].astype(np.float64), N)
        err = np.abs(xy[t].astype(np.float64) - want).max()
        say("  step", t, "max |dxy|", err)
        assert err <= 1e-6, (t, err)


def _uneven_instance(spec):
    m = voronoi_map(spec["seed"], spec["R"], spec["n_target"], fractal=True)
    return m, lognormal_values(spec["seed"], spec["R"], spec["sigma"]).astype(np.float32)


def test_uneven_batch_at_full_size_matches_oracle(ctx):
    """The 256-cartogram uneven batch as the benchmark runs it (textures
    256^2 to 2048^2 in one launch per kernel, compensated FP32, 256x64
    tiles, block tables for the unequal instances, four edges per emit
    thread, the density table as its own launch): one iteration of sampled
    instances of every texture size matches the oracle."""
    import multiprocessing as mp
    from synth import uneven_batch_specs
    specs = uneven_batch_specs(4000, 256)
    with mp.get_context("fork").Pool(16) as pool:
        maps = pool.map(_uneven_instance, specs, chunksize=4)
    Ns = [sp["N"] for sp in specs]
    px = sum(N * N for N in Ns)
    ctx.set_tile_shape(max(Ns), 1, px, 256, 64)
    descs = [dict(map=ctx.map_from(m), xy0=m.xy32(), N=N, values=v, precision=1, fixed_iters=1)
             for (m, v), N in zip(maps, Ns)]
    assert sum(d["map"].n_edges for d in descs) > 8192 * 256
    say("uneven batch of", len(descs), "at full size, one iteration")
    res = ctx.step_series(descs)
    picks = [next(k for k, N in enumerate(Ns) if N == n) for n in sorted(set(Ns))]
    for k in picks:
        m, v = maps[k]
        want, _ = oc.iterate_once(m.xy32().astype(np.float64), m, v.astype(np.float64), Ns[k])
        err = np.abs(_np(res[k]["xy"])[0].astype(np.float64) - want).max()
        say("  instance", k, "N", Ns[k], "max |dxy|", err)
        assert err <= 1e-6, (k, Ns[k], err)


def test_double_tables_with_several_writer_blocks_per_cu(ctx):
    """Double-precision (S, T) pairs written by 512 writer blocks (several per
    CU): repeated runs are bit-identical and agree with the float-stored
    double-accumulated mode to float rounding."""
    from paper_2604_13880_amd import binding as B
    m = voronoi_map(2000, 100, 50000, fractal=True)
    s = lognormal_values(2000, 100, 1.5).astype(np.float32)
    gm = ctx.map_from(m)
    N = 1024
    for prec in (B.F64, B.F64ACC):
        ctx.set_tile_shape(N, prec, N * N, 128, 16)
    d = lambda prec: dict(map=gm, xy0=m.xy32(), N=N, values=s, precision=prec, fixed_iters=2)
    say("double tables, 128x16 tiles at 1024^2")
    runs = [_np(ctx.step_series([d(B.F64)], graph_iters=-1)[0]["xy"]) for _ in range(3)]
    ref = _np(ctx.step_series([d(B.F64ACC)], graph_iters=-1)[0]["xy"])
    assert all(np.array_equal(runs[0], r) for r in runs[1:])
    assert np.abs(runs[0] - ref).max() <= 1e-6


def test_cached_iteration_graph_reads_the_new_call(ctx):
    """A second call with the same launches replays the first call's graph:
    it must compute from its own inputs (bit-equal to a fresh context and to
    eager launches)."""
    from paper_2604_13880_amd import binding as B
    m = voronoi_map(4300, 24, 3000, fractal=True)
    s1 = lognormal_values(4300, 24, 1.0).astype(np.float32)
    s2 = lognormal_values(4301, 24, 1.5).astype(np.float32)
    gm = ctx.map_from(m)
    d = lambda s: dict(map=gm, xy0=m.xy32(), N=256, values=s, fixed_iters=12)
    r1 = ctx.step_series([d(s1)], graph_iters=4)[0]
    r2 = ctx.step_series([d(s2)], graph_iters=4)[0]        # same launches: the cached graph
    fresh = B.Context(0)
    try:
        f2 = fresh.step_series([dict(d(s2), map=fresh.map_from(m))], graph_iters=4)[0]
    finally:
        fresh.close()
    e2 = ctx.step_series([d(s2)], graph_iters=-4)[0]
    assert not np.array_equal(_np(r1["xy"]), _np(r2["xy"]))
    assert np.array_equal(_np(r2["xy"]), _np(f2["xy"]))
    assert np.array_equal(_np(r2["xy"]), _np(e2["xy"]))
