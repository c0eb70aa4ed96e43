"""Warm start through the C ABI: log-density input, tracer fields, the
move by a pixel-centre field (against the oracle's definition), and the
fallback to the plain start when a field does not help or folds the map."""
import numpy as np
import pytest

from oracle import cartogram as oc
from synth import lognormal_values, square_grid_map, voronoi_map

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2604_13880_amd import binding as B
    c = B.Context(0)
    yield c
    c.close()


def test_log_density_matches_oracle(ctx):
    import torch
    m = voronoi_map(1000, 32, 2000, fractal=False)
    s = lognormal_values(1000, 32, 1.0).astype(np.float32)
    gm = ctx.map_from(m)
    for N, b in ((256, 1.0), (128, 0.9)):
        lab, cnt, _ = ctx.rasterize(gm, m.xy32(), N)
        got = ctx.log_density(lab, cnt, torch.from_numpy(s).cuda(), shape=b).cpu().numpy()
        labels = lab.cpu().numpy().view(np.uint16)
        want = oc.log_density(labels, cnt.cpu().numpy(), s.astype(np.float64), b=b)
        assert np.max(np.abs(got - want)) < 1e-5


def test_log_density_of_several_maps_in_one_call(ctx):
    """The batched call gives, for every map, the texture of the single-map
    calls (same kernels: bit-equal), and the oracle's within 1e-5."""
    import torch
    N = 128
    maps = [(voronoi_map(1100 + k, 12 + 9 * k, 800 + 400 * k, fractal=k % 2 == 1),
             lognormal_values(1100 + k, 12 + 9 * k, 1.0).astype(np.float32)) for k in range(3)]
    gms = [ctx.map_from(m) for m, s in maps]
    got = ctx.log_density_maps(gms, [torch.from_numpy(m.xy32()).cuda() for m, s in maps], N,
                               [torch.from_numpy(s).cuda() for m, s in maps], shape=0.8).cpu().numpy()
    for k, ((m, s), gm) in enumerate(zip(maps, gms)):
        lab, cnt, _ = ctx.rasterize(gm, m.xy32(), N)
        one = ctx.log_density(lab, cnt, torch.from_numpy(s).cuda(), shape=0.8).cpu().numpy()
        assert np.array_equal(got[k], one)
        want = oc.log_density(lab.cpu().numpy().view(np.uint16), cnt.cpu().numpy(), s.astype(np.float64), b=0.8)
        assert np.max(np.abs(got[k] - want)) < 1e-5


def test_tracer_grid_and_field(ctx):
    import torch
    G = 64
    grid = ctx.tracer_grid(G).cpu().numpy()
    assert np.array_equal(grid.astype(np.float64), oc.tracer_grid(G))
    moved = torch.from_numpy(grid + 0.01).cuda()
    f = ctx.tracer_field(G, moved).cpu().numpy()
    assert f.shape == (G, G, 2) and np.allclose(f, 0.01, atol=1e-7)


def _plain_and_field(ctx, m, s, N, G):
    import torch
    gm = ctx.map_from(m)
    grid = ctx.tracer_grid(G)
    r = ctx.step_series([dict(map=gm, xy0=m.xy32(), N=N, values=s, extra=grid)])[0]
    field = ctx.tracer_field(G, r["extra_xy"][0])
    torch.cuda.synchronize()
    return gm, r, field


def test_warm_start_from_a_converged_field(ctx):
    m = square_grid_map(3, 6)
    s = lognormal_values(0, 9, 0.25).astype(np.float32)
    N, G = 256, 64
    gm, plain, field = _plain_and_field(ctx, m, s, N, G)
    assert plain["status"][0] == 0
    # the move itself: stop right after the warm start (max_iters = 0); the
    # step chosen among the trial steps is the oracle's
    r0 = ctx.step_series([dict(map=gm, xy0=m.xy32(), N=N, values=s, init_field=field, max_iters=0)])[0]
    assert not (r0["flags"][0] & 4)
    alpha, want = oc.warm_start_choose(m, s.astype(np.float64), N, m.xy32().astype(np.float64),
                                       field.cpu().numpy().astype(np.float64))
    assert alpha > 0
    assert np.max(np.abs(r0["xy"][0].cpu().numpy() - want)) < 1e-6
    plain0 = ctx.step_series([dict(map=gm, xy0=m.xy32(), N=N, values=s, max_iters=0)])[0]
    assert r0["xi"][0] < 0.5 * plain0["xi"][0]
    # the whole run: converged, in fewer iterations
    rw = ctx.step_series([dict(map=gm, xy0=m.xy32(), N=N, values=s, init_field=field)])[0]
    assert rw["status"][0] == 0 and not (rw["flags"][0] & 4)
    assert rw["iters"][0] < plain["iters"][0], (rw["iters"][0], plain["iters"][0])


def test_partial_step_when_the_full_field_folds(ctx):
    # a field twice too long folds the map; a shorter trial step is taken
    m = square_grid_map(3, 6)
    s = lognormal_values(0, 9, 0.25).astype(np.float32)
    N, G = 256, 64
    gm, plain, field = _plain_and_field(ctx, m, s, N, G)
    f2 = 2.5 * field
    r0 = ctx.step_series([dict(map=gm, xy0=m.xy32(), N=N, values=s, init_field=f2, max_iters=0)])[0]
    alpha, want = oc.warm_start_choose(m, s.astype(np.float64), N, m.xy32().astype(np.float64),
                                       f2.cpu().numpy().astype(np.float64))
    if alpha == 0:
        assert r0["flags"][0] & 4
    else:
        assert not (r0["flags"][0] & 4)
    assert np.max(np.abs(r0["xy"][0].cpu().numpy() - want)) < 1e-6


@pytest.mark.parametrize("kind", ["zero", "folding"])
def test_rejected_warm_start_falls_back_to_the_plain_run(ctx, kind):
    import torch
    m = voronoi_map(1000, 32, 2000, fractal=False)
    s = lognormal_values(1000, 32, 1.0).astype(np.float32)
    gm = ctx.map_from(m)
    G = 32
    if kind == "zero":
        field = torch.zeros((G, G, 2), device="cuda")
    else:  # neighbouring cells pushed in opposite directions: the map folds
        sign = np.where((np.arange(G)[:, None] + np.arange(G)[None, :]) % 2 == 0, 1.0, -1.0)
        field = torch.from_numpy(np.stack([0.2 * sign, -0.2 * sign], -1).astype(np.float32)).cuda()
    desc = dict(map=gm, xy0=m.xy32(), N=256, values=s, fixed_iters=5)
    plain = ctx.step_series([desc])[0]
    warm = ctx.step_series([dict(desc, init_field=field)])[0]
    assert warm["flags"][0] & 4
    assert torch.equal(warm["xy"], plain["xy"])
    assert warm["xi"][0] == plain["xi"][0]
