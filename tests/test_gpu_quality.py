"""GPU geographic-distortion measures (cg_quality) against the oracle's
(Background, "Quality Measures"): adjacency counts, best overlaps over
pixel translations and pixel counts bit for bit, shape distortions from
the same integers, barycentres and the relative position error to FP64
rounding.  Cases: deformed maps at 256^2 and 1024^2, label images of
random noise (the overlap bounds prune little, so the search runs nearly
exhaustively; brute force on the oracle side), regions too large for the
search kernel's LDS copy, empty regions, and the map against itself."""
import numpy as np
import pytest
import torch

from oracle import cartogram as oc
from oracle import quality as oq
from synth import lognormal_values, square_grid_map, voronoi_map

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2604_13880_amd import binding as B
    c = B.Context(0)
    yield c
    c.close()


def _compare(ctx, m, N, xy_map, xy_cart, lab_map, lab_cart, brute=False):
    gm = ctx.map_from(m)
    tl = lambda a: torch.from_numpy(np.ascontiguousarray(a).astype(np.uint16).view(np.int16)).cuda()
    q = ctx.quality(gm, N, xy_map, xy_cart, tl(lab_map), tl(lab_cart))
    R = m.n_regions
    tau, nm, nc, common = oq.topology_distortion(lab_map, lab_cart)
    assert q["adjacency"].cpu().tolist() == [nm, nc, common]
    assert q["tau"] == tau
    H, hmean, hmax, best = oq.shape_distortion(lab_map, lab_cart, R, brute=brute)
    assert np.array_equal(q["overlap"].cpu().numpy(), best)
    pix = q["pixels"].cpu().numpy()
    for v in range(1, R + 1):
        assert pix[0, v] == int((lab_map == v).sum()) and pix[1, v] == int((lab_cart == v).sum())
    assert np.array_equal(q["shape"].cpu().numpy(), H)
    assert abs(q["shape_mean"] - hmean) <= 1e-14 and q["shape_max"] == hmax
    bm = oq.barycenters(np.asarray(xy_map, np.float64), m.ring_off, m.ring_idx, m.ring_reg, R)
    bc = oq.barycenters(np.asarray(xy_cart, np.float64), m.ring_off, m.ring_idx, m.ring_reg, R)
    gb = q["bary"].cpu().numpy()
    assert np.abs(gb[0, 1:] - bm[1:]).max() <= 1e-12 and np.abs(gb[1, 1:] - bc[1:]).max() <= 1e-12
    assert abs(q["rel_pos"] - oq.relative_position_error(bm, bc)) <= 1e-12
    return q


@pytest.mark.parametrize("N,seed,R,n,iters", [(256, 1000, 32, 2000, 12), (1024, 2000, 100, 50000, 64)])
def test_deformed_map_matches_oracle(ctx, N, seed, R, n, iters):
    m = voronoi_map(seed, R, n, fractal=seed != 1000)
    s = lognormal_values(seed, R, 1.5 if N == 1024 else 1.0).astype(np.float32)
    gm = ctx.map_from(m)
    r = ctx.step_series([dict(map=gm, xy0=m.xy32(), N=N, values=s, fixed_iters=iters, precision=1)])[0]
    xc = r["xy"][0].cpu().numpy()
    lm = ctx.rasterize(gm, m.xy32(), N)[0].cpu().numpy().view(np.uint16)
    lc = ctx.rasterize(gm, xc, N)[0].cpu().numpy().view(np.uint16)
    q = _compare(ctx, m, N, m.xy32(), xc, lm, lc)
    assert 0 < q["shape_mean"] < 1 and q["rel_pos"] > 0


def test_map_against_itself(ctx):
    m = voronoi_map(1000, 32, 2000, fractal=False)
    gm = ctx.map_from(m)
    lm = ctx.rasterize(gm, m.xy32(), 128)[0]
    q = ctx.quality(gm, 128, m.xy32(), m.xy32(), lm, lm)
    assert q["tau"] == 0.0 and q["shape_mean"] == 0.0 and q["shape_max"] == 0.0 and q["rel_pos"] == 0.0
    a = q["adjacency"].cpu().tolist()
    assert a[0] == a[1] == a[2] > 32


@pytest.mark.parametrize("N,density", [(32, 0.5), (64, 0.3), (64, 0.7)])
def test_noise_images_match_brute_force(ctx, N, density):
    # four regions whose pixels are scattered at random over overlapping
    # boxes: upper bounds are weak, the search visits most translations
    m = square_grid_map(2, 2)
    rng = np.random.default_rng(N + int(100 * density))
    def img():
        lab = np.zeros((N, N), np.uint16)
        for v in range(1, 5):
            y0, x0 = rng.integers(0, N // 2, 2)
            h, w = rng.integers(3, N // 2, 2)
            blk = (rng.random((h, w)) < density) & (lab[y0:y0 + h, x0:x0 + w] == 0)
            lab[y0:y0 + h, x0:x0 + w][blk] = v
        return lab
    a, b = img(), img()
    _compare(ctx, m, N, m.xy32(), m.xy32(), a, b, brute=True)


def test_regions_beyond_the_lds_copy_and_empty_regions(ctx):
    # 2 x 2 squares over most of a 1024^2 texture: each bit image takes
    # ~460 rows x 8 words, both together more than the search kernel's LDS copy;
    # region 4 is missing from the cartogram raster, region 3 shrunk
    m = square_grid_map(2, 4, lo=0.05, hi=0.95)
    gm = ctx.map_from(m)
    N = 1024
    lm = ctx.rasterize(gm, m.xy32(), N)[0].cpu().numpy().view(np.uint16).copy()
    lc = np.roll(np.roll(lm, 37, 0), -11, 1).copy()
    lc[lc == 4] = 0
    ys, xs = np.nonzero(lc == 3)
    lc[ys[::3], xs[::3]] = 0
    q = _compare(ctx, m, N, m.xy32(), m.xy32(), lm, lc)
    assert q["shape"][4].item() == 1.0 and q["overlap"][4].item() == 0
    assert q["overlap"][1].item() == int((lm == 1).sum())   # a pure translation overlaps completely


def test_labels_above_the_region_count_are_rejected(ctx):
    from paper_2604_13880_amd import binding as B
    m = square_grid_map(2, 2)
    gm = ctx.map_from(m)
    lab = torch.zeros((64, 64), dtype=torch.int16, device="cuda")
    bad = lab.clone()
    bad[10, 10] = 5
    with pytest.raises(B.CartogramError):
        ctx.quality(gm, 64, m.xy32(), m.xy32(), lab, bad)
    with pytest.raises(B.CartogramError):
        ctx.quality(gm, 60, m.xy32(), m.xy32(), lab, lab)
