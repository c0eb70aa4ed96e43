"""Precision form: every accumulation mode of the GPU path against the
FP64 oracle on the 2048^2 series map (200 fractal regions, its first time
step), per result (the benchmark spec's precision form; the integral images of
Background, eq.(1); areas and errors of "Quality Measures"):

  * S and T of the map's density, max abs difference / total mass C;
  * region areas (FP64 shoelace of the float32 positions);
  * positions and max area error after 3 whole iterations from the same
    start (the oracle keeping a float32 state, as the GPU does).

Bounds: S and T as the integral-image parity tests (F32 3e-6, COMP and
F64ACC 3e-7, F64 1e-12); areas 1e-12; positions 1e-5 and max area error
1e-4 after 3 iterations.  The measured table is printed (pytest -s)."""
import numpy as np
import pytest
import torch

from oracle import cartogram as oc
from synth import random_walk_series, voronoi_map

pytestmark = pytest.mark.gpu

BOUND = {"F32": 3e-6, "COMP": 3e-7, "F64ACC": 3e-7, "F64": 1e-12}


def test_accumulation_modes_against_the_oracle():
    from paper_2604_13880_amd import binding as B
    ctx = B.Context(0)
    m = voronoi_map(3000, 200, 200000, fractal=True)
    s = random_walk_series(3000, 200, 1)[0].astype(np.float32)
    N = 2048
    gm = ctx.map_from(m)
    xy0 = torch.from_numpy(m.xy32()).cuda()
    lab, cnt, _ = ctx.rasterize(gm, xy0, N)
    labels = lab.cpu().numpy().view(np.uint16)
    lut, _ = oc.density_lut(cnt.cpu().numpy(), s.astype(np.float64))
    lut32 = (lut / lut.mean()).astype(np.float32)
    im_o = oc.integral_images(oc.density_texture(labels, lut32.astype(np.float64)))
    C = im_o.C
    A_o = oc.region_areas(m.xy32().astype(np.float64), m.ring_off, m.ring_idx, m.ring_reg, 200)
    A_g = ctx.region_areas(gm, xy0)[0].cpu().numpy()
    e_area = float(np.abs(A_g[1:] - A_o[1:]).max())
    print(f"\nregion areas: max |A - A_oracle| = {e_area:.2e}", flush=True)
    assert e_area <= 1e-12
    run_o = oc.run(m, s.astype(np.float64), N, fixed_iters=3, state_dtype=np.float32)
    vals = torch.from_numpy(s).cuda()
    print(f"{'mode':7s} {'|dS|/C':>9s} {'|dT|/C':>9s} {'|dxy| 3 it':>11s} {'|dxi| 3 it':>11s}", flush=True)
    for name, prec in (("F32", B.F32), ("COMP", B.COMP), ("F64ACC", B.F64ACC), ("F64", B.F64)):
        im = ctx.integral_image(N, labels=lab, lut=torch.from_numpy(lut32).cuda(), precision=prec)
        eS = float(np.abs(im.S[:, : N + 1].double().cpu().numpy() - im_o.S).max() / C)
        eT = float(np.abs(im.T[:, : N + 1].double().cpu().numpy() - im_o.T).max() / C)
        r = ctx.step_series([dict(map=gm, xy0=xy0, N=N, values=vals, precision=prec, fixed_iters=3)])[0]
        exy = float(np.abs(r["xy"][0].cpu().numpy().astype(np.float64) - run_o.xy).max())
        exi = abs(float(r["xi"][0]) - run_o.xi)
        print(f"{name:7s} {eS:9.2e} {eT:9.2e} {exy:11.2e} {exi:11.2e}", flush=True)
        assert eS <= BOUND[name] and eT <= BOUND[name]
        assert exy <= 1e-5 and exi <= 1e-4
    ctx.close()
