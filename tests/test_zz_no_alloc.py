"""The allocation-free integral images (cg_integral_image_noalloc) through
the C ABI against the allocating entry point cg_integral_image: the same
kernels on the same inputs give the same tables bit for bit, on two calls
in a row (the second with a smaller texture, so it runs on what the first
left in the shared static scratch), and both match the FP64 oracle within
the accumulation-mode tolerances of the other integral-image tests.  The
calls leave the device's free memory unchanged, and a texture whose
scratch does not fit the static buffer is rejected before any launch."""
import numpy as np
import pytest

from oracle import cartogram as oc
from synth import lognormal_values, voronoi_map

pytestmark = pytest.mark.gpu

# |S - S_oracle| / C bounds per accumulation mode (F32, COMP, F64, F64ACC)
INIM_TOL = {0: 3e-6, 1: 3e-7, 2: 1e-12, 3: 3e-7}


def _label_case(seed, R, n, N, sigma):
    m = voronoi_map(seed, R, n, fractal=True)
    lab, cnt, _ = oc.rasterize(m.xy, m.ring_off, m.ring_idx, m.ring_reg, m.n_regions, N)
    lut, _ = oc.density_lut(cnt, lognormal_values(seed, R, sigma))
    return lab, (lut / lut.mean()).astype(np.float32)


def _np(t):
    return t.detach().cpu().numpy()


def _same(a, b, N):
    return (np.array_equal(_np(a.S)[:, : N + 1], _np(b.S)[:, : N + 1])
            and np.array_equal(_np(a.T)[:, : N + 1], _np(b.T)[:, : N + 1])
            and np.array_equal(_np(a.HA), _np(b.HA)) and np.array_equal(_np(a.HB), _np(b.HB)))


def _vs_oracle(im, ref, prec, N):
    C = ref.C
    errs = [np.abs(_np(im.S)[:, : N + 1].astype(np.float64) - ref.S).max() / C,
            np.abs(_np(im.T)[:, : N + 1].astype(np.float64) - ref.T).max() / C,
            np.abs(_np(im.HA).astype(np.float64) - ref.HA).max() / C,
            np.abs(_np(im.HB).astype(np.float64) - ref.HB).max() / C]
    print("  vs oracle", prec, N, ["%.2e" % e for e in errs], flush=True)
    return max(errs) <= INIM_TOL[prec]


def test_noalloc_equals_the_allocating_call():
    import torch
    from paper_2604_13880_amd import binding as B
    ctx = B.Context(0)
    try:
        cases = [(1024, B.COMP) + _label_case(2000, 100, 50000, 1024, 1.5),
                 (256, B.F64ACC) + _label_case(1000, 32, 2000, 256, 1.0)]
        dev = []
        for N, prec, lab, lut in cases:
            lab_d = torch.from_numpy(lab.view(np.int16)).cuda()
            lut_d = torch.from_numpy(lut).cuda()
            ref = ctx.integral_image(N, labels=lab_d, lut=lut_d, precision=prec)
            out = ctx.inim_alloc(N, prec)
            for t in (out.S, out.T, out.HA, out.HB):
                t.fill_(float("nan"))
            dev.append((lab_d, lut_d, ref, out))
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        for (N, prec, _, _), (lab_d, lut_d, _, out) in zip(cases, dev):   # two calls in a row, 1024^2 then 256^2
            print("noalloc call N", N, "precision", prec, flush=True)
            ctx.integral_image(N, labels=lab_d, lut=lut_d, precision=prec, out=out, noalloc=True)
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
        assert free1 == free0, (free0, free1)
        for (N, prec, lab, lut), (_, _, ref, out) in zip(cases, dev):
            assert _same(out, ref, N), N
            assert _vs_oracle(out, oc.integral_images(lut.astype(np.float64)[lab.astype(np.int64)]), prec, N)
        # a dense texture, double tables, after the label calls
        N = 512
        d = np.random.default_rng(5).lognormal(0, 1, (N, N)).astype(np.float32)
        ref = ctx.integral_image(N, density=d, precision=B.F64)
        out = ctx.integral_image(N, density=d, precision=B.F64, noalloc=True)
        assert _same(out, ref, N)
        assert _vs_oracle(out, oc.integral_images(d.astype(np.float64)), B.F64, N)
    finally:
        ctx.close()


def test_noalloc_rejects_scratch_beyond_the_static_buffer():
    import torch
    from paper_2604_13880_amd import binding as B
    ctx = B.Context(0)
    try:
        N = 8192                       # 128 x 32 tiles need about 150 MB of carries
        lab = torch.zeros((N, N), dtype=torch.int16, device="cuda")
        lut = torch.ones(1, dtype=torch.float32, device="cuda")
        out = ctx.inim_alloc(N, B.F32)
        with pytest.raises(B.CartogramError, match="static buffer"):
            ctx.integral_image(N, labels=lab, lut=lut, precision=B.F32, out=out, noalloc=True)
        torch.cuda.synchronize()
    finally:
        ctx.close()
