"""Benchmark of the integral-image cartogram hot path on one MI355X.

A step is one whole cartogram: every iteration of rasterise -> density ->
integral images -> move vertices -> areas -> stopping rule, run by
libcg's HIP kernels through cg_step_series (captured HIP graphs), from
the original map until the stopping rule ends it.  Inputs are resident in
HBM before the timed region starts.

Default workload: 100 seeded Voronoi regions with midpoint-displaced
fractal boundaries (~50k vertices), values lognormal(sigma = 1.5), a
1024^2 texture, iterate until the max area error is below 1% (or the
paper's stopping rule ends the run), compensated-FP32 integral images.

Printed: one JSON line (rank 0).  `roofline` times the integral-image
writer kernel (sat_final, the largest HBM writer and the longest kernel
of an iteration) with HIP events recorded on its own stream around one
launch in every `--profile-every` iterations of the timed region;
`traffic` is the HBM byte count per launch of the same kernel from the
rocprofv3 counter summary under profiles/ (scaled by a copy kernel of
known size), reported only while the kernel source still matches the
hash recorded with the counters.  `cpu_baseline` times the FP64 oracle
on a bounded sample of the same workload on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ms to 1% area error per cartogram; Mpx-iter/s; learned+batched vs plain"
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "fractal100_1024": dict(seed=2000, seeds=10, R=100, n=50000, fractal=True, sigma=1.5, N=1024, precision=1,
                    desc="100 fractal Voronoi regions (~50k vertices), 10 seeded maps (timed step k runs map "
                         "k mod 10), lognormal sigma 1.5, 1024^2 texture, iterate to max area error < 1% or the "
                         "stopping rule, compensated FP32 integral images"),
    "voronoi32_256": dict(seed=1000, R=32, n=2000, fractal=False, sigma=1.0, N=256, precision=1, fixed=20,
                    desc="32 Voronoi regions (~2k vertices), lognormal sigma 1, 256^2 texture, 20 iterations"),
    "series64_fractal200_2048": dict(seed=3000, R=200, n=200000, fractal=True, sigma=1.0, N=2048, precision=3, T=64,
                    desc="200 fractal Voronoi regions (~200k vertices), 2048^2, 64 time steps of a geometric "
                         "random walk (step sigma 0.1), all steps batched (direct), FP64-accumulated integral images"),
    "uneven256_256to2048": dict(seed=4000, count=256, precision=1,
                    desc="256 independent fractal Voronoi cartograms, textures 256^2-2048^2, 16-300 regions, "
                         "lognormal sigma 0.5-2, ~500 R N/1024 vertices each, one launch per kernel per iteration "
                         "for all instances, compensated FP32 integral images, each to its own stopping rule"),
}


def _uneven_map(spec):
    from synth import lognormal_values, voronoi_map
    m = voronoi_map(spec["seed"], spec["R"], spec["n_target"], fractal=True)
    return m, lognormal_values(spec["seed"], spec["R"], spec["sigma"]).astype(np.float32)


def run_uneven(a, B, ctx, torch):
    """An uneven batch of independent cartograms in one series call."""
    import multiprocessing as mp
    from synth import uneven_batch_specs
    w = WORKLOADS["uneven256_256to2048"]
    specs = uneven_batch_specs(w["seed"], w["count"])
    log("uneven256_256to2048: generating", len(specs), "maps")
    with mp.get_context("fork").Pool(16) as pool:
        maps = pool.map(_uneven_map, specs, chunksize=4)
    gms = [ctx.map_from(m) for m, s in maps]
    descs = [dict(map=g, xy0=torch.from_numpy(m.xy32()).cuda(), N=sp["N"], values=torch.from_numpy(s).cuda(),
                  precision=w["precision"]) for g, (m, s), sp in zip(gms, maps, specs)]
    px = sum(sp["N"] ** 2 for sp in specs)
    shape = ctx.autotune(2048, w["precision"], max(1, px // (2048 * 2048)), cache_path=a.tune_cache)
    ctx.step_series(descs, graph_iters=a.graph_iters)      # warm-up
    torch.cuda.synchronize()
    ctx.profile_stage(a.stage, a.profile_every)
    t0 = time.perf_counter()
    res = ctx.step_series(descs, graph_iters=a.graph_iters)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    stage_ms, stage_n = ctx.profile_read()
    ctx.profile_stage(None)
    iters = np.array([int(r["iters"][0]) for r in res], dtype=np.int64)
    status = np.array([int(r["status"][0]) for r in res])
    Ns = np.array([sp["N"] for sp in specs], dtype=np.int64)
    # the same cartograms one per call (first 32), for the batching gain
    k = 32
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for d in descs[:k]:
        ctx.step_series([d], graph_iters=a.graph_iters)
    torch.cuda.synchronize()
    ms_single = (time.perf_counter() - t1) * 1e3
    px_iter = float((Ns * Ns * iters).sum())
    # achieved bytes of the timed kernel: an iteration's launch covers every
    # instance still running; use the mean active pixel count per launch
    roof = None
    if a.stage in ("sat_final", "sat_reduce", "raster_fill") and stage_n:
        # a launch covers the instances still running: mean algorithmic bytes per launch
        per = sum(alg_bytes(a.stage, int(N), w["precision"], 0) * int(it) for N, it in zip(Ns, iters))
        per /= max(int(iters.max()), 1)
        ach = per / (stage_ms / stage_n * 1e-3) / 1e9
        roof = dict(bound="hbm", kernel=a.stage, achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=ach / HBM_PEAK_GBS, traffic=counter_traffic(a.stage, "uneven256_256to2048"),
                    avg_launch_us=stage_ms / stage_n * 1e3, launches=stage_n, alg_bytes_per_launch=per,
                    note="bytes per launch = mean over the run's iterations of the instances still running")
    return dict(workload=w["desc"], instances=len(specs), texture_mpx=px / 1e6, ms_batch=ms,
                ms_per_cartogram=ms / len(specs), mpx_iter_per_s=px_iter / (ms / 1e3) / 1e6,
                iterations_mean=float(iters.mean()), iterations_max=int(iters.max()),
                converged=int((status == 0).sum()), stalled=int((status == 1).sum()), tile=list(shape),
                single_calls_ms_per_cartogram=ms_single / k, single_calls_maps=k, roofline=roof)

STORE_BYTES = {0: 4, 1: 4, 2: 8, 3: 4}  # stored table entry per precision (F32, COMP, F64, F64ACC)
PREC_NAMES = ["F32", "COMP", "F64", "F64ACC"]
KERNEL_SOURCES = {
    "sat_final": ["paper_2604_13880_amd/csrc/sat.hip", "paper_2604_13880_amd/csrc/cg_dev.h"],
    "sat_reduce": ["paper_2604_13880_amd/csrc/sat.hip", "paper_2604_13880_amd/csrc/cg_dev.h"],
    "raster_fill": ["paper_2604_13880_amd/csrc/raster.hip", "paper_2604_13880_amd/csrc/cg_dev.h"],
    "map_points": ["paper_2604_13880_amd/csrc/mapping.hip", "paper_2604_13880_amd/csrc/cg_dev.h"],
}


def alg_bytes(stage, N, prec, n_pts):
    """Bytes one launch of `stage` must move for one N x N instance:
    what the method reads and writes, not what the kernel happens to."""
    b = STORE_BYTES[prec]
    if stage == "sat_final":    # labels read + S and T written, (N+1)^2 entries each
        return 2 * N * N + 2 * (N + 1) ** 2 * b
    if stage == "sat_reduce":   # labels read
        return 2 * N * N
    if stage == "raster_fill":  # labels written
        return 2 * N * N
    if stage == "map_points":   # positions in and out + 4 corner nodes x (S, T) gathered per point
        return n_pts * (16 + 8 * b)
    raise ValueError(f"no algorithmic byte count for stage {stage}")


def sources_hash(stage):
    h = hashlib.sha256()
    for f in KERNEL_SOURCES.get(stage, []):
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counter_traffic(stage, workload):
    """HBM bytes per launch from profiles/<kernel>_<workload>_counters.txt,
    or None when absent or taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", f"{stage}_{workload}_counters.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256_16") != sources_hash(stage):
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def roofline(stage, ms, n, N, prec, n_pts, instances, workload):
    per = alg_bytes(stage, N, prec, n_pts) * instances
    avg_ms = ms / max(n, 1)
    ach = per / (avg_ms * 1e-3) / 1e9 if n else None
    return dict(bound="hbm", kernel=stage, achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s",
                frac=(ach / HBM_PEAK_GBS) if ach else None, traffic=counter_traffic(stage, workload),
                avg_launch_us=avg_ms * 1e3, launches=n, alg_bytes_per_launch=per)


def run_learned(a, B, ctx, torch):
    """Warm start by the trained net followed by the plain
    iteration, against the plain method, on held-out seeded maps."""
    from paper_2604_13880_amd import learned as Lr
    path = os.path.join(ROOT, "paper_2604_13880_amd", "weights", Lr.WEIGHTS_NAME)
    if not os.path.exists(path):
        return {"skipped": f"no trained weights at {os.path.relpath(path, ROOT)}"}
    net = B.Net(ctx, max_batch=Lr.PREDICT_BATCH, **Lr.NET_CFG)
    net.load(path)
    log("learned_512: generating", a.learned_maps, "held-out maps")
    maps = Lr.make_maps(range(Lr.TEST_SEED0, Lr.TEST_SEED0 + a.learned_maps), workers=16)
    rep = Lr.compare(ctx, net, maps, single=min(16, a.learned_maps), area_source=1)
    rep["workload"] = ("held-out seeded maps, 50-150 fractal Voronoi regions (~250 vertices per region), "
                       "lognormal sigma 1, 512^2 texture, polygon-area density, to max area error < 1% or the "
                       f"stopping rule; warm side = log-density on a {Lr.N_NET}^2 grid + one plain iteration ({Lr.N_NET}^2 tracer "
                       f"grid) + U-Net forward at {Lr.N_NET}^2 + graded warm start (field box-averaged to {Lr.N_NET // Lr.WARM_POOL}^2) + plain "
                       "iterations; 32 cartograms per call on both sides; equal quality: each map stopped at the "
                       "plain run's final max area error")
    rep["speedup_learned_batched_vs_plain_single"] = rep["plain_single_ms_per_cartogram"] / rep["warm_ms_per_cartogram"]
    rep["speedup_learned_batched_vs_plain_batched"] = rep["plain_ms_per_cartogram"] / rep["warm_ms_per_cartogram"]
    eq = rep["equal_quality"]
    rep["speedup_learned_batched_vs_plain_batched_equal_quality"] = eq["plain_ms_per_cartogram"] / eq["warm_ms_per_cartogram"]
    net.close()
    return rep


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(m, values, N, gpu_iters, sample_iters):
    """The FP64 oracle as it stands, timed on the host on the first
    `sample_iters` iterations of the same workload; the per-iteration
    time is scaled to the GPU run's iteration count."""
    from oracle import cartogram as oc
    xy = m.xy.copy()
    t0 = time.perf_counter()
    for _ in range(sample_iters):
        xy, _ = oc.iterate_once(xy, m, values, N)
        A = oc.region_areas(xy, m.ring_off, m.ring_idx, m.ring_reg, m.n_regions)
        oc.cartographic_errors(A, values)
    dt = time.perf_counter() - t0
    ms_iter = dt * 1e3 / sample_iters
    return dict(value=ms_iter * gpu_iters, unit="ms per cartogram", cores=1, kind="oracle",
                ms_per_iteration=ms_iter, sample_seconds=dt,
                sample=f"first {sample_iters} iterations of the first map (FP64 numpy, one thread), "
                       f"per-iteration time x {gpu_iters:g} iterations (mean of the GPU runs)")


def precision_table(ctx, B, m, values, N):
    """Max |S - S64| / C and |T - T64| / C of the float-stored modes against
    double accumulation and storage, on the map's density texture, and the
    position and max-area-error differences after 20 whole iterations."""
    import torch
    gm = ctx.map_from(m)
    lab, cnt, _ = ctx.rasterize(gm, torch.from_numpy(m.xy32()).cuda(), N)
    c = cnt.double().cpu().numpy()
    lut = np.zeros(m.n_regions + 1, np.float32)
    lut[1:] = np.where(c[1:] > 0, values / np.maximum(c[1:], 1), 0)
    lut[0] = values.sum() / max(c[1:].sum(), 1)
    lut /= lut.mean()
    lutt = torch.from_numpy(lut).cuda()
    ref = ctx.integral_image(N, labels=lab, lut=lutt, precision=B.F64)
    C = float(ref.S[N, N])
    out = {}
    for name, prec in (("F32", B.F32), ("COMP", B.COMP), ("F64ACC", B.F64ACC)):
        im = ctx.integral_image(N, labels=lab, lut=lutt, precision=prec)
        eS = float((im.S[:, : N + 1].double() - ref.S[:, : N + 1]).abs().max()) / C
        eT = float((im.T[:, : N + 1].double() - ref.T[:, : N + 1]).abs().max()) / C
        out[name] = {"S_rel": eS, "T_rel": eT}
    # whole iterations: positions and max area error after 20 iterations
    # against the double-precision mode
    xy0 = torch.from_numpy(m.xy32()).cuda()
    vals = torch.from_numpy(np.asarray(values, np.float32)).cuda()
    runs = {}
    for name, prec in (("F64", B.F64), ("F32", B.F32), ("COMP", B.COMP), ("F64ACC", B.F64ACC)):
        runs[name] = ctx.step_series([dict(map=gm, xy0=xy0, N=N, values=vals, precision=prec, fixed_iters=20)])[0]
    for name in ("F32", "COMP", "F64ACC"):
        out[name]["xy_20_iters_max_abs"] = float((runs[name]["xy"] - runs["F64"]["xy"]).abs().max())
        out[name]["xi_20_iters_abs"] = abs(float(runs[name]["xi"][0]) - float(runs["F64"]["xi"][0]))
    return out


def run_series(a, w, B, ctx, torch):
    """Every step of a 64-step value series as one direct batch."""
    from synth import random_walk_series, voronoi_map
    log("series64_fractal200_2048: generating map")
    m = voronoi_map(w["seed"], w["R"], w["n"], fractal=True)
    S = random_walk_series(w["seed"], w["R"], w["T"], sigma0=w["sigma"]).astype(np.float32)
    N = w["N"]
    gm = ctx.map_from(m)
    shape = ctx.autotune(N, w["precision"], w["T"], cache_path=a.tune_cache)
    desc = dict(map=gm, xy0=torch.from_numpy(m.xy32()).cuda(), N=N, values=torch.from_numpy(S).cuda(),
                precision=w["precision"], frames=10)
    ctx.step_series([desc], graph_iters=a.graph_iters)
    torch.cuda.synchronize()
    ctx.profile_stage(a.stage, a.profile_every)
    t0 = time.perf_counter()
    for _ in range(a.series_steps):
        r = ctx.step_series([desc], graph_iters=a.graph_iters)[0]
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / a.series_steps
    stage_ms, stage_n = ctx.profile_read()
    ctx.profile_stage(None)
    iters = r["iters"].astype(np.int64)
    return dict(workload=w["desc"], ms_per_series=ms, ms_per_cartogram=ms / w["T"],
                mpx_iter_per_s=float(N * N * iters.sum() / (ms / 1e3) / 1e6),
                iterations_mean=float(iters.mean()), iterations_max=int(iters.max()),
                converged=int((r["status"] == 0).sum()), steps=int(w["T"]), tile=list(shape),
                frames_per_transition=10, precision_vs_f64=precision_table(ctx, B, m, S[0], N),
                roofline=roofline(a.stage, stage_ms, stage_n, N, w["precision"], m.n_vertices, w["T"], "series64_fractal200_2048"))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="fractal100_1024", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=96)
    ap.add_argument("--tune-cache", default=None,
                    help="tile-shape table file: read if present, written otherwise (profiling runs share one)")
    ap.add_argument("--graph-iters", type=int, default=-32,
                    help="iterations between convergence polls; negative = eager launches "
                         "(HIP events around the timed stage are only recorded outside graphs)")
    ap.add_argument("--stage", default="sat_final", choices=sorted(KERNEL_SOURCES),
                    help="kernel timed with HIP events for the roofline")
    ap.add_argument("--profile-every", type=int, default=8, help="time one launch of the stage per this many iterations")
    ap.add_argument("--no-series", action="store_true", help="skip the batched 64-step series of 2048^2 cartograms")
    ap.add_argument("--series-steps", type=int, default=1, help="timed repetitions of the batched series")
    ap.add_argument("--no-uneven", action="store_true", help="skip the uneven batch of 256 cartograms")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned warm start at 512^2")
    ap.add_argument("--learned-maps", type=int, default=64, help="held-out maps of the learned comparison")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device-to-device 5 times (calibrates the HBM traffic counters)")
    a = ap.parse_args()
    if a.copy_probe:
        import torch
        x = torch.ones(a.copy_probe * 1024 * 1024 // 4, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_per_copy": x.numel() * 4, "copies": 5}))
        return
    if a.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {a.gpus} is not supported: the library runs "
              f"on one GPU (instances would shard across GPUs data-parallel)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2604_13880_amd import binding as B
    from synth import lognormal_values, voronoi_map

    w = WORKLOADS[a.workload]
    nseed = w.get("seeds", 1)
    log("workload", a.workload, "generating", nseed, "maps")
    maps = [(voronoi_map(w["seed"] + k, w["R"], w["n"], fractal=w["fractal"]),
             lognormal_values(w["seed"] + k, w["R"], w["sigma"]).astype(np.float32)) for k in range(nseed)]
    m, values = maps[0]
    N = w["N"]
    ctx = B.Context(0)
    descs = [dict(map=ctx.map_from(mk), xy0=torch.from_numpy(mk.xy32()).cuda(), N=N,
                  values=torch.from_numpy(vk).cuda(), precision=w["precision"], fixed_iters=w.get("fixed", 0))
             for mk, vk in maps]
    tile = ctx.autotune(N, w["precision"], 1, cache_path=a.tune_cache)
    torch.cuda.synchronize()

    warmup = max(a.warmup, nseed)          # every map once before the timed steps
    log("warmup", warmup)
    for k in range(warmup):
        ctx.step_series([descs[k % nseed]], graph_iters=a.graph_iters)
    torch.cuda.synchronize()

    ctx.profile_stage(a.stage, a.profile_every)
    log("timed", a.steps)
    runs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(a.steps):
        runs.append(ctx.step_series([descs[k % nseed]], graph_iters=a.graph_iters)[0])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stage_ms, stage_n = ctx.profile_read()
    ctx.profile_stage(None)
    ms_step = (t1 - t0) * 1e3 / a.steps
    its = np.array([int(r["iters"][0]) for r in runs])
    xis = np.array([float(r["xi"][0]) for r in runs])
    sts = np.array([int(r["status"][0]) for r in runs])
    iters = float(its.mean())
    mpx = N * N * float(its.sum()) / ((t1 - t0)) / 1e6

    roof = roofline(a.stage, stage_ms, stage_n, N, w["precision"], m.n_vertices, 1, a.workload)

    series = None
    if not a.no_series and a.workload == "fractal100_1024":
        series = run_series(a, WORKLOADS["series64_fractal200_2048"], B, ctx, torch)

    uneven = None
    if not a.no_uneven and a.workload == "fractal100_1024":
        uneven = run_uneven(a, B, ctx, torch)

    learned = None
    if not a.no_learned and a.workload == "fractal100_1024":
        learned = run_learned(a, B, ctx, torch)

    cpu = None
    if not a.no_cpu:
        log("cpu baseline", a.cpu_iters, "iterations")
        cpu = cpu_baseline(m, values.astype(np.float64), N, iters, a.cpu_iters)   # first map, mean GPU iterations

    out = {
        "metric": METRIC, "value": ms_step, "unit": "ms per cartogram", "n_gpus": 1,
        "steps": a.steps, "warmup": warmup, "ms_per_step": ms_step, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic (seeded Voronoi maps)",
        "config": {"workload": w["desc"], "texture": N, "regions": w["R"], "vertices": m.n_vertices,
                   "precision": PREC_NAMES[w["precision"]]},
        "mpx_iter_per_s": mpx, "maps": nseed, "iterations": iters, "final_xi_mean": float(xis.mean()),
        "final_xi": [round(float(x), 5) for x in xis[:nseed]],
        "status": [["converged", "stalled", "maxiter", "error"][int(v)] for v in sts[:nseed]],
        "reached_tol": int((sts == 0).sum()), "ms_per_iteration": ms_step / max(iters, 1),
        "tile": list(tile), "roofline": roof, "cpu_baseline": cpu, "batched_series": series,
        "uneven_batch": uneven, "learned_warm_start": learned,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
