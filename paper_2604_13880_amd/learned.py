"""Learned warm start: training data from the plain method, training of
the U-Net by the library's kernels, and warm-started runs.

Every numerical step runs in libcg (binding.py); this module only orders
the calls.  Data: seeded Voronoi maps with fractal boundaries (synth),
the plain iteration run to its stopping rule with a pixel-centre tracer
grid moved along.  Input = the log-density texture of the original map
and the tracer displacement after FEATURE_ITERS plain iterations (the
first iterations carry the global part of the deformation, which the
net's receptive field cannot see); target = the displacement of the
tracers at the end of the run (the converged deformation).  The net's
head adds RESIDUAL_GAIN times the early displacement, so it learns the
correction to a scaled early iterate.

    python -m paper_2604_13880_amd.learned train --out W.bin [--maps 10000]
    python -m paper_2604_13880_amd.learned eval --weights W.bin [--maps 512]
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

TRAIN_SEED0 = 5_000_000     # training maps: seeds TRAIN_SEED0 + k
TEST_SEED0 = 6_000_000      # held-out maps
N_TEX = 512              # texture of the cartograms
N_NET = 128              # grid of the net's input and output (pixel centres of a 128^2 grid)
FEATURE_ITERS = 1
WARM_POOL = 2            # the predicted field is box-averaged over 2 x 2 cells (a 64^2 field) before use
PREDICT_BATCH = 32
WEIGHTS_NAME = "warm_start_128.bin"
RESIDUAL_GAIN = 2.4      # median ratio of the final to the first-iteration displacement on training maps
NET_CFG = dict(base_channels=32, levels=4, height=N_NET, width=N_NET, out_scale=0.1, in_channels=3,
               residual_gain=RESIDUAL_GAIN)


def _make_map(args):
    from synth import lognormal_values, voronoi_map
    seed, rmin, rmax, per_region, sigma = args
    rng = np.random.default_rng(seed)
    R = int(rng.integers(rmin, rmax + 1))
    m = voronoi_map(seed, R, per_region * R, fractal=True)
    s = lognormal_values(seed, R, sigma).astype(np.float32)
    return m, s


def make_maps(seeds, rmin=50, rmax=150, per_region=250, sigma=1.0, workers=16):
    """Seeded maps and values (host), generated in parallel processes."""
    args = [(int(s), rmin, rmax, per_region, sigma) for s in seeds]
    if workers <= 1 or len(args) < 4:
        return [_make_map(a) for a in args]
    with mp.get_context("fork").Pool(workers) as pool:
        return pool.map(_make_map, args, chunksize=max(1, len(args) // (4 * workers)))


def device_inputs(maps):
    """Positions and values of every map on the device: two uploads, one
    view per map (reused by every call on the same maps)."""
    import torch
    xy = torch.from_numpy(np.concatenate([m.xy32() for m, s in maps])).cuda()
    vals = torch.from_numpy(np.concatenate([s for m, s in maps]).astype(np.float32)).cuda()
    xys, vs, o, r = [], [], 0, 0
    for m, s in maps:
        xys.append(xy[o:o + m.n_vertices])
        vs.append(vals[r:r + len(s)])
        o += m.n_vertices
        r += len(s)
    return xys, vs


def net_inputs(ctx, maps, N=N_NET, shape=1.0, gmaps=None, batch=64, dev=None):
    """log-density textures [n][N][N] (device float32) of the original maps,
    `batch` maps per library call (positions and values uploaded at once)."""
    import torch
    out = torch.empty((len(maps), N, N), dtype=torch.float32, device="cuda")
    xys, vs = device_inputs(maps) if dev is None else dev
    for b0 in range(0, len(maps), batch):
        part = maps[b0:b0 + batch]
        gm = [ctx.map_from(m) for m, s in part] if gmaps is None else gmaps[b0:b0 + batch]
        out[b0:b0 + len(part)] = ctx.log_density_maps(gm, xys[b0:b0 + batch], N, vs[b0:b0 + batch], shape=shape)
    return out


def plain_runs(ctx, maps, N=N_TEX, G=N_TEX, batch=32, graph_iters=8, gmaps=None, dev=None, **kw):
    """Plain runs to the stopping rule with a G x G tracer grid; returns the
    tracer displacement fields [n][G][G][2] (device) and per-map stats."""
    import torch
    grid = ctx.tracer_grid(G)
    fields = torch.empty((len(maps), G, G, 2), dtype=torch.float32, device="cuda")
    stats = dict(iters=np.zeros(len(maps), np.int32), status=np.zeros(len(maps), np.int32),
                 xi=np.zeros(len(maps)))
    for b0 in range(0, len(maps), batch):
        part = maps[b0:b0 + batch]
        gm = [ctx.map_from(m) for m, s in part] if gmaps is None else gmaps[b0:b0 + batch]
        if dev is None:
            descs = [dict(map=g, xy0=m.xy32(), N=N, values=s, extra=grid, **kw) for g, (m, s) in zip(gm, part)]
        else:
            descs = [dict(map=g, xy0=dev[0][b0 + k], N=N, values=dev[1][b0 + k], extra=grid, **kw)
                     for k, g in enumerate(gm)]
        res = ctx.step_series(descs, graph_iters=graph_iters)
        for k, r in enumerate(res):
            fields[b0 + k] = ctx.tracer_field(G, r["extra_xy"][0])
            stats["iters"][b0 + k] = r["iters"][0]
            stats["status"][b0 + k] = r["status"][0]
            stats["xi"][b0 + k] = r["xi"][0]
    return fields, stats


def features(ctx, maps, N=N_TEX, G=N_NET, gmaps=None, dev=None, **kw):
    """Net input [n][G][G][3]: log-density on the G x G grid and the
    displacement of a G x G tracer grid after FEATURE_ITERS plain
    iterations at texture N (same stopping parameters otherwise)."""
    import torch
    kw = dict(kw)
    kw.pop("max_iters", None)
    dev = device_inputs(maps) if dev is None else dev
    X0 = net_inputs(ctx, maps, G, gmaps=gmaps, dev=dev)
    # a few iterations: eager launches (a captured graph would cost more than it saves)
    D, _ = plain_runs(ctx, maps, N, G, gmaps=gmaps, dev=dev, graph_iters=-FEATURE_ITERS, fixed_iters=FEATURE_ITERS,
                      **kw)
    return torch.cat([X0[..., None], D], dim=-1).contiguous()


def train(net, X, Y, epochs=4, batch=16, lr=1e-3, lr_end=1e-4, seed=0, log=print, max_seconds=None):
    """Adam on mean squared error over shuffled mini-batches; the learning
    rate decays geometrically from lr to lr_end over the run.  Returns the
    mean training loss of every epoch."""
    import torch
    n = X.shape[0]
    rng = np.random.default_rng(seed)
    steps = epochs * ((n + batch - 1) // batch)
    gamma = (lr_end / lr) ** (1.0 / max(steps - 1, 1))
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    hist, step, t0 = [], 0, time.perf_counter()
    for ep in range(epochs):
        order = torch.from_numpy(rng.permutation(n)).cuda()
        loss.zero_()
        nb = 0
        for b0 in range(0, n, batch):
            idx = order[b0:b0 + batch]
            xb = X.index_select(0, idx).contiguous()
            yb = Y.index_select(0, idx).contiguous()
            net.zero_grads()
            net.forward(xb)
            net.backward(yb, loss)          # adds this batch's mean loss
            net.adam_step(lr * gamma ** step)
            step += 1
            nb += 1
            if max_seconds and time.perf_counter() - t0 > max_seconds:
                break
        hist.append(float(loss.item()) / max(nb, 1))
        log(f"epoch {ep} mean loss {hist[-1]:.4e} steps {step} elapsed {time.perf_counter() - t0:.1f}s")
        if max_seconds and time.perf_counter() - t0 > max_seconds:
            break
    return hist


def predict(net, X, batch=PREDICT_BATCH, pool=1):
    """Predicted fields [n][G/pool][G/pool][2]."""
    import torch
    G = X.shape[1] // pool
    out = torch.empty((X.shape[0], G, G, 2), dtype=torch.float32, device="cuda")
    batch = min(batch, net.max_batch)
    for b0 in range(0, X.shape[0], batch):
        F = net.forward(X[b0:b0 + batch].contiguous())
        for k in range(F.shape[0]):
            out[b0 + k] = F[k] if pool == 1 else net.ctx.field_pool(F[k], pool)
    return out


def run_batched(ctx, gmaps, maps, fields=None, N=N_TEX, batch=32, graph_iters=8, dev=None, **kw):
    """Runs of many maps, `batch` cartograms per cg_step_series call."""
    out = dict(iters=[], status=[], xi=[], flags=[])
    for b0 in range(0, len(maps), batch):
        descs = []
        for k in range(b0, min(b0 + batch, len(maps))):
            m, s = maps[k]
            if dev is None:
                d = dict(map=gmaps[k], xy0=m.xy32(), N=N, values=s, **kw)
            else:
                d = dict(map=gmaps[k], xy0=dev[0][k], N=N, values=dev[1][k], **kw)
            if fields is not None:
                d["init_field"] = fields[k]
            descs.append(d)
        for r in ctx.step_series(descs, graph_iters=graph_iters):
            for key in out:
                out[key].append(r[key][0])
    return {k: np.asarray(v) for k, v in out.items()}


def compare(ctx, net, maps, N=N_TEX, batch=32, graph_iters=8, single=0, **kw):
    """Plain vs warm-started runs of the same maps: iterations, final
    errors, fallbacks and wall time per cartogram.  The warm side includes
    the net's input (log-density and the first plain iteration) and its
    forward pass.  Both sides run `batch` cartograms per call; `single` > 0
    also times the plain method one cartogram per call on that many maps.
    A second warm run stops at equal quality: each map's tolerance is the
    max area error the plain run ended with (at least the usual 1%)."""
    import torch
    gmaps = [ctx.map_from(m) for m, s in maps]
    n = len(maps)
    dev = device_inputs(maps)   # positions and values on the device, for both sides
    dv = lambda a, b: (dev[0][a:b], dev[1][a:b])
    # untimed first calls of both paths (buffer allocation, code loading)
    k0 = min(n, 4)
    run_batched(ctx, gmaps[:k0], maps[:k0], None, N, batch, graph_iters, dev=dv(0, k0), **kw)
    Fw = predict(net, features(ctx, maps[:k0], N, gmaps=gmaps[:k0], dev=dv(0, k0), **kw), pool=WARM_POOL)
    run_batched(ctx, gmaps[:k0], maps[:k0], Fw, N, batch, graph_iters, dev=dv(0, k0), **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain = run_batched(ctx, gmaps, maps, None, N, batch, graph_iters, dev=dev, **kw)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    X = features(ctx, maps, N, gmaps=gmaps, dev=dev, **kw)
    F = predict(net, X, pool=WARM_POOL)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    warm = run_batched(ctx, gmaps, maps, F, N, batch, graph_iters, dev=dev, **kw)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    # equal quality: per-map tolerance = the plain run's final max error
    tol = np.maximum(plain["xi"] * (1 + 1e-6), kw.get("tol", 0.01))
    kq = {k: v for k, v in kw.items() if k != "tol"}
    eq_w = dict(iters=[], xi=[], status=[])
    eq_p = dict(iters=[], xi=[], status=[])
    eq_ms = {}
    for side, fields, acc in (("warm", F, eq_w), ("plain", None, eq_p)):
        torch.cuda.synchronize()
        te = time.perf_counter()
        for b0 in range(0, n, batch):
            descs = []
            for k in range(b0, min(b0 + batch, n)):
                d = dict(map=gmaps[k], xy0=dev[0][k], N=N, values=dev[1][k], tol=float(tol[k]), **kq)
                if fields is not None:
                    d["init_field"] = fields[k]
                descs.append(d)
            for r in ctx.step_series(descs, graph_iters=graph_iters):
                acc["iters"].append(int(r["iters"][0]))
                acc["xi"].append(float(r["xi"][0]))
                acc["status"].append(int(r["status"][0]))
        torch.cuda.synchronize()
        eq_ms[side] = (time.perf_counter() - te) * 1e3 / n
    eqw = {k: np.asarray(v) for k, v in eq_w.items()}
    eqp = {k: np.asarray(v) for k, v in eq_p.items()}
    reached_w = eqw["status"] == 0
    reached_p = eqp["status"] == 0
    rep = dict(maps=n, batch=batch, plain_ms_per_cartogram=(t1 - t0) * 1e3 / n,
               warm_ms_per_cartogram=(t3 - t1) * 1e3 / n, warm_net_ms_per_cartogram=(t2 - t1) * 1e3 / n,
               plain_iters_mean=float(plain["iters"].mean()), warm_iters_mean=float(warm["iters"].mean()),
               plain_converged=int((plain["status"] == 0).sum()), warm_converged=int((warm["status"] == 0).sum()),
               plain_xi_mean=float(plain["xi"].mean()), warm_xi_mean=float(warm["xi"].mean()),
               plain_xi_median=float(np.median(plain["xi"])), warm_xi_median=float(np.median(warm["xi"])),
               fallbacks=int(((warm["flags"] & 4) != 0).sum()),
               iters_saved_mean=float((plain["iters"] - warm["iters"]).mean()),
               equal_quality=dict(
                   maps_reaching_plain_quality_warm=int(reached_w.sum()),
                   maps_reaching_plain_quality_plain=int(reached_p.sum()),
                   warm_iters_mean=float(eqw["iters"].mean()), plain_iters_mean=float(eqp["iters"].mean()),
                   plain_ms_per_cartogram=eq_ms["plain"],
                   warm_ms_per_cartogram=eq_ms["warm"] + (t2 - t1) * 1e3 / n,   # with the net's inputs and forward
                   iters_saved_mean_where_both_reach=float((eqp["iters"] - eqw["iters"])[reached_w & reached_p].mean())
                   if (reached_w & reached_p).any() else None),
               warm_field_pool=WARM_POOL)
    # time to the 1% max area error: the maps that reach it on both sides,
    # run again as their own batches (the plain side also one per call)
    both = np.nonzero((plain["status"] == 0) & (warm["status"] == 0))[0]
    if len(both):
        sm = [maps[i] for i in both]
        sg = [gmaps[i] for i in both]
        sd = ([dev[0][i] for i in both], [dev[1][i] for i in both])
        torch.cuda.synchronize()
        u0 = time.perf_counter()
        run_batched(ctx, sg, sm, None, N, batch, graph_iters, dev=sd, **kw)
        torch.cuda.synchronize()
        u1 = time.perf_counter()
        Fs = predict(net, features(ctx, sm, N, gmaps=sg, dev=sd, **kw), pool=WARM_POOL)
        run_batched(ctx, sg, sm, Fs, N, batch, graph_iters, dev=sd, **kw)
        torch.cuda.synchronize()
        u2 = time.perf_counter()
        ks = min(len(both), 16)
        run_batched(ctx, sg[:ks], sm[:ks], None, N, 1, graph_iters, dev=(sd[0][:ks], sd[1][:ks]), **kw)
        torch.cuda.synchronize()
        u3 = time.perf_counter()
        rep["to_tol"] = dict(maps=int(len(both)), plain_ms_per_cartogram=(u1 - u0) * 1e3 / len(both),
                             warm_ms_per_cartogram=(u2 - u1) * 1e3 / len(both),
                             plain_single_ms_per_cartogram=(u3 - u2) * 1e3 / ks, plain_single_maps=ks)
    else:
        rep["to_tol"] = None
    if single > 0:
        k = min(single, n)
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        run_batched(ctx, gmaps[:k], maps[:k], None, N, 1, graph_iters, dev=dv(0, k), **kw)
        torch.cuda.synchronize()
        rep["plain_single_ms_per_cartogram"] = (time.perf_counter() - t4) * 1e3 / k
    return rep


def main(argv=None):
    import torch
    from paper_2604_13880_amd import binding as B
    ap = argparse.ArgumentParser()
    ap.add_argument("cmd", choices=["train", "eval"])
    ap.add_argument("--out", default=os.path.join(HERE, "weights", WEIGHTS_NAME))
    ap.add_argument("--weights", default=os.path.join(HERE, "weights", WEIGHTS_NAME))
    ap.add_argument("--maps", type=int, default=10000)
    ap.add_argument("--epochs", type=int, default=4)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--max-train-seconds", type=float, default=None)
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--max-iters", type=int, default=512)
    ap.add_argument("--area-source", type=int, default=1, help="0 pixel counts, 1 polygon areas")
    ap.add_argument("--eval-maps", type=int, default=0, help="after training, compare on this many held-out maps")
    ap.add_argument("--single", type=int, default=0, help="also time the plain method one cartogram per call")
    ap.add_argument("--base-channels", type=int, default=NET_CFG["base_channels"])
    ap.add_argument("--json", default=None)
    a = ap.parse_args(argv)
    log = lambda *m: print(*m, file=sys.stderr, flush=True)
    ctx = B.Context(0)
    report = {}
    kw = dict(max_iters=a.max_iters, area_source=a.area_source)
    if a.cmd == "train":
        t1 = time.perf_counter()
        X = torch.empty((a.maps, N_NET, N_NET, 3), dtype=torch.float32, device="cuda")
        Y = torch.empty((a.maps, N_NET, N_NET, 2), dtype=torch.float32, device="cuda")
        its, sts, xis = [], [], []
        chunk = 1024
        for c0 in range(0, a.maps, chunk):
            c1 = min(a.maps, c0 + chunk)
            maps = make_maps(range(TRAIN_SEED0 + c0, TRAIN_SEED0 + c1), workers=a.workers)
            gm = [ctx.map_from(m) for m, s in maps]
            X[c0:c1] = features(ctx, maps, gmaps=gm, **kw)
            Yc, st = plain_runs(ctx, maps, N_TEX, N_NET, gmaps=gm, **kw)
            Y[c0:c1] = Yc
            its.append(st["iters"])
            sts.append(st["status"])
            xis.append(st["xi"])
            del maps, Yc, gm
            log(f"data {c1}/{a.maps} after {time.perf_counter() - t1:.1f}s")
        st = dict(iters=np.concatenate(its), status=np.concatenate(sts), xi=np.concatenate(xis))
        torch.cuda.synchronize()
        log(f"training data in {time.perf_counter() - t1:.1f}s: iterations mean {st['iters'].mean():.1f}, "
            f"converged {(st['status'] == 0).sum()}, xi mean {st['xi'].mean():.4f}")
        cfg = dict(NET_CFG, base_channels=a.base_channels)
        net = B.Net(ctx, max_batch=max(a.batch, 8), seed=1, **cfg)
        t2 = time.perf_counter()
        hist = train(net, X, Y, epochs=a.epochs, batch=a.batch, lr=a.lr, log=log, max_seconds=a.max_train_seconds)
        torch.cuda.synchronize()
        os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
        net.save(a.out)
        report = dict(maps=a.maps, area_source=a.area_source, data_seconds=t2 - t1,
                      train_seconds=time.perf_counter() - t2, epochs=len(hist), loss=hist,
                      plain_iters_mean=float(st["iters"].mean()), plain_converged=int((st["status"] == 0).sum()),
                      plain_xi_mean=float(st["xi"].mean()))
        log(f"saved {a.out}")
        if a.eval_maps > 0:
            maps = make_maps(range(TEST_SEED0, TEST_SEED0 + a.eval_maps), workers=a.workers)
            report["eval"] = compare(ctx, net, maps, single=a.single, **kw)
    else:
        net = B.Net(ctx, max_batch=PREDICT_BATCH, **dict(NET_CFG, base_channels=a.base_channels))
        net.load(a.weights)
        maps = make_maps(range(TEST_SEED0, TEST_SEED0 + a.maps), workers=a.workers)
        report = compare(ctx, net, maps, single=a.single, **kw)
    print(json.dumps(report), flush=True)
    if a.json:
        with open(a.json, "w") as f:
            json.dump(report, f)


if __name__ == "__main__":
    main()
