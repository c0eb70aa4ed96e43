"""Writes c2_xi_history.txt: the FP64 oracle's max-area-error history of
the ten seeded 1024^2 cartograms (100 fractal Voronoi regions, ~50k
vertices, lognormal values sigma 1.5; seeds 2000-2009) run with the
stopping rule of the static construction (max area error below 1%, no new
minimum within 32 iterations, at most 512 iterations; pixel-count
density, shape parameter 1).

Calls only the oracle and the seeded input generators.  Takes about
one to three minutes per map and core, depending on the host; the maps
run in parallel processes and report every 64 iterations.

    python tests/golden/make_c2_xi_history.py [--workers 8]
"""
from __future__ import annotations

import argparse
import os
import sys
import time

os.environ.setdefault("OMP_NUM_THREADS", "1")
os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")
os.environ.setdefault("MKL_NUM_THREADS", "1")

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

SEEDS = list(range(2000, 2010))
R, N_VERT, SIGMA, N = 100, 50000, 1.5, 1024
EVERY = 4          # history kept every EVERY iterations (and the last one)


def one(seed: int):
    import numpy as np
    from oracle import cartogram as oc
    from synth import lognormal_values, voronoi_map
    m = voronoi_map(seed, R, N_VERT, fractal=True)
    s = lognormal_values(seed, R, SIGMA).astype(np.float32).astype(np.float64)
    t0 = time.perf_counter()

    def report(k, xi):
        if k % 64 == 0:
            print(f"seed {seed}: iteration {k}, xi {xi:.4f} ({time.perf_counter() - t0:.0f} s)", flush=True)

    r = oc.run(m, s, N, progress=report)
    return seed, r.iters, r.status, r.eps, r.xi, r.xi_history, time.perf_counter() - t0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--out", default=os.path.join(HERE, "c2_xi_history.txt"))
    a = ap.parse_args()
    import multiprocessing as mp
    names = ["converged", "stalled", "maxiter"]
    res = []
    with mp.get_context("fork").Pool(a.workers) as pool:
        for r in pool.imap_unordered(one, SEEDS, chunksize=1):   # each map reported as it ends
            res.append(r)
            print(f"seed {r[0]}: {r[1]} iterations, {names[r[2]]}, xi {r[4]:.4f} ({r[6]:.0f} s)", flush=True)
    res.sort()
    with open(a.out, "w") as fh:
        fh.write("# Max area error history of the FP64 oracle on the ten seeded 1024^2\n"
                 "# cartograms (100 fractal Voronoi regions, ~50k vertices, lognormal\n"
                 "# sigma 1.5, seeds 2000-2009), run with the stopping rule of the static\n"
                 "# construction (Method, end of 'Construction of Static Cartograms':\n"
                 "# max area error < 0.01, no new minimum within 32 iterations, at most\n"
                 "# 512 iterations); pixel-count density, shape parameter 1.\n"
                 "# Written by tests/golden/make_c2_xi_history.py (oracle only).\n"
                 f"# format: run <seed> <iterations> <status> <final eps> <final xi>\n"
                 f"#         xi <seed> <iteration> <xi>   (every {EVERY} iterations and the last)\n")
        for seed, iters, status, eps, xi, hist, dt in res:
            fh.write(f"run {seed} {iters} {names[status]} {eps:.9g} {xi:.9g}\n")
            for k, v in enumerate(hist):
                if k % EVERY == 0 or k == len(hist) - 1:
                    fh.write(f"xi {seed} {k} {v:.9g}\n")


if __name__ == "__main__":
    main()
