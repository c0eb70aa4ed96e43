"""Whole runs of the ten seeded 1024^2 cartograms (100 fractal Voronoi
regions, ~50k vertices, lognormal sigma 1.5) on the GPU against the FP64
oracle's runs recorded in tests/golden/c2_xi_history.txt (written by the
oracle alone): same stopping status and iteration count, and the final
mean and max area errors within stated bounds.

Bounds.  One iteration of the GPU path matches the oracle's to 1e-6 in
position on identical inputs, but over hundreds of iterations the float32
state and the label flips it causes let the two trajectories drift apart;
the max area error is a maximum over regions of relative errors and its
value at the iteration cap is set by the few regions with the most extreme
values.  The bound is the stopping tolerance itself, 0.01 in the max area
error, and 0.002 in the mean error (measured: at most 0.0011 and 0.0001).
The comparison includes the iteration at which each run stops, since the
cap (512) ends every run here: the method does not reach a 1% max area
error on these maps, in FP64 or on the GPU."""
import os

import numpy as np
import pytest

from synth import lognormal_values, voronoi_map

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "c2_xi_history.txt")
STATUS = {"converged": 0, "stalled": 1, "maxiter": 2}


def golden():
    runs, hist = {}, {}
    with open(GOLDEN) as fh:
        for line in fh:
            f = line.split()
            if not f or f[0].startswith("#"):
                continue
            if f[0] == "run":
                runs[int(f[1])] = (int(f[2]), STATUS[f[3]], float(f[4]), float(f[5]))
            else:
                hist.setdefault(int(f[1]), {})[int(f[2])] = float(f[3])
    return runs, hist


@pytest.fixture(scope="module")
def ctx():
    from paper_2604_13880_amd import binding as B
    c = B.Context(0)
    yield c
    c.close()


def test_ten_whole_runs_match_the_oracle(ctx):
    runs, _ = golden()
    assert sorted(runs) == list(range(2000, 2010))
    for seed, (iters, status, eps, xi) in sorted(runs.items()):
        m = voronoi_map(seed, 100, 50000, fractal=True)
        s = lognormal_values(seed, 100, 1.5).astype(np.float32)
        gm = ctx.map_from(m)
        r = ctx.step_series([dict(map=gm, xy0=m.xy32(), N=1024, values=s, precision=1)], graph_iters=32)[0]
        print(f"seed {seed}: gpu {int(r['iters'][0])} it xi {float(r['xi'][0]):.5f}, oracle {iters} it xi {xi:.5f}",
              flush=True)
        assert int(r["status"][0]) == status and int(r["iters"][0]) == iters
        assert abs(float(r["xi"][0]) - xi) <= 0.01
        assert abs(float(r["eps"][0]) - eps) <= 0.002


@pytest.mark.parametrize("seed", [2000, 2005])
def test_intermediate_errors_match_the_oracle_history(ctx, seed):
    _, hist = golden()
    m = voronoi_map(seed, 100, 50000, fractal=True)
    s = lognormal_values(seed, 100, 1.5).astype(np.float32)
    gm = ctx.map_from(m)
    for k in (16, 64, 256):
        r = ctx.step_series([dict(map=gm, xy0=m.xy32(), N=1024, values=s, precision=1, max_iters=k)],
                            graph_iters=32)[0]
        assert int(r["iters"][0]) == k
        assert abs(float(r["xi"][0]) - hist[seed][k]) <= 0.01, (k, float(r["xi"][0]), hist[seed][k])
