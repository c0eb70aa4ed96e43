"""The stored whole-run histories of the 1024^2 cartograms
(tests/golden/c2_xi_history.txt) are the oracle's: its first iterations on
one map are recomputed here and must reproduce the stored errors, and the
stored runs must obey the stopping rule they were written under (Method,
end of 'Construction of Static Cartograms')."""
import os

import numpy as np

from oracle import cartogram as oc
from synth import lognormal_values, voronoi_map

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "c2_xi_history.txt")


def _read():
    runs, hist = {}, {}
    with open(GOLDEN) as fh:
        for line in fh:
            f = line.split()
            if not f or f[0].startswith("#"):
                continue
            if f[0] == "run":
                runs[int(f[1])] = (int(f[2]), f[3], float(f[4]), float(f[5]))
            else:
                hist.setdefault(int(f[1]), {})[int(f[2])] = float(f[3])
    return runs, hist


def test_first_iterations_reproduce_the_stored_history():
    runs, hist = _read()
    seed = 2005
    m = voronoi_map(seed, 100, 50000, fractal=True)
    s = lognormal_values(seed, 100, 1.5).astype(np.float32).astype(np.float64)
    r = oc.run(m, s, 1024, fixed_iters=8)
    for k in (0, 4, 8):
        assert abs(r.xi_history[k] - hist[seed][k]) <= 1e-8 * max(1.0, hist[seed][k])


def test_stored_runs_follow_the_stopping_rule():
    runs, hist = _read()
    assert sorted(runs) == list(range(2000, 2010))
    for seed, (iters, status, eps, xi) in runs.items():
        h = hist[seed]
        assert h[iters] == xi and 0 < eps <= xi
        # every run ended at the cap: no error below 1% was ever recorded
        assert status == "maxiter" and iters == 512
        assert min(h.values()) >= 0.01
