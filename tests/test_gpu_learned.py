"""What the trained warm-start net gains over the plain method, on
held-out seeded maps (512^2, 50-150 fractal regions, lognormal sigma 1,
polygon-area density), both sides batched 32 cartograms per call.

The net (weights under paper_2604_13880_amd/weights, written by
`python -m paper_2604_13880_amd.learned train`) predicts the converged
displacement from the log-density and the first plain iteration; the
graded warm start applies it, and the plain iteration runs to the same
stopping rule.  Gains asserted: the warm-started runs end with a lower
mean max-area-error, and reach the plain runs' final error in fewer
iterations where both reach it."""
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_2604_13880_amd.learned import WEIGHTS_NAME

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WEIGHTS = os.path.join(ROOT, "paper_2604_13880_amd", "weights", WEIGHTS_NAME)


def test_learned_warm_start_gain():
    import torch
    from paper_2604_13880_amd import binding as B
    from paper_2604_13880_amd import learned as Lr
    assert os.path.exists(WEIGHTS), "trained weights are part of the repository"
    ctx = B.Context(0)
    net = B.Net(ctx, max_batch=Lr.PREDICT_BATCH, **Lr.NET_CFG)
    net.load(WEIGHTS)
    maps = Lr.make_maps(range(Lr.TEST_SEED0, Lr.TEST_SEED0 + 32), workers=8)
    rep = Lr.compare(ctx, net, maps, area_source=1)
    print(json.dumps(rep), flush=True)
    assert rep["warm_xi_mean"] < rep["plain_xi_mean"]
    eq = rep["equal_quality"]
    assert eq["iters_saved_mean_where_both_reach"] is not None and eq["iters_saved_mean_where_both_reach"] > 0
    net.close()
    torch.cuda.synchronize()
    ctx.close()
