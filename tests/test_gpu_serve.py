"""Continuous-batching server: jobs that arrive while others run are admitted
as the HBM budget allows, run side by side in one job layout, and each
result equals the same job run alone (bit for bit), whatever it ran beside."""
import numpy as np
import pytest
import torch

from paper_2401_13708_amd import synth
from paper_2401_13708_amd.embed import Schedule
from paper_2401_13708_amd.serve import FifoServer, Request, Server, footprint_bytes, summarize

pytestmark = pytest.mark.gpu


def _requests(iters=40):
    sizes = [400, 1500, 90, 700, 2500, 300]
    arrivals = [0.0, 0.0, 0.02, 0.05, 0.1, 0.1]
    reqs = []
    for j, (n, t) in enumerate(zip(sizes, arrivals)):
        X = synth.branching_walk(n, 16, depth=4, seed=600 + j).astype(np.float32)
        reqs.append(Request(j, t, X, iters=iters + 7 * j, seed=700 + j))
    return reqs


def test_served_results_equal_results_alone(ctx):
    sched = Schedule(ee_iters=20)
    reqs = _requests()
    budget = footprint_bytes(2500) + footprint_bytes(1500) + footprint_bytes(400)
    srv = Server(ctx, budget, schedule=sched)
    got = {r.rid: r for r in srv.run(reqs)}
    alone = {r.rid: r for r in FifoServer(ctx, schedule=sched).run(reqs)}
    assert sorted(got) == sorted(alone) == list(range(len(reqs)))
    for rid in got:
        assert np.array_equal(got[rid].Y, alone[rid].Y), rid
    # jobs ran side by side, and never beyond the budget (one big job alone
    # may exceed it)
    assert srv.max_active >= 2
    assert srv.relayouts >= 2
    s = summarize(list(got.values()))
    assert s["jobs"] == len(reqs) and s["p99_latency_s"] >= s["p50_latency_s"] > 0


def test_budget_smaller_than_a_job_serves_one_at_a_time(ctx):
    sched = Schedule(ee_iters=5)
    reqs = _requests(iters=10)[:3]
    srv = Server(ctx, 1, schedule=sched)
    out = srv.run(reqs)
    assert srv.max_active == 1 and len(out) == 3
