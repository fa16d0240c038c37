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


def test_footprint_covers_a_running_job():
    # the admission estimate bounds what one job's iterations add on the
    # device beyond its P: tree storage, traversal workspace and state
    # (measured on a fresh context, after P is built)
    from paper_2401_13708_amd import hts
    from paper_2401_13708_amd.embed import Embedding
    n, k = 20000, 90
    c = hts.Context(0)
    try:
        X = torch.from_numpy(synth.gaussian_mixture(n, 16, seed=9)).float().cuda()
        _, rp, col, val = hts.build_affinities(c, X, 30.0, k, p_dtype=torch.float32, want_knn=False)
        del X
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        free0 = torch.cuda.mem_get_info()[0]
        Y0 = torch.from_numpy(synth.disk_uniform(n, 1e-4, seed=4)).cuda()
        emb = Embedding(c, rp, col, val, Y0, theta=0.5)
        emb.run(300)     # past early exaggeration: the walks and their item lists have grown
        torch.cuda.synchronize()
        assert c.check() == 0
        used = free0 - torch.cuda.mem_get_info()[0]
        p_bytes = rp.numel() * 8 + col.numel() * 4 + val.numel() * 4
        est = footprint_bytes(n, k, 20, c.item_list) - p_bytes
        print("n", n, "used", used, "estimate beyond P", est, flush=True)
        assert used <= est, (used, est)
        # and it is not a loose bound: the traversal workspace dominates both
        assert used >= 0.6 * est, (used, est)
        emb.close()
    finally:
        c.close()
