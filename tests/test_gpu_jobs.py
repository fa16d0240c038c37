"""Several embeddings in one job layout: each job's tree, gradient, Z, step
and whole iterations are bit for bit those of the same job alone (whose
parity with the oracle the other GPU tests establish), and one job of a mix is
also checked against the oracle directly.

Sizes are ragged: a 2-point job, sizes just above and at a multiple of the
64-point query block, jobs smaller than one 256-point build block next to
jobs spanning many, and jobs at different stages (radii) of an embedding."""
import numpy as np
import pytest
import torch

import oracle
from paper_2401_13708_amd import hts, synth
from paper_2401_13708_amd.batch import Job, JobBatch
from paper_2401_13708_amd.embed import Embedding
from gpu_inputs import STAGES, embedding, rel

pytestmark = pytest.mark.gpu

SIZES = [700, 2, 257, 3000, 64, 65, 1000, 3, 129]


def _jobs(dtype, sizes=SIZES, seed=40):
    out = []
    for j, n in enumerate(sizes):
        Y = embedding(n, STAGES[j % len(STAGES)], dtype, seed=seed + j)
        rp, col, val = synth.random_csr(n, min(30, n - 1), seed=seed + 100 + j, dtype=dtype)
        out.append((Y, rp, col, val))
    return out


def _concat(parts):
    Y = np.concatenate([p[0] for p in parts])
    rps, cols, vals, nnz, off = [], [], [], 0, 0
    for Yj, rp, col, val in parts:
        rps.append(rp[:-1] + nnz)
        cols.append(col + off)
        vals.append(val)
        nnz += col.size
        off += Yj.shape[0]
    rps.append(np.array([nnz]))
    return Y, np.concatenate(rps).astype(np.int64), np.concatenate(cols).astype(np.int32), \
        np.concatenate(vals)


def _d(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _single_tree(ctx, Y):
    t = hts.Tree(ctx, Y.shape[0], 20)
    hts.build_polar_tree(ctx, _d(Y), t)
    e = hts.tree_export(ctx, t, Y.shape[0])
    t.close()
    return e


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_job_trees_match_single_trees(ctx, dtype):
    parts = _jobs(dtype)
    Y, _, _, _ = _concat(parts)
    t = hts.Tree(ctx, Y.shape[0] + 100, 20)
    t.set_jobs(SIZES)
    hts.build_polar_tree(ctx, _d(Y), t)
    e = hts.tree_export(ctx, t, Y.shape[0])
    t.close()
    k0, p0 = 0, 0
    for (Yj, _, _, _) in parts:
        s = _single_tree(ctx, Yj)
        m = s["count"].size
        sl = slice(k0, k0 + m)
        for key in ("count", "depth"):
            assert np.array_equal(e[key][sl], s[key]), key
        assert np.array_equal(e["next"][sl] - k0, s["next"])
        assert np.array_equal(e["first"][sl] - p0, s["first"])
        assert np.array_equal(e["mid"][sl], s["mid"])
        assert np.array_equal(e["r_cell"][sl], s["r_cell"])
        assert np.array_equal(e["perm"][p0:p0 + Yj.shape[0]] - p0, s["perm"])
        k0 += m
        p0 += Yj.shape[0]
    assert k0 == e["count"].size


def _single_bh(ctx, Yj, rp, col, val, ex, theta):
    t = hts.Tree(ctx, Yj.shape[0], 20)
    Yd = _d(Yj)
    hts.build_polar_tree(ctx, Yd, t)
    g, z = hts.gradient_bh(ctx, Yd, _d(rp), _d(col), _d(val), t, theta, ex)
    torch.cuda.synchronize()
    t.close()
    return g.cpu().numpy(), float(z.cpu()[0])


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("theta,item_list", [(0.5, None), (0.0, None), (0.5, 1)])
def test_job_gradients_match_single(ctx, dtype, theta, item_list):
    # with a one-item share per phase-A wave as well: the waves of a job are
    # the same in the layout and alone, so are their splits
    if item_list is not None:
        ctx.set_item_points(16)
        ctx.set_item_list(item_list)
    try:
        _job_gradients_match_single(ctx, dtype, theta)
    finally:
        ctx.set_item_points(hts.DEFAULT_ITEM_POINTS)
        ctx.set_item_list(hts.DEFAULT_ITEM_LIST)


def _job_gradients_match_single(ctx, dtype, theta):
    parts = _jobs(dtype)
    Y, rp, col, val = _concat(parts)
    exs = np.array([12.0 if j % 2 else 1.0 for j in range(len(SIZES))])
    t = hts.Tree(ctx, Y.shape[0], 20)
    t.set_jobs(SIZES)
    Yd = _d(Y)
    hts.build_polar_tree(ctx, Yd, t)
    g, z = hts.gradient_bh_jobs(ctx, Yd, _d(rp), _d(col), _d(val), t, _d(exs), theta)
    torch.cuda.synchronize()
    assert ctx.check() == 0
    t.close()
    g, z = g.cpu().numpy(), z.cpu().numpy()
    p0 = 0
    for j, (Yj, rpj, colj, valj) in enumerate(parts):
        gs, zs = _single_bh(ctx, Yj, rpj, colj, valj, exs[j], theta)
        assert np.array_equal(g[p0:p0 + Yj.shape[0]], gs), j
        assert z[j] == zs, j
        p0 += Yj.shape[0]


def test_job_gradient_matches_oracle(ctx):
    parts = _jobs(np.float64)
    Y, rp, col, val = _concat(parts)
    t = hts.Tree(ctx, Y.shape[0], 20)
    t.set_jobs(SIZES)
    Yd = _d(Y)
    hts.build_polar_tree(ctx, Yd, t)
    g, z = hts.gradient_bh_jobs(ctx, Yd, _d(rp), _d(col), _d(val), t,
                                _d(np.full(len(SIZES), 12.0)), 0.5)
    torch.cuda.synchronize()
    t.close()
    g, z = g.cpu().numpy(), z.cpu().numpy()
    p0 = 0
    for j, (Yj, rpj, colj, valj) in enumerate(parts):
        if Yj.shape[0] >= 64:
            go, zo, _ = oracle.gradient_bh(Yj, rpj, colj, valj, oracle.Tree(Yj), 0.5, 12.0)
            assert rel(g[p0:p0 + Yj.shape[0]], go) < 1e-10, j
            assert z[j] == pytest.approx(zo, rel=1e-10), j
        p0 += Yj.shape[0]


def test_job_steps_match_single(ctx):
    parts = _jobs(np.float32)
    Y, _, _, _ = _concat(parts)
    n = Y.shape[0]
    g = synth.rng(8)
    U = (g.normal(size=(n, 2)) * 1e-3).astype(np.float32)
    G = g.uniform(0.2, 3.0, size=(n, 2)).astype(np.float32)
    grad = (g.normal(size=(n, 2)) * 10).astype(np.float32)
    eta = np.array([s / 12000.0 for s in SIZES])
    mu = np.array([0.5 if j % 3 else 0.8 for j in range(len(SIZES))])
    t = hts.Tree(ctx, n, 20)
    t.set_jobs(SIZES)
    st = [_d(a.copy()) for a in (Y, U, G, grad)]
    hts.step_jobs(ctx, t, st[0], st[1], st[2], st[3], _d(eta), _d(mu))
    torch.cuda.synchronize()
    t.close()
    p0 = 0
    for j, n_j in enumerate(SIZES):
        sl = slice(p0, p0 + n_j)
        one = [_d(a[sl].copy()) for a in (Y, U, G, grad)]
        hts.step(ctx, one[0], one[1], one[2], one[3], eta[j], mu[j])
        torch.cuda.synchronize()
        for a, b in zip(st[:3], one[:3]):
            assert torch.equal(a[sl], b), j
        p0 += n_j


def test_jobs_schedule(ctx):
    it = torch.tensor([0, 249, 250, 600], dtype=torch.int32, device="cuda")
    ex = torch.empty(4, dtype=torch.float64, device="cuda")
    mu = torch.empty_like(ex)
    hts.jobs_schedule(ctx, it, 250, 12.0, 0.5, 0.8, ex, mu)
    assert ex.cpu().tolist() == [12.0, 12.0, 1.0, 1.0]
    assert mu.cpu().tolist() == [0.5, 0.5, 0.8, 0.8]
    assert it.cpu().tolist() == [1, 250, 251, 601]


def test_batch_iterations_match_single_runs(ctx):
    # whole iterations (schedule, tree, gradient, step) across the switch at
    # iteration 250, with one job started 240 iterations later than the rest
    sizes = [900, 2, 300, 65, 2000]
    jobs, singles = [], []
    for j, n in enumerate(sizes):
        Y0 = synth.disk_uniform(n, 1e-4, seed=70 + j)
        rp, col, val = synth.random_csr(n, min(30, n - 1), seed=80 + j, dtype=np.float32)
        jobs.append(Job(_d(rp), _d(col), _d(val), _d(Y0)))
    start = [0, 0, 240, 0, 0]
    b = JobBatch(ctx, jobs, start_iter=start)
    b.run(20)
    torch.cuda.synchronize()
    assert ctx.check() == 0
    for j, job in enumerate(jobs):
        e = Embedding(ctx, job.rp, job.col, job.val, job.Y0)
        e.it = start[j]
        e.run(20)
        torch.cuda.synchronize()
        Yb, Ub, Gb = b.state(j)
        assert torch.equal(Yb, e.Y), j
        assert torch.equal(Ub, e.update), j
        assert torch.equal(Gb, e.gains), j
        e.close()
    b.close()


def test_set_jobs_validation(ctx):
    t = hts.Tree(ctx, 100, 20)
    with pytest.raises(hts.HTSError):
        t.set_jobs([50, 1])
    with pytest.raises(hts.HTSError):
        t.set_jobs([60, 60])
    t.set_jobs([50, 40])
    Y = _d(embedding(80, "mid", np.float32))
    with pytest.raises(hts.HTSError):
        hts.build_polar_tree(ctx, Y, t)      # 80 points, the layout holds 90
    t.close()


def test_graph_replays_equal_eager_iterations(ctx):
    # one iteration of all jobs captured as a HIP graph and replayed: every
    # replay equals the eager iteration, with other GPU work in between
    sizes = [700, 2, 3000, 65]
    jobs = []
    for j, n in enumerate(sizes):
        Y0 = synth.disk_uniform(n, 1e-4, seed=90 + j)
        rp, col, val = synth.random_csr(n, min(30, n - 1), seed=95 + j, dtype=np.float32)
        jobs.append(Job(_d(rp), _d(col), _d(val), _d(Y0)))
    start = [0, 245, 0, 10]
    eager = JobBatch(ctx, jobs, start_iter=start)
    want = []
    for _ in range(12):
        eager.iterate()
        want.append(eager.Y.clone())
    torch.cuda.synchronize()
    b = JobBatch(ctx, jobs, start_iter=start).capture()     # the first iteration runs eagerly
    assert torch.equal(b.Y, want[0])
    scratch = torch.ones(1 << 20, device="cuda")
    for k in range(1, 12):
        b.iterate()
        scratch.mul_(1.0001)                                   # unrelated work between replays
        torch.cuda.synchronize()
        assert torch.equal(b.Y, want[k]), k
    assert ctx.check() == 0
    eager.close()
    b.close()


def test_set_jobs_rejects_job_bits_beyond_the_key(ctx):
    # the job index sits above the 2 max_depth cell bits of a 64-bit key:
    # at depth 24, 2^16 jobs fill the key exactly and one more cannot fit
    t = hts.Tree(ctx, 2 * (1 << 16) + 2, 24)
    with pytest.raises(hts.HTSError, match="key bits"):
        t.set_jobs([2] * ((1 << 16) + 1))
    t.set_jobs([2] * (1 << 16))
    t.close()


def test_graph_recaptured_after_workspace_growth():
    # a captured batch iteration points into the context's workspaces; when a
    # later call on the context grows one (here an exact gradient of a larger
    # embedding), the next iteration runs eagerly and is captured again
    # instead of replaying into freed memory, and every iteration still
    # equals the eager run
    c = hts.Context(0)
    sizes = [500, 65, 1200]
    jobs = []
    for j, n in enumerate(sizes):
        Y0 = synth.disk_uniform(n, 1e-4, seed=130 + j)
        rp, col, val = synth.random_csr(n, min(30, n - 1), seed=135 + j, dtype=np.float32)
        jobs.append(Job(_d(rp), _d(col), _d(val), _d(Y0)))
    eager = JobBatch(c, jobs)
    want = []
    for _ in range(8):
        eager.iterate()
        want.append(eager.Y.clone())
    eager.close()
    b = JobBatch(c, jobs).capture()
    assert torch.equal(b.Y, want[0])
    g0 = c.generation()
    for k in (1, 2, 3):
        b.iterate()
        torch.cuda.synchronize()
        assert torch.equal(b.Y, want[k]), k
    n = 30000
    Yl = _d(synth.disk_state(n, "mid", seed=140))
    rp, col, val = synth.random_csr(n, 30, seed=141, dtype=np.float32)
    hts.gradient_exact(c, Yl, _d(rp), _d(col), _d(val), 1.0)
    torch.cuda.synchronize()
    assert c.generation() != g0
    for k in range(4, 8):
        b.iterate()
        torch.cuda.synchronize()
        assert torch.equal(b.Y, want[k]), k
    assert b.graph_gen == c.generation()
    assert c.check() == 0
    b.close()
    c.close()
