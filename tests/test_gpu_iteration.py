"""The one-call iteration hts_iteration_bh (tree, Barnes-Hut gradient and step)
against the three separate calls: the same Y, update, gains, gradient and Z
bit for bit, iteration after iteration; replayed from a captured HIP graph
too."""
import numpy as np
import pytest
import torch

from paper_2401_13708_amd import hts, synth
from paper_2401_13708_amd.embed import Schedule
from gpu_inputs import affinities, embedding

pytestmark = pytest.mark.gpu


def _d(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _state(n, dtype, stage, seed):
    Y = embedding(n, stage, dtype, seed=seed)
    U = np.zeros_like(Y)
    G = np.ones_like(Y)
    return [_d(Y), _d(U), _d(G)]


def _separate(ctx, st, P, tree, theta, ex, eta, mu, grad, z):
    Y, U, G = st
    hts.build_polar_tree(ctx, Y, tree)
    hts.gradient_bh(ctx, Y, *P, tree, theta, ex, grad, z)
    hts.step(ctx, Y, U, G, grad, eta, mu)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("n,stage", [(3000, "late"), (2, "mid"), (65, "early"), (1337, "edge")])
def test_fused_iteration_equals_the_three_calls(ctx, dtype, n, stage):
    _, _, rp, col, val = affinities(max(n, 3))
    if n < 3:
        rp, col, val = synth.random_csr(n, 1, seed=7, dtype=np.float64)
    P = [_d(rp), _d(col), _d(val.astype(dtype))]
    a = _state(n, dtype, stage, 11)
    b = [t.clone() for t in a]
    ta, tb = hts.Tree(ctx, n, 20), hts.Tree(ctx, n, 20)
    ga, gb = torch.empty_like(a[0]), torch.empty_like(b[0])
    za, zb = torch.zeros(1, dtype=torch.float64, device="cuda"), torch.zeros(1, dtype=torch.float64,
                                                                             device="cuda")
    sched = Schedule()
    for it in range(240, 262):          # across the end of early exaggeration
        ex, mu, eta = sched.at(it, n)
        hts.iteration_bh(ctx, *a, *P, ta, 0.5, ex, eta, mu, ga, za)
        _separate(ctx, b, P, tb, 0.5, ex, eta, mu, gb, zb)
        torch.cuda.synchronize()
        for x, y, nm in zip(a + [ga, za], b + [gb, zb], ("Y", "update", "gains", "grad", "z")):
            assert torch.equal(x, y), (it, nm)
    assert ctx.check() == 0
    ta.close()
    tb.close()


def test_fused_iteration_replayed_from_a_graph(ctx):
    # captured once, replayed with other work between the replays: every
    # replay is the next eager iteration
    n = 4099
    _, _, rp, col, val = affinities(n)
    P = [_d(rp), _d(col), _d(val.astype(np.float32))]
    a = _state(n, np.float32, "mid", 12)
    b = [t.clone() for t in a]
    ta, tb = hts.Tree(ctx, n, 20), hts.Tree(ctx, n, 20)
    ga, gb = torch.empty_like(a[0]), torch.empty_like(b[0])
    za, zb = torch.zeros(1, dtype=torch.float64, device="cuda"), torch.zeros(1, dtype=torch.float64,
                                                                             device="cuda")
    ex, mu, eta = 1.0, 0.8, n / 12000.0
    # the eager iteration before the capture creates the workspaces
    hts.iteration_bh(ctx, *a, *P, ta, 0.5, ex, eta, mu, ga, za)
    _separate(ctx, b, P, tb, 0.5, ex, eta, mu, gb, zb)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        hts.iteration_bh(ctx, *a, *P, ta, 0.5, ex, eta, mu, ga, za)
    scratch = torch.ones(1 << 20, device="cuda")
    for k in range(6):
        g.replay()
        scratch.mul_(1.0001)
        _separate(ctx, b, P, tb, 0.5, ex, eta, mu, gb, zb)
        torch.cuda.synchronize()
        for x, y, nm in zip(a + [ga, za], b + [gb, zb], ("Y", "update", "gains", "grad", "z")):
            assert torch.equal(x, y), (k, nm)
    assert ctx.check() == 0
    del g
    ta.close()
    tb.close()


def test_fused_iteration_argument_errors(ctx):
    n = 300
    _, _, rp, col, val = affinities(n)
    P = [_d(rp), _d(col), _d(val.astype(np.float32))]
    st = _state(n, np.float32, "mid", 13)
    grad = torch.empty_like(st[0])
    small = hts.Tree(ctx, 100, 20)
    with pytest.raises(hts.HTSError, match="n_max"):
        hts.iteration_bh(ctx, *st, *P, small, 0.5, 1.0, 0.1, 0.5, grad)
    small.close()
    other = hts.Context(0)
    t_other = hts.Tree(other, n, 20)
    with pytest.raises(hts.HTSError, match="another context"):
        hts.iteration_bh(ctx, *st, *P, t_other, 0.5, 1.0, 0.1, 0.5, grad)
    t_other.close()
    other.close()
    jobs = hts.Tree(ctx, n, 20)
    jobs.set_jobs([100, 200])
    with pytest.raises(hts.HTSError, match="jobs"):
        hts.iteration_bh(ctx, *st, *P, jobs, 0.5, 1.0, 0.1, 0.5, grad)
    jobs.close()
    t = hts.Tree(ctx, n, 20)
    with pytest.raises(hts.HTSError, match="momentum"):
        hts.iteration_bh(ctx, *st, *P, t, 0.5, 1.0, 0.1, 1.5, grad)
    t.close()
