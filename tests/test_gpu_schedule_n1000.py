"""The small workload end to end: N = 1000 points, D = 32 (10 Gaussian
clusters, seed 1), FP64, perplexity 30 and k = 90, the whole 750-iteration
schedule of Sec. 5 (250 iterations with exaggeration 12 and momentum 0.5,
then 500 with momentum 0.8; learning rate n / 12000) from a uniform disk of
radius 1e-4, run by the GPU driver and by the same loop over the oracle:
exact gradient, Barnes-Hut at theta = 0 and at theta = 0.5.

At this size the double-precision dynamics do not amplify rounding: two
oracle runs whose starts differ by one part in 1e15 stay within 1e-14 of each
other after 750 iterations, and so do the oracle's exact and theta = 0 runs.
The GPU's trajectories are therefore held to the oracle's at every iteration
(1e-9).  At theta = 0.5 a criterion decision taken within rounding of its
threshold may go the other way on the two sides, after which the runs part;
the iteration where they part is reported, and the final cost of eq. (3) is
compared within 1e-2 (and with the exact run's)."""
import functools

import numpy as np
import pytest
import torch

import oracle
from paper_2401_13708_amd import hts, synth
from paper_2401_13708_amd.embed import Embedding

pytestmark = pytest.mark.gpu

N, D, ITERS = 1000, 32, 750
TRAJ_TOL = 1e-9


@functools.lru_cache(maxsize=None)
def problem():
    X = synth.gaussian_mixture(N, D, seed=1)
    _, rp, col, val = oracle.build_affinities(X, 30.0, 90)
    Y0 = synth.disk_uniform(N, 1e-4, seed=1 + 10 ** 6, dtype=np.float64)
    return rp, col, val, Y0


@functools.lru_cache(maxsize=None)
def oracle_run(mode):
    """Y after every iteration of the oracle loop; mode "exact" or theta."""
    rp, col, val, Y = problem()
    U, G = np.zeros_like(Y), np.ones_like(Y)
    out = np.empty((ITERS, N, 2))
    for it in range(ITERS):
        ex, mu = (12.0, 0.5) if it < 250 else (1.0, 0.8)
        if mode == "exact":
            g, _ = oracle.gradient_exact(Y, rp, col, val, ex)
        else:
            g, _, _ = oracle.gradient_bh(Y, rp, col, val, oracle.Tree(Y), mode, ex)
        Y, U, G = oracle.step(Y, U, G, g, N / 12000.0, mu)
        out[it] = Y
    return out


def gpu_run(ctx, mode):
    rp, col, val, Y0 = problem()
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    emb = Embedding(ctx, d(rp), d(col), d(val), d(Y0), theta=0.0 if mode == "exact" else mode,
                    exact=mode == "exact")
    out = np.empty((ITERS, N, 2))
    for it in range(ITERS):
        emb.iterate()
        out[it] = emb.Y.cpu().numpy()
    assert ctx.check() == 0
    emb.close()
    return out


def gpu_cost(ctx, Y):
    rp, col, val, _ = problem()
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    kl = torch.zeros(1, dtype=torch.float64, device="cuda")
    hts.gradient_exact(ctx, d(Y), d(rp), d(col), d(val), 1.0, kl=kl)
    torch.cuda.synchronize()
    return float(kl.cpu()[0])


def deviation(a, b):
    return np.abs(a - b).reshape(ITERS, -1).max(axis=1)


def test_exact_schedule_follows_the_oracle(ctx):
    g, o = gpu_run(ctx, "exact"), oracle_run("exact")
    dev = deviation(g, o)
    print("exact: largest |dY| %.2e (iteration %d)" % (dev.max(), int(dev.argmax())))
    assert dev.max() < TRAJ_TOL
    # the embedding left the start (radius 1e-4) for the rim
    assert np.sqrt((g[-1] ** 2).sum(axis=1)).max() > 0.9
    rp, col, val, _ = problem()
    c, co = gpu_cost(ctx, g[-1]), oracle.kl_cost(o[-1], rp, col, val, 1.0)
    assert c == pytest.approx(co, rel=1e-9)


def test_theta0_schedule_follows_exact_and_the_oracle(ctx):
    g = gpu_run(ctx, 0.0)
    assert deviation(g, gpu_run(ctx, "exact")).max() < TRAJ_TOL
    dev = deviation(g, oracle_run(0.0))
    print("theta 0: largest |dY| against the oracle %.2e" % dev.max())
    assert dev.max() < TRAJ_TOL


def test_theta05_schedule_against_the_oracle(ctx):
    g, o = gpu_run(ctx, 0.5), oracle_run(0.5)
    dev = deviation(g, o)
    parted = np.nonzero(dev > TRAJ_TOL)[0]
    first = int(parted[0]) if parted.size else None
    print("theta 0.5: largest |dY| %.2e; runs part at iteration %s" % (dev.max(), first))
    # before they part, the runs agree to rounding
    upto = first if first is not None else ITERS
    assert upto > 0 and dev[:upto].max() < TRAJ_TOL
    rp, col, val, _ = problem()
    c = gpu_cost(ctx, g[-1])
    co = oracle.kl_cost(o[-1], rp, col, val, 1.0)
    ce = oracle.kl_cost(oracle_run("exact")[-1], rp, col, val, 1.0)
    print("final cost: GPU %.6f, oracle %.6f, oracle exact run %.6f" % (c, co, ce))
    assert c == pytest.approx(co, rel=1e-2)
    assert c == pytest.approx(ce, rel=1e-2)
