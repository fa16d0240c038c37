#!/usr/bin/env python3
"""Barnes-Hut hyperbolic t-SNE iterations per second on one MI355X.

Workload: N = 70000 points, D = 784, values in (0, 1) from a 10-class rank-20
sigmoid factor model (a synthetic stand-in for the 70k x 784 digit data of the
paper's Table 1); perplexity 30, k = 90; polar-quadtree Barnes-Hut at
theta = 0.5; the schedule of Sec. 5 (250 iterations with exaggeration 12 and
momentum 0.5, then momentum 0.8), single-precision forces.  A step is one
whole iteration: tree build + Barnes-Hut gradient + Riemannian step, inputs
resident in HBM.  The affinities P are built once on the GPU before timing.

The cost of an iteration changes along the schedule (the embedding spreads
towards the rim and the traversal deepens), so the timed steps are taken from
fixed points of it: the schedule is run once with the counting kernels (which
give the same results) to reach the embeddings at iterations 0, 250, 500 and
999, and the K timed steps are split evenly over windows that start there.
Per-kernel events, traversal counters and the dominant kernel's roofline come
from the same windows; the FP32 error is stated per window against the GPU's
FP64 Barnes-Hut and exact gradients, and the CPU baseline runs the FP64 oracle
on the same snapshot bytes and P.

Prints one JSON line.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "BH gradient iters/sec at N=70k θ=0.5 vs exact; jobs/sec + p50/p99 job latency"
HBM_PEAK_GBS = 8000.0
# Non-packed FP32 / FP64 vector rate: 256 CU x 64 lanes x 2.4 GHz x 2 (FMA)
VALU_PEAK_TFLOPS = 78.6
# Algorithmic flops of the Barnes-Hut traversal: a criterion
# test computes t = 2|y-m|^2 ia ib and compares (9 flops); an interaction
# (accepted cell or leaf point) adds sinh d, d, w, the force factor, the
# direction vector and the three accumulations (26 flops).
F_TEST, F_PAIR = 9, 26
# The Euclidean traversal of the h-SNE term: a test forms |y-c|^2 and
# compares (6 flops); an interaction adds w = 1/(1+|y-c|^2), N w^2, the
# direction vector and the three accumulations (12 flops).
F_TEST_E, F_PAIR_E = 6, 12
# The attractive term, which the launch of the traversal's second kernel also
# computes: per non-zero of P the distance argument (a test without its
# compare) and the pair term without the Z accumulation.
F_ATTR, F_ATTR_E = (F_TEST - 1) + (F_PAIR - 2), (F_TEST_E - 1) + (F_PAIR_E - 2)
METRIC_HSNE = "h-SNE BH gradient iters/sec at N=70k θ=0.5 (Euclidean + λ hyperbolic term)"
PROFILE_DIR = os.path.join(ROOT, "profiles")
# iterations of the 1000-iteration schedule where the timed windows start
SNAPSHOTS = (0, 250, 500, 999)


def _src_hash(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2401_13708_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


KERNEL_SOURCES = {"traverse": ["k_bh.hip", "hts_math.hpp", "hts_impl.hpp"],
                  "items": ["k_bh.hip", "hts_math.hpp", "hts_impl.hpp"],
                  "attract": ["k_grad.hip", "hts_math.hpp", "hts_impl.hpp"],
                  "tree": ["k_tree.hip", "k_sort.hip", "hts_math.hpp", "hts_impl.hpp"]}


def _traffic(kernel, windows, setting):
    """HBM bytes per launch from the committed rocprofv3 PMC summary, if it
    was taken on these windows of the same workload setting (N, theta, the
    attractive rows' launch, the traversal's tuning) and the kernel's sources
    are unchanged since."""
    path = os.path.join(PROFILE_DIR, "traffic_%s.json" % kernel)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_hash") != _src_hash(KERNEL_SOURCES[kernel]):
        return None
    if rec.get("windows") != windows:
        return None
    if rec.get("setting") != setting:
        return None
    return rec.get("bytes_per_launch")


def window_steps(k, nw):
    """k steps split over nw windows, the first k mod nw windows one longer."""
    return [k // nw + (1 if w < k % nw else 0) for w in range(nw)]


def rel_l2(a, b):
    import numpy as np
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def rel_row(a, b):
    """largest per-point error over the largest per-point norm of b"""
    import numpy as np
    a = np.asarray(a, np.float64).reshape(-1, 2)
    b = np.asarray(b, np.float64).reshape(-1, 2)
    return float(np.linalg.norm(a - b, axis=1).max() / max(np.linalg.norm(b, axis=1).max(), 1e-300))


def paper_grad_error(g_hat, g):
    """The gradient error of Sec. 5-B: the gradient vectors read as points of
    the disk, sqrt(sum d(g_hat_i, g_i)^2) / sqrt(sum d(0, g_i)^2) with d of
    eq. (8); None when a vector does not lie inside the unit disk."""
    import numpy as np
    a = np.asarray(g_hat, np.float64).reshape(-1, 2)
    b = np.asarray(g, np.float64).reshape(-1, 2)
    na, nb = np.sum(a * a, axis=1), np.sum(b * b, axis=1)
    if na.max() >= 1.0 or nb.max() >= 1.0:
        return None
    t = 2.0 * np.sum((a - b) ** 2, axis=1) / ((1.0 - na) * (1.0 - nb))
    d = np.log1p(t + np.sqrt(t * (t + 2.0)))
    d0 = 2.0 * np.arctanh(np.sqrt(nb))
    return float(np.sqrt(np.sum(d * d)) / max(np.sqrt(np.sum(d0 * d0)), 1e-300))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(snaps, rp, col, val, theta, gpu_grads, hsne_lambda=None, bh_rows=2048,
                 exact_rows=(64, 512)):
    """The FP64 oracle on the host cores, on the snapshot embeddings the GPU
    windows start from (their FP32 bytes, promoted) and the GPU-built P.

    All cores: one whole iteration per snapshot (insertion tree, Barnes-Hut
    gradient, step).  One thread: the tree and the step, plus the Barnes-Hut
    traversal of `bh_rows` sampled queries scaled to all n.  The exact
    gradient's time per iteration is scaled from `exact_rows` sampled rows
    (one thread, all cores).  Also the GPU gradient's error against the
    oracle's Barnes-Hut at the same theta, per snapshot."""
    import numpy as np
    import oracle
    from paper_2401_13708_amd import synth
    n = rp.size - 1
    threads = oracle.get_threads()
    out = {"per_snapshot": []}
    t_all, t_one, t_ex1, t_exa = [], [], [], []
    for k, (it, Y, U, G) in enumerate(snaps):
        ex = 12.0 if it < 250 else 1.0
        mu = 0.5 if it < 250 else 0.8
        # all cores, one whole iteration
        oracle.set_threads(threads)
        t0 = time.perf_counter()
        tree = oracle.Tree(Y)
        if hsne_lambda is None:
            g, z, _ = oracle.gradient_bh(Y, rp, col, val, tree, theta, ex)
        else:
            g, _, z = oracle.hsne_gradient_bh(Y, rp, col, val, tree, theta, hsne_lambda, ex)
        oracle.step(Y, U, G, g, n / 12000.0, mu)
        t_all.append(time.perf_counter() - t0)
        rec = {"iteration": it, "all_cores_s": round(t_all[-1], 3)}
        if gpu_grads is not None:
            rec["gpu_fp32_vs_oracle_rel_l2"] = rel_l2(gpu_grads[k], g)
            rec["gpu_fp32_vs_oracle_rel_row"] = rel_row(gpu_grads[k], g)
        # one thread: tree + sampled traversals scaled to n + step (the
        # oracle samples rows of the hyperbolic gradient only, so for h-SNE
        # there is no one-thread figure)
        oracle.set_threads(1)
        tree1 = None
        if hsne_lambda is None:
            rows = synth.subsample(n, bh_rows, seed=300 + k)
            t0 = time.perf_counter()
            tree1 = oracle.Tree(Y)
            t_tree = time.perf_counter() - t0
            t0 = time.perf_counter()
            oracle.gradient_bh_rows(Y, rp, col, val, tree1, theta, rows, z, ex)
            t_rows = time.perf_counter() - t0
            t0 = time.perf_counter()
            oracle.step(Y, U, G, g, n / 12000.0, mu)
            t_step = time.perf_counter() - t0
            t_one.append(t_tree + t_rows * n / rows.size + t_step)
            rec["one_thread_s_est"] = round(t_one[-1], 3)
        # exact gradient rows, one thread and all cores
        for nt, m, acc in ((1, exact_rows[0], t_ex1), (threads, exact_rows[1], t_exa)):
            oracle.set_threads(nt)
            er = synth.subsample(n, m, seed=400 + k)
            t0 = time.perf_counter()
            oracle.gradient_exact_rows(Y, rp, col, val, er, z, ex)
            acc.append((time.perf_counter() - t0) * n / m)
        del tree, tree1
        out["per_snapshot"].append(rec)
    oracle.set_threads(threads)
    nsnap = len(snaps)
    out.update({
        "value": nsnap / sum(t_all), "unit": "iters/s", "cores": threads, "kind": "oracle",
        "cpu_model": cpu_model(),
        "one_thread_iters_per_s": nsnap / sum(t_one) if t_one else None,
        "exact_s_per_iter_one_thread": sum(t_ex1) / nsnap,
        "exact_s_per_iter_all_cores": sum(t_exa) / nsnap,
        "sample": "FP64 oracle on the GPU windows' snapshot embeddings (iterations %s of the "
                  "schedule, FP32 bytes promoted) and the GPU-built P (nnz=%d): one whole "
                  "iteration per snapshot on %d threads (insertion tree + %s at theta=%.1f + "
                  "step; the value); one thread (hyperbolic iteration only): tree + step + %d "
                  "sampled query traversals scaled to N; exact hyperbolic gradient from %d / %d "
                  "sampled rows (1 thread / %d) scaled to N" % (",".join(str(s[0]) for s in snaps), int(rp[-1]), threads,
                            "Barnes-Hut gradient" if hsne_lambda is None else
                            "h-SNE Barnes-Hut gradient", theta, bh_rows, exact_rows[0],
                            exact_rows[1], threads),
    })
    return out


def _job_set(ctx, dev, count, seed, n_lo, n_hi, dims, iters_note=""):
    """Jobs of uneven size: N log-uniform in [n_lo, n_hi]; data per job from
    the generator of its workload; P built on the GPU (not timed)."""
    import numpy as np
    import torch
    from paper_2401_13708_amd import hts, synth
    from paper_2401_13708_amd.batch import Job
    g = np.random.default_rng(seed)
    sizes = np.round(np.exp(g.uniform(np.log(n_lo), np.log(n_hi), size=count))).astype(int)
    clusters = g.integers(5, 21, size=count)
    dsel = g.choice(dims, size=count)
    jobs = []
    for j, n in enumerate(sizes):
        X = synth.gaussian_mixture(int(n), int(dsel[j]), n_clusters=int(clusters[j]),
                                   seed=seed + j).astype(np.float32)
        _, rp, col, val = hts.build_affinities(ctx, torch.from_numpy(X).to(dev), 30.0, 90,
                                               p_dtype=torch.float32, want_knn=False)
        Y0 = torch.from_numpy(synth.disk_uniform(int(n), 1e-4, seed=seed + j + 10 ** 6)).to(dev)
        jobs.append(Job(rp, col, val, Y0, name="job%d" % j))
    return jobs


def bench_jobs(args):
    """64 jobs of uneven size: all advanced together in one job layout, against
    the same jobs run one after another with the single-job calls."""
    import numpy as np
    import torch
    from paper_2401_13708_amd import hts
    from paper_2401_13708_amd.batch import JobBatch, autotune_traversal
    from paper_2401_13708_amd.embed import Embedding
    dev = torch.device("cuda", 0)
    ctx = hts.Context(0)
    t0 = time.perf_counter()
    jobs = _job_set(ctx, dev, args.jobs, 400, 500, 50000, [50])
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    total_n = sum(j.n for j in jobs)
    print("bench: %d jobs, %d points in all, set up in %.1fs" % (len(jobs), total_n, setup_s),
          file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    (best, best_launch, best_attract), table = autotune_traversal(ctx, jobs, theta=args.theta)
    tune_s = time.perf_counter() - t0
    print("bench: work-item size %d (ms/iteration %s)" % (best, {k: round(v, 3) for k, v in table.items()}),
          file=sys.stderr, flush=True)
    # one job at a time through the single-job calls, with the tuned work-item
    # size (the same sums as the batched runs) and the library's default
    # launch shapes (the tuned ones are for the whole layout; they change
    # nothing in the result)
    ctx.set_traversal_launch(hts.DEFAULT_ITEMS_GRID, hts.DEFAULT_ITEMS_WAVES)
    ctx.set_attract_launch(hts.DEFAULT_ATTRACT_LAUNCH)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    finals = []
    for job in jobs:
        e = Embedding(ctx, job.rp, job.col, job.val, job.Y0, theta=args.theta)
        e.run(args.job_iters)
        finals.append(e.Y)
        e.close()
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    ctx.set_traversal_launch(*best_launch)
    ctx.set_attract_launch(best_attract)
    print("bench: sequential %.2fs" % t_seq, file=sys.stderr, flush=True)
    # all jobs in one layout
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b = JobBatch(ctx, jobs, theta=args.theta)
    b.run(args.job_iters)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    if ctx.check() != 0:
        raise RuntimeError("device error word set")
    diff = max(float((b.state(j)[0] - finals[j]).abs().max()) for j in range(len(jobs)))
    print("bench: batched %.2fs, max |dY| vs sequential %g" % (t_batch, diff), file=sys.stderr,
          flush=True)
    b.close()
    # all jobs in one layout, each iteration one replay of a captured HIP graph
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bg = JobBatch(ctx, jobs, theta=args.theta).capture()
    bg.run(args.job_iters - 1)
    torch.cuda.synchronize()
    t_graph = time.perf_counter() - t0
    diff_g = max(float((bg.state(j)[0] - finals[j]).abs().max()) for j in range(len(jobs)))
    print("bench: batched with graph replay %.2fs, max |dY| vs sequential %g" % (t_graph, diff_g),
          file=sys.stderr, flush=True)
    bg.close()
    value = len(jobs) / t_graph
    out = {
        "metric": "jobs/sec: %d uneven hyperbolic t-SNE jobs in one job layout (one HIP graph "
                  "replay per iteration) vs one at a time" % len(jobs),
        "value": round(value, 3), "unit": "jobs/s", "n_gpus": 1, "steps": args.job_iters,
        "warmup": 0, "ms_per_step": round(1000.0 * t_graph / args.job_iters, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "%d jobs, N log-uniform in [500, 50000] (%d points in all), D=50 "
                               "Gaussian mixtures of 5-20 clusters, perplexity 30, k=90, theta=%.2f, "
                               "%d iterations each (schedule of Sec. 5)"
                               % (len(jobs), total_n, args.theta, args.job_iters),
                   "jobs": len(jobs), "sizes": [j.n for j in jobs]},
        "sequential_jobs_per_s": round(len(jobs) / t_seq, 3),
        "batched_eager_jobs_per_s": round(len(jobs) / t_batch, 3),
        "speedup_vs_sequential": round(t_seq / t_graph, 2),
        "max_abs_diff_vs_sequential": max(diff, diff_g),
        "autotune": {"item_points": best, "traversal_launch": list(best_launch),
                     "attract_launch": best_attract,
                     "ms_per_iteration": {str(k): round(v, 4) for k, v in table.items()},
                     "tune_s": round(tune_s, 2)},
        "setup_s": round(setup_s, 2),
        "roofline": None, "cpu_baseline": None,
    }
    ctx.close()
    print(json.dumps(out), flush=True)


def bench_serve(args):
    """Poisson arrivals of jobs of uneven size served by the continuous-
    batching server, against the same arrivals served one job at a time."""
    import numpy as np
    import torch
    from paper_2401_13708_amd import hts, synth
    from paper_2401_13708_amd.serve import FifoServer, Request, Server, summarize
    dev = torch.device("cuda", 0)
    ctx = hts.Context(0)
    count = args.serve_jobs
    g = np.random.default_rng(5)
    sizes = np.round(np.exp(g.uniform(np.log(1000), np.log(100000), size=count))).astype(int)
    dims = g.choice([32, 50, 100], size=count)
    t0 = time.perf_counter()
    reqs = []
    for j in range(count):
        n = int(sizes[j])
        depth = int(min(10, max(3, np.ceil(np.log2(n / 100.0)))))
        X = synth.branching_walk(n, int(dims[j]), depth=depth, seed=500 + j).astype(np.float32)
        reqs.append(Request(j, 0.0, X, iters=args.serve_iters, seed=500 + j + 10 ** 6))
    gen_s = time.perf_counter() - t0
    print("bench: %d requests generated in %.1fs (%d points in all)" % (count, gen_s, int(sizes.sum())),
          file=sys.stderr, flush=True)
    budget = int(args.hbm_budget_gb * (1 << 30))
    # capacity: a burst of the first requests, all there at once
    burst = [Request(r.rid, 0.0, r.X, r.iters, r.seed) for r in reqs[:args.calib_jobs]]
    srv = Server(ctx, budget, theta=args.theta)
    cal = summarize(srv.run(burst))
    cap = cal["jobs_per_s"]
    rate = args.arrival_rate if args.arrival_rate > 0 else 0.8 * cap
    arr = np.cumsum(np.random.default_rng(5 + 1).exponential(1.0 / rate, size=count))
    arr -= arr[0]
    for r, a in zip(reqs, arr):
        r.arrival = float(a)
    print("bench: burst capacity %.2f jobs/s; arrival rate %.2f jobs/s" % (cap, rate),
          file=sys.stderr, flush=True)
    srv = Server(ctx, budget, theta=args.theta)
    got = srv.run(reqs)
    sb = summarize(got, skip=16)
    print("bench: served %s" % sb, file=sys.stderr, flush=True)
    fifo = summarize(FifoServer(ctx, theta=args.theta).run(reqs), skip=16)
    print("bench: one at a time %s" % fifo, file=sys.stderr, flush=True)
    out = {
        "metric": "served jobs/sec and p50/p99 completion latency, Poisson arrivals, continuous "
                  "batching vs one job at a time",
        "value": round(sb["jobs_per_s"], 3), "unit": "jobs/s", "n_gpus": 1,
        "steps": args.serve_iters, "warmup": 16, "ms_per_step": None,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "%d requests, Poisson arrivals at %.2f jobs/s (0.8 x burst capacity "
                               "unless given), N log-uniform in [1000, 100000], D in {32, 50, 100}, "
                               "branching-walk data of depth ceil(log2(N/100)) in [3, 10], "
                               "perplexity 30, k=90, theta=%.2f, %d iterations each, first 16 "
                               "excluded, HBM budget %.1f GiB"
                               % (count, rate, args.theta, args.serve_iters, args.hbm_budget_gb),
                   "requests": count, "arrival_rate": rate},
        "p50_latency_s": round(sb["p50_latency_s"], 3),
        "p99_latency_s": round(sb["p99_latency_s"], 3),
        "one_at_a_time": {k: round(v, 3) for k, v in fifo.items()},
        "speedup_jobs_per_s": round(sb["jobs_per_s"] / fifo["jobs_per_s"], 2),
        "max_active_jobs": srv.max_active, "relayouts": srv.relayouts,
        "setup_overlapped_s": round(srv.setup_overlap_s, 3),
        "burst_capacity_jobs_per_s": round(cap, 3),
        "roofline": None, "cpu_baseline": None,
    }
    ctx.close()
    print(json.dumps(out), flush=True)


def bench_single(args):
    """The N = 70k iteration, timed in windows that start at fixed points of
    the schedule (see the module docstring)."""
    import numpy as np
    import torch
    from paper_2401_13708_amd import hts, synth
    from paper_2401_13708_amd.embed import Embedding

    dev = torch.device("cuda", 0)
    n, d = args.n, args.d
    t0 = time.perf_counter()
    X = synth.sigmoid_factor_mixture(n, d, seed=2)
    Y0 = synth.disk_uniform(n, 1e-4, seed=2 + 10 ** 6)
    gen_s = time.perf_counter() - t0
    print("bench: generated X %dx%d in %.1fs" % (n, d, gen_s), file=sys.stderr, flush=True)
    if args.write_native_input:
        # X, then the optimiser state (Y, update, gains) at iteration it0 of
        # the schedule: the state a window of the timed pass starts from
        it0 = args.native_start_iteration
        Ys, Us, Gs = Y0, np.zeros_like(Y0), np.ones_like(Y0)
        if it0 > 0:
            ctx = hts.Context(0)
            _, rp, col, val = hts.build_affinities(ctx, torch.from_numpy(X).to(dev), 30.0, 90,
                                                   p_dtype=torch.float32, want_knn=False)
            emb = Embedding(ctx, rp, col, val, torch.from_numpy(Y0).to(dev), theta=args.theta)
            emb.run(it0)
            torch.cuda.synchronize()
            Ys, Us, Gs = (a.cpu().numpy() for a in (emb.Y, emb.update, emb.gains))
        with open(args.write_native_input, "wb") as f:
            f.write(np.array([n], np.int64).tobytes() + np.array([d, it0], np.int32).tobytes())
            f.write(np.ascontiguousarray(X, np.float32).tobytes())
            for a in (Ys, Us, Gs):
                f.write(np.ascontiguousarray(a, np.float32).tobytes())
        print("bench: wrote %s (iteration %d)" % (args.write_native_input, it0), file=sys.stderr,
              flush=True)
        return 0

    ctx = hts.Context(0)
    if args.item_list is not None:
        ctx.set_item_list(args.item_list)
    if args.item_points is not None:
        ctx.set_item_points(args.item_points)
    if args.items_grid is not None or args.items_waves is not None:
        ctx.set_traversal_launch(args.items_grid or hts.DEFAULT_ITEMS_GRID,
                                 args.items_waves or hts.DEFAULT_ITEMS_WAVES)
    if args.attract_launch is not None:
        ctx.set_attract_launch(args.attract_launch)
    Xd = torch.from_numpy(X).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, rp, col, val = hts.build_affinities(ctx, Xd, 30.0, 90, p_dtype=torch.float32, want_knn=False)
    torch.cuda.synchronize()
    aff_s = time.perf_counter() - t0
    nnz = int(col.numel())
    del Xd
    print("bench: affinities nnz=%d in %.2fs" % (nnz, aff_s), file=sys.stderr, flush=True)

    hs = args.hsne_lambda
    if hs is not None and hs < 0:
        raise SystemExit("bench.py: --hsne-lambda must be >= 0")
    K = hts.STATS_BLOCK
    nst = 2 * K if hs is None else 4 * K
    snapshots = [int(v) for v in args.snapshots.split(",")]
    if sorted(set(snapshots)) != snapshots or snapshots[0] < 0:
        raise SystemExit("bench.py: --snapshots must be increasing iterations >= 0")
    steps_w = window_steps(args.steps, len(snapshots))
    windows = [[s, k] for s, k in zip(snapshots, steps_w)]

    Y0d = torch.from_numpy(Y0).to(dev)
    emb = Embedding(ctx, rp, col, val, Y0d, theta=args.theta, split_rule=args.split_rule,
                    hsne_lambda=hs, fused=not args.separate_calls)
    ee = emb.sched.ee_iters

    # the schedule up to the last snapshot with the counting kernels (same
    # results as the timed ones), keeping the state at every snapshot
    st_sched = torch.zeros(nst, dtype=torch.int64, device=dev)
    snaps = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(snapshots[-1]):
        if it in snapshots:
            snaps[it] = emb.snapshot()
        emb.iterate(st_sched)
    snaps[snapshots[-1]] = emb.snapshot()
    torch.cuda.synchronize()
    traj_s = time.perf_counter() - t0
    if ctx.check() != 0:
        raise RuntimeError("device error word set while reaching the snapshots")
    rmax = {s: float(torch.linalg.vector_norm(snaps[s][0].double(), dim=1).max()) for s in snapshots}
    print("bench: schedule to iteration %d in %.2fs (counting kernels); max radius %s"
          % (snapshots[-1], traj_s, {s: round(r, 6) for s, r in rmax.items()}),
          file=sys.stderr, flush=True)
    # warm-up (counting kernels again, so that the plain kernels run only in
    # the timed windows and the per-kernel pass over the same windows)
    scratch = torch.zeros(nst, dtype=torch.int64, device=dev)
    emb.restore(snaps[snapshots[0]])
    for _ in range(args.warmup):
        emb.iterate(scratch)
    torch.cuda.synchronize()
    if ctx.check() != 0:
        raise RuntimeError("device error word set during warm-up")

    def run_windows(events=False, stats=False):
        res = []
        for s, k in windows:
            st = torch.zeros(nst, dtype=torch.int64, device=dev) if stats else None
            if k == 0:
                res.append((0.0, {}, st))
                continue
            emb.restore(snaps[s])
            torch.cuda.synchronize()
            ctx.timing(events)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(k):
                emb.iterate(st)
            e1.record()
            torch.cuda.synchronize()
            kt = ctx.timing_read() if events else {}
            ctx.timing(False)
            bits = ctx.check()
            if bits:
                raise RuntimeError("device error word 0x%x in the window from %d" % (bits, s))
            res.append((e0.elapsed_time(e1), kt, st))
        return res

    # pass 1: the headline, nothing but the iterations on the stream
    w0 = time.perf_counter()
    r1 = run_windows()
    wall = time.perf_counter() - w0
    ms_total = sum(r[0] for r in r1)
    ms_step = ms_total / args.steps
    value = 1000.0 / ms_step
    print("bench: %d steps in windows %s: %.4f ms/step (%s)" % (
        args.steps, windows, ms_step, [round(r[0] / max(1, k), 4) for r, (_, k) in zip(r1, windows)]),
        file=sys.stderr, flush=True)
    # pass 2: per-kernel durations from HIP events around each launch
    kt_tot, kt_win = {}, []
    if not args.no_kernel_events:
        for r, (_, k) in zip(run_windows(events=True), windows):
            kt_win.append({c: round(v[0] / k, 4) for c, v in r[1].items() if v[1]} if k else {})
            for c, v in r[1].items():
                a = kt_tot.setdefault(c, [0.0, 0])
                a[0] += v[0]
                a[1] += v[1]
        print("bench: kernel ms/step %s" % {c: round(v[0] / args.steps, 4) for c, v in kt_tot.items() if v[1]},
              file=sys.stderr, flush=True)
    # pass 3: traversal counters (the counting kernels) over the same windows
    st_win, st_tot = [], [0] * nst
    if not args.no_stats:
        for r in run_windows(stats=True):
            c = r[2].cpu().numpy().tolist()
            st_win.append(c)
            st_tot = [a + b for a, b in zip(st_tot, c)]

    def counts(c, steps):
        steps = max(1, steps)
        return {"tests": c[0] // steps, "accepted_cells": c[1] // steps, "leaf_pairs": c[2] // steps,
                "wave_node_visits": c[3] // steps, "wave_visits_with_work": c[4] // steps,
                "points_covered": c[5] // steps,
                "share_of_item_walks": [round(b / a, 3) if a else 0.0 for a, b in zip(c[:K], c[K:2 * K])]}

    def counts_of(c, steps):
        return counts(c[:2 * K], steps) if hs is None else \
            {"euclidean": counts(c[:2 * K], steps), "hyperbolic": counts(c[2 * K:4 * K], steps)}

    # FP32 error per window: the timed single-precision gradient against the
    # GPU's double-precision instantiation (same theta) and, for the
    # hyperbolic gradient, against the double exact gradient; the cost of
    # eq. (3) from the exact call and the Barnes-Hut Z's effect on it
    errors, gpu_grads = [], []
    if not args.no_errors:
        val64 = val.double()
        tree64 = hts.Tree(ctx, n)
        if args.split_rule:
            tree64.set_split(args.split_rule)
        st32 = torch.zeros(nst, dtype=torch.int64, device=dev)
        st64 = torch.zeros(nst, dtype=torch.int64, device=dev)
        for s in snapshots:
            ex = 12.0 if s < ee else 1.0
            emb.restore(snaps[s])
            Y32 = emb.Y
            Y64 = Y32.double()
            hts.build_polar_tree(ctx, Y32, emb.tree)
            hts.build_polar_tree(ctx, Y64, tree64)
            if hs is None:
                g32, z32 = hts.gradient_bh(ctx, Y32, rp, col, val, emb.tree, args.theta, ex,
                                           stats=st32)
                g64, z64 = hts.gradient_bh(ctx, Y64, rp, col, val64, tree64, args.theta, ex,
                                           stats=st64)
            else:
                g32, z32 = hts.gradient_hsne(ctx, Y32, rp, col, val, emb.tree, hs, args.theta, ex,
                                             stats=st32)
                g64, z64 = hts.gradient_hsne(ctx, Y64, rp, col, val64, tree64, hs, args.theta, ex,
                                             stats=st64)
            e = {"start": s, "bh_fp32_vs_bh_fp64_rel_l2": rel_l2(g32.cpu(), g64.cpu()),
                 "bh_fp32_vs_bh_fp64_rel_row": rel_row(g32.cpu(), g64.cpu()),
                 "z_fp32_vs_fp64_rel": [abs(float(a) - float(b)) / float(b)
                                        for a, b in zip(z32.cpu(), z64.cpu())]}
            if hs is None:
                kl = torch.zeros(1, dtype=torch.float64, device=dev)
                gx64, zx64 = hts.gradient_exact(ctx, Y64, rp, col, val64, ex, kl=kl)
                gx32, zx32 = hts.gradient_exact(ctx, Y32, rp, col, val, ex)
                zb, zx, c = float(z64[0]), float(zx64[0]), float(kl[0])
                # the same errors for the Riemannian gradient the step applies
                # (each row scaled by (1 - |y|^2)^2 / 4), and in the form of
                # Sec. 5-B (distances of eq. (8) between gradient vectors)
                yh = Y64.cpu().numpy()
                sc = ((1.0 - np.sum(yh * yh, axis=1)) ** 2 / 4.0)[:, None]
                rb, rx = sc * g32.cpu().numpy(), sc * gx64.cpu().numpy()
                e.update({
                    "bh_fp32_vs_exact_riemannian_rel_l2": rel_l2(rb, rx),
                    "bh_fp32_vs_exact_paper_form": paper_grad_error(rb, rx),
                    "bh_fp32_vs_exact_paper_form_euclidean_variation":
                        paper_grad_error(g32.cpu().numpy(), gx64.cpu().numpy())})
                e.update({
                    "bh_fp32_vs_exact_fp64_rel_l2": rel_l2(g32.cpu(), gx64.cpu()),
                    "bh_fp32_vs_exact_fp64_rel_row": rel_row(g32.cpu(), gx64.cpu()),
                    "bh_fp64_vs_exact_fp64_rel_l2": rel_l2(g64.cpu(), gx64.cpu()),
                    "exact_fp32_vs_exact_fp64_rel_l2": rel_l2(gx32.cpu(), gx64.cpu()),
                    "z_bh_fp64_vs_exact_rel": abs(zb - zx) / zx,
                    "cost_exact": c,
                    "cost_with_bh_z_rel_err": abs(np.log(zb) - np.log(zx)) / abs(c)})
            torch.cuda.synchronize()
            if ctx.check() != 0:
                raise RuntimeError("device error word set in the error pass")
            errors.append(e)
            gpu_grads.append(g32.cpu().numpy().astype(np.float64))
        tree64.close()
        print("bench: errors %s" % errors, file=sys.stderr, flush=True)

    # exact O(N^2) gradient + step at the same N, from the same snapshots
    exact_ips = None
    if args.exact_steps > 0 and hs is None:
        exw = window_steps(args.exact_steps, len(snapshots))
        exm = Embedding(ctx, rp, col, val, Y0d, exact=True)
        exm.restore(snaps[snapshots[0]])
        exm.iterate()
        ms_ex = 0.0
        for s, k in zip(snapshots, exw):
            if k == 0:
                continue
            exm.restore(snaps[s])
            torch.cuda.synchronize()
            f0, f1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            f0.record()
            for _ in range(k):
                exm.iterate()
            f1.record()
            torch.cuda.synchronize()
            ms_ex += f0.elapsed_time(f1)
        exact_ips = 1000.0 * args.exact_steps / ms_ex
        exm.close()
        print("bench: exact %.3f ms/step" % (1000.0 / exact_ips), file=sys.stderr, flush=True)

    if args.copy_calibration_mib > 0:
        # one elementwise kernel that reads and writes exactly this many bytes
        # (the scale for the HBM byte counters of a profiler run)
        m = args.copy_calibration_mib * (1 << 20) // 4
        a = torch.ones(m, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        torch.neg(a, out=b)
        torch.cuda.synchronize()
        del a, b

    # roofline of the dominant kernel of the timed windows
    rows_in_items = hts.attract_in_items(ctx.attract_launch, n)
    # what a committed traffic record must have been taken with
    setting = {"n": n, "theta": args.theta, "hsne_lambda": hs, "split_rule": args.split_rule,
               "item_points": ctx.item_points, "item_list": ctx.item_list,
               "traversal_launch": list(ctx.traversal_launch), "attract_rows_in_items": rows_in_items}
    names = {"tree": "tree build", "attract": "k_attract",
             "traverse": "k_bh_top" if rows_in_items else "k_bh_top (with the attractive rows)",
             "items": "k_bh_items (with the attractive rows)" if rows_in_items else "k_bh_items",
             "finalize": "k_bh_gather + k_bh_finalize", "step": "k_step"}
    kms = {c: v[0] for c, v in kt_tot.items()}
    launches = {c: v[1] for c, v in kt_tot.items()}
    dom = max(names, key=lambda c: kms.get(c, 0.0))
    roof = None
    if launches.get(dom, 0) > 0:
        avg_s = kms[dom] / launches[dom] / 1000.0
        if dom in ("traverse", "items") and not args.no_stats:
            def part(c):  # the kernel's share of one traversal's counters
                return c[K:2 * K] if dom == "items" else [a - b for a, b in zip(c[:K], c[K:2 * K])]
            # the counting pass covers the same windows as the timed launches,
            # one traversal (two for h-SNE) per timed iteration
            iters = sum(k for _, k in windows)
            if hs is None:
                sh = part(st_tot[:2 * K])
                flops = sh[0] * F_TEST + (sh[1] + sh[2]) * F_PAIR
                if (dom == "items") == rows_in_items:
                    flops += iters * nnz * F_ATTR
            else:  # two launches per iteration: the Euclidean walk, then the hyperbolic one
                se, sh = part(st_tot[:2 * K]), part(st_tot[2 * K:4 * K])
                flops = (se[0] * F_TEST_E + (se[1] + se[2]) * F_PAIR_E + sh[0] * F_TEST
                         + (sh[1] + sh[2]) * F_PAIR)
                if (dom == "items") == rows_in_items:
                    flops += iters * nnz * (F_ATTR_E + F_ATTR)
            flops /= launches[dom]
            ach = flops / avg_s / 1e12
            roof = {"bound": "alu", "achieved": round(ach, 3), "peak": VALU_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": round(ach / VALU_PEAK_TFLOPS, 4),
                    "traffic": _traffic(dom, windows, setting), "kernel": names[dom],
                    "avg_launch_us": round(avg_s * 1e6, 2), "flops_per_launch": round(flops),
                    "launches": launches[dom], "windows": windows}
        elif dom not in ("traverse", "items"):
            byts = {"attract": 8.0 * nnz + 8.0 * (n + 1) + 16.0 * n + 8.0 * n,
                    "tree": 8.0 * n + 16 * n + 2 * 5 * 12.0 * n + 16 * n + 48.0 * 2 * n,
                    "finalize": 24.0 * n, "step": 56.0 * n}[dom]
            ach = byts / avg_s / 1e9
            roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                    "traffic": _traffic(dom, windows, setting) if dom in KERNEL_SOURCES else None,
                    "kernel": names[dom], "avg_launch_us": round(avg_s * 1e6, 2),
                    "launches": launches[dom], "windows": windows}

    cpu = None
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle on the snapshots", file=sys.stderr, flush=True)
        rph = rp.cpu().numpy()
        colh = col.cpu().numpy()
        valh = val.cpu().numpy().astype(np.float64)
        host = [(s, snaps[s][0].cpu().numpy().astype(np.float64),
                 snaps[s][1].cpu().numpy().astype(np.float64),
                 snaps[s][2].cpu().numpy().astype(np.float64)) for s in snapshots]
        cpu = cpu_baseline(host, rph, colh, valh, args.theta, gpu_grads or None, hs)

    workload = ("hyperbolic t-SNE Barnes-Hut iteration" if hs is None else
                "h-SNE Barnes-Hut iteration (Euclidean term + %g x hyperbolic term)" % hs)
    win_out = []
    for w, ((s, k), r) in enumerate(zip(windows, r1)):
        rec = {"start": s, "steps": k, "ms_per_step": round(r[0] / k, 4) if k else None,
               "max_radius": round(rmax[s], 7)}
        if kt_win:
            rec["kernel_ms_per_step"] = kt_win[w]
        if st_win:
            rec["counts_per_step"] = counts_of(st_win[w], k)
        if errors:
            rec["errors"] = errors[w]
        win_out.append(rec)
    worst = {}
    for e in errors:
        for key, v in e.items():
            if key.endswith(("rel_l2", "rel_row", "_rel", "rel_err", "_form")) and \
                    isinstance(v, float):
                worst[key] = max(worst.get(key, 0.0), v)
    out = {
        "metric": METRIC if hs is None else METRIC_HSNE,
        "value": round(value, 2),
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "%s, N=%d D=%d sigmoid factor mixture, perplexity 30, k=90, "
                               "theta=%.2f, %d steps in windows starting at iterations %s of the "
                               "1000-iteration schedule" % (workload, n, d, args.theta, args.steps,
                                                            ",".join(map(str, snapshots))),
                   "n": n, "d": d, "theta": args.theta, "perplexity": 30, "k": 90, "nnz": nnz,
                   "split_rule": "equal lengths, eq. (10)" if args.split_rule == 0
                   else "equal areas, eq. (9)", "hsne_lambda": hs, "item_list": ctx.item_list,
                   "item_points": ctx.item_points, "traversal_launch": list(ctx.traversal_launch),
                   "attract_launch": ctx.attract_launch,
                   "windows": windows},
        "windows": win_out,
        "exact_iters_per_s": round(exact_ips, 3) if exact_ips else None,
        "speedup_vs_exact": round(value / exact_ips, 1) if exact_ips else None,
        "kernel_ms_per_step": {c: round(v[0] / args.steps, 4) for c, v in kt_tot.items() if v[1]},
        "bh_counts_per_step": counts_of(st_tot, args.steps) if st_win else None,
        "schedule_counts_per_iteration": counts_of(st_sched.cpu().numpy().tolist(),
                                                   snapshots[-1]),
        "fp32_errors_worst_window": worst or None,
        "setup_s": {"generate": round(gen_s, 2), "affinities_gpu": round(aff_s, 3),
                    "schedule_to_last_snapshot": round(traj_s, 3), "timed_wall": round(wall, 3)},
        "roofline": roof,
        "cpu_baseline": cpu,
        "paper_context": {"accelerated_s_per_iter": 4.57, "exact_s_per_iter": 191.0,
                          "dataset": "MNIST 70000x784", "hardware": "CPU, unstated"},
    }
    emb.close()
    ctx.close()
    print(json.dumps(out), flush=True)


def bench_hier(args):
    """The hierarchical workload (N = 200000, D = 50, binary branching random
    walk of depth 10): the schedule is run once at theta = 0.5 to the
    snapshot iterations; then, for each theta of the sweep, the timed steps in
    windows from those snapshots and, at every snapshot, the gradient's error
    against the double-precision exact gradient on a 5000-point subsample
    (Sec. 5, effect of theta)."""
    import numpy as np
    import torch
    from paper_2401_13708_amd import hts, synth
    from paper_2401_13708_amd.embed import Embedding
    dev = torch.device("cuda", 0)
    n, d = args.hier_n, 50
    t0 = time.perf_counter()
    X = synth.branching_walk(n, d, depth=10, seed=3)
    Y0 = synth.disk_uniform(n, 1e-4, seed=3 + 10 ** 6)
    gen_s = time.perf_counter() - t0
    ctx = hts.Context(0)
    t0 = time.perf_counter()
    _, rp, col, val = hts.build_affinities(ctx, torch.from_numpy(X).to(dev), 30.0, 90,
                                           p_dtype=torch.float32, want_knn=False)
    torch.cuda.synchronize()
    aff_s = time.perf_counter() - t0
    print("bench: hierarchical N=%d, nnz=%d, affinities %.2fs" % (n, col.numel(), aff_s),
          file=sys.stderr, flush=True)
    snapshots = [int(v) for v in args.snapshots.split(",")]
    steps_w = window_steps(args.steps, len(snapshots))
    emb = Embedding(ctx, rp, col, val, torch.from_numpy(Y0).to(dev), theta=0.5)
    snaps = {}
    for it in range(snapshots[-1]):
        if it in snapshots:
            snaps[it] = emb.snapshot()
        emb.iterate()
    snaps[snapshots[-1]] = emb.snapshot()
    torch.cuda.synchronize()
    rows = torch.from_numpy(synth.subsample(n, 5000, seed=23)).to(dev)
    val64 = val.double()
    ref = {}
    for s in snapshots:
        ex = 12.0 if s < emb.sched.ee_iters else 1.0
        Y64 = snaps[s][0].double()
        g, _ = hts.gradient_exact(ctx, Y64, rp, col, val64, ex)
        ref[s] = (g[rows].cpu().numpy(), Y64[rows].cpu().numpy())
    torch.cuda.synchronize()
    sweep = []
    for theta in (0.3, 0.5, 0.8):
        e = Embedding(ctx, rp, col, val, torch.from_numpy(Y0).to(dev), theta=theta)
        for _ in range(args.warmup):
            e.iterate()
        ms = 0.0
        errs = []
        for s, k in zip(snapshots, steps_w):
            e.restore(snaps[s])
            ex = 12.0 if s < e.sched.ee_iters else 1.0
            hts.build_polar_tree(ctx, e.Y, e.tree)
            g, _ = hts.gradient_bh(ctx, e.Y, rp, col, val, e.tree, theta, ex)
            gr, yr = ref[s]
            gb = g[rows].cpu().numpy().astype(np.float64)
            sc = ((1.0 - np.sum(yr * yr, axis=1)) ** 2 / 4.0)[:, None]
            errs.append({"start": s, "rel_l2": rel_l2(gb, gr),
                         "riemannian_rel_l2": rel_l2(sc * gb, sc * gr),
                         "paper_form": paper_grad_error(sc * gb, sc * gr)})
            if k == 0:
                continue
            e.restore(snaps[s])
            torch.cuda.synchronize()
            f0, f1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            f0.record()
            for _ in range(k):
                e.iterate()
            f1.record()
            torch.cuda.synchronize()
            ms += f0.elapsed_time(f1)
        if ctx.check() != 0:
            raise RuntimeError("device error word set at theta %g" % theta)
        e.close()
        sweep.append({"theta": theta, "iters_per_s": round(1000.0 * args.steps / ms, 2),
                      "ms_per_step": round(ms / args.steps, 4), "errors_vs_exact": errs})
        print("bench: theta %.1f %.4f ms/step %s" % (theta, ms / args.steps, errs),
              file=sys.stderr, flush=True)
    # the exact gradient + step at the same size, a few steps from the last snapshot
    exm = Embedding(ctx, rp, col, val, torch.from_numpy(Y0).to(dev), exact=True)
    exm.restore(snaps[snapshots[-1]])
    exm.iterate()
    torch.cuda.synchronize()
    f0, f1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    f0.record()
    for _ in range(3):
        exm.iterate()
    f1.record()
    torch.cuda.synchronize()
    exact_ips = 3000.0 / f0.elapsed_time(f1)
    exm.close()
    mid = [r for r in sweep if r["theta"] == 0.5][0]
    out = {
        "metric": "BH gradient iters/sec at N=200k (hierarchical data), theta swept over "
                  "{0.3, 0.5, 0.8}, with the error against the exact gradient",
        "value": mid["iters_per_s"], "unit": "iters/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": mid["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "hyperbolic t-SNE Barnes-Hut iteration, N=%d D=50 binary branching "
                               "random walk of depth 10 (leaves sigma 0.05), perplexity 30, k=90, "
                               "steps in windows from iterations %s of the schedule (reached at "
                               "theta 0.5); value at theta 0.5" % (n, ",".join(map(str, snapshots))),
                   "n": n, "d": d, "nnz": int(col.numel()),
                   "windows": [[s, k] for s, k in zip(snapshots, steps_w)],
                   "error_rows": 5000},
        "theta_sweep": sweep,
        "exact_iters_per_s": round(exact_ips, 3),
        "speedup_vs_exact_at_theta_0_5": round(mid["iters_per_s"] / exact_ips, 1),
        "setup_s": {"generate": round(gen_s, 2), "affinities_gpu": round(aff_s, 3)},
        "roofline": None, "cpu_baseline": None,
    }
    emb.close()
    ctx.close()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200,
                    help="timed steps, split evenly over the windows")
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--snapshots", default=",".join(map(str, SNAPSHOTS)),
                    help="iterations of the schedule where the timed windows start")
    ap.add_argument("--n", type=int, default=70000)
    ap.add_argument("--d", type=int, default=784)
    ap.add_argument("--theta", type=float, default=0.5)
    ap.add_argument("--exact-steps", type=int, default=12)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernel-events", action="store_true")
    ap.add_argument("--no-stats", action="store_true", help="time without traversal counters")
    ap.add_argument("--no-errors", action="store_true", help="skip the per-window error pass")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run a plain device copy of this size (for PMC calibration)")
    ap.add_argument("--split-rule", type=int, choices=[0, 1], default=0,
                    help="radial split: 0 equal lengths (eq. (10)), 1 equal areas (eq. (9))")
    ap.add_argument("--write-native-input", metavar="PATH", default=None,
                    help="write X and Y0 of the single workload for paper_2401_13708_amd/native/hts_run "
                         "and exit (no GPU use unless --native-start-iteration is given)")
    ap.add_argument("--native-start-iteration", type=int, default=0,
                    help="with --write-native-input: run this many iterations on the GPU first and "
                         "write the embedding reached (the native run continues the schedule there)")
    ap.add_argument("--item-points", type=int, default=None,
                    help="Barnes-Hut work-item size S (library default 256)")
    ap.add_argument("--separate-calls", action="store_true",
                    help="iterate with the three separate calls instead of hts_iteration_bh")
    ap.add_argument("--items-grid", type=int, default=None,
                    help="workgroups of the traversal's second kernel (library default 0: 32 one-wave "
                         "workgroups per first-kernel wave)")
    ap.add_argument("--items-waves", type=int, default=None,
                    help="waves per workgroup of that kernel: 1, 2 or 4 (library default 1)")
    ap.add_argument("--attract-launch", type=int, choices=[0, 1, 2], default=None,
                    help="launch of the attractive term: 0 automatic (library default), 1 beside "
                         "phase A, 2 at the end of phase B")
    ap.add_argument("--item-list", type=int, default=None,
                    help="item-list entries per phase-A wave (library default 256)")
    ap.add_argument("--hsne-lambda", type=float, default=None,
                    help="time the h-SNE iteration (Euclidean + lambda x hyperbolic term) instead")
    ap.add_argument("--workload", choices=["single", "hier", "jobs", "serve"], default="single",
                    help="single: the N=70k iteration (default); hier: N=200k hierarchical data, "
                         "theta swept; jobs: 64 uneven jobs batched; serve: Poisson arrivals "
                         "through the continuous-batching server")
    ap.add_argument("--hier-n", type=int, default=200000)
    ap.add_argument("--jobs", type=int, default=64)
    ap.add_argument("--job-iters", type=int, default=1000)
    ap.add_argument("--serve-jobs", type=int, default=256)
    ap.add_argument("--serve-iters", type=int, default=500)
    ap.add_argument("--calib-jobs", type=int, default=24)
    ap.add_argument("--arrival-rate", type=float, default=0.0)
    ap.add_argument("--hbm-budget-gb", type=float, default=32.0)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the library runs on one GPU; --gpus %d (WORLD_SIZE %s) is not "
              "supported: sharding by query rows across GPUs is not implemented"
              % (args.gpus, os.environ.get("WORLD_SIZE", "1")), file=sys.stderr)
        sys.exit(2)
    if args.steps < 1:
        raise SystemExit("bench.py: --steps must be >= 1")
    if args.workload == "hier":
        return bench_hier(args)
    if args.workload == "jobs":
        return bench_jobs(args)
    if args.workload == "serve":
        return bench_serve(args)
    return bench_single(args)


if __name__ == "__main__":
    main()
