#!/usr/bin/env python3
"""Barnes-Hut hyperbolic t-SNE iterations per second on one MI355X.

Workload: N = 70000 points, D = 784, values in (0, 1) from a 10-class rank-20
sigmoid factor model (a synthetic stand-in for the 70k x 784 digit data of the
paper's Table 1); perplexity 30, k = 90; polar-quadtree Barnes-Hut at
theta = 0.5; the schedule of Sec. 5 (250 iterations with exaggeration 12 and
momentum 0.5, then momentum 0.8), single-precision forces.  A step is one
whole iteration: tree build + Barnes-Hut gradient + Riemannian step, inputs
resident in HBM.  The affinities P are built once on the GPU before timing.

Prints one JSON line.  The exact O(N^2) gradient is timed beside it at the
same N, and the FP64 CPU oracle on the host cores as the CPU baseline.
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
METRIC_HSNE = "h-SNE BH gradient iters/sec at N=70k θ=0.5 (Euclidean + λ hyperbolic term)"
PROFILE_DIR = os.path.join(ROOT, "profiles")


def _src_hash(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2401_13708_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


KERNEL_SOURCES = {"traverse": ["k_bh.hip", "hts_math.hpp", "hts_impl.hpp"],
                  "items": ["k_bh.hip", "hts_math.hpp", "hts_impl.hpp"],
                  "attract": ["k_grad.hip", "hts_math.hpp", "hts_impl.hpp"],
                  "tree": ["k_tree.hip", "hts_math.hpp", "hts_impl.hpp"]}


def _traffic(kernel):
    """HBM bytes per launch from the committed rocprofv3 PMC summary, if the
    kernel's sources are unchanged since the counters were taken."""
    path = os.path.join(PROFILE_DIR, "traffic_%s.json" % kernel)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_hash") != _src_hash(KERNEL_SOURCES[kernel]):
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(n, seconds, theta, hsne_lambda=None):
    import numpy as np
    import oracle
    from paper_2401_13708_amd import synth
    rp, col, val = synth.random_csr(n, 90, seed=11, dtype=np.float64)
    Y = synth.disk_state(n, "mid", seed=7).astype(np.float64)
    U = np.zeros_like(Y)
    G = np.ones_like(Y)
    cores = oracle.get_threads()
    it = 0
    t0 = time.perf_counter()
    while True:
        t = oracle.Tree(Y)
        if hsne_lambda is None:
            g, z, _ = oracle.gradient_bh(Y, rp, col, val, t, theta, 12.0)
        else:
            g, _, _ = oracle.hsne_gradient_bh(Y, rp, col, val, t, theta, hsne_lambda, 12.0)
        Y, U, G = oracle.step(Y, U, G, g, n / 12000.0, 0.5)
        del t
        it += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    what = "Barnes-Hut gradient" if hsne_lambda is None else \
        "h-SNE Barnes-Hut gradient (Euclidean + %g x hyperbolic)" % hsne_lambda
    return {"value": it / el, "unit": "iters/s", "cores": cores, "kind": "oracle",
            "sample": "%d full iterations (polar quadtree by insertion + %s at "
                      "theta=%.1f + step) of the FP64 oracle at N=%d on a synthetic clustered "
                      "embedding with a k-NN-shaped random P (nnz=%d), %.1f s, OpenMP over "
                      "queries" % (it, what, theta, n, int(rp[-1]), el)}


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
    from paper_2401_13708_amd.batch import JobBatch, autotune_item_points
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
    best, table = autotune_item_points(ctx, jobs, theta=args.theta)
    tune_s = time.perf_counter() - t0
    print("bench: work-item size %d (ms/iteration %s)" % (best, {k: round(v, 3) for k, v in table.items()}),
          file=sys.stderr, flush=True)
    # one job at a time through the single-job calls
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
        "autotune": {"item_points": best, "ms_per_iteration": {str(k): round(v, 4) for k, v in table.items()},
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
        "burst_capacity_jobs_per_s": round(cap, 3),
        "roofline": None, "cpu_baseline": None,
    }
    ctx.close()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=990)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=70000)
    ap.add_argument("--d", type=int, default=784)
    ap.add_argument("--theta", type=float, default=0.5)
    ap.add_argument("--exact-steps", type=int, default=10)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-kernel-events", action="store_true")
    ap.add_argument("--no-stats", action="store_true", help="time without traversal counters")
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
    ap.add_argument("--item-list", type=int, default=None,
                    help="item-list entries per phase-A wave (library default 256)")
    ap.add_argument("--hsne-lambda", type=float, default=None,
                    help="time the h-SNE iteration (Euclidean + lambda x hyperbolic term) instead")
    ap.add_argument("--workload", choices=["single", "jobs", "serve"], default="single",
                    help="single: the N=70k iteration (default); jobs: 64 uneven jobs batched; "
                         "serve: Poisson arrivals through the continuous-batching server")
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
    if args.workload == "jobs":
        return bench_jobs(args)
    if args.workload == "serve":
        return bench_serve(args)

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
        it0 = args.native_start_iteration
        Ys = Y0
        if it0 > 0:
            ctx = hts.Context(0)
            _, rp, col, val = hts.build_affinities(ctx, torch.from_numpy(X).to(dev), 30.0, 90,
                                                   p_dtype=torch.float32, want_knn=False)
            emb = Embedding(ctx, rp, col, val, torch.from_numpy(Y0).to(dev), theta=args.theta)
            emb.run(it0)
            torch.cuda.synchronize()
            Ys = emb.Y.cpu().numpy()
        with open(args.write_native_input, "wb") as f:
            f.write(np.array([n], np.int64).tobytes() + np.array([d, it0], np.int32).tobytes())
            f.write(np.ascontiguousarray(X, np.float32).tobytes())
            f.write(np.ascontiguousarray(Ys, np.float32).tobytes())
        print("bench: wrote %s (iteration %d)" % (args.write_native_input, it0), file=sys.stderr, flush=True)
        return 0

    ctx = hts.Context(0)
    if args.item_list is not None:
        ctx.set_item_list(args.item_list)
    if args.item_points is not None:
        ctx.set_item_points(args.item_points)
    Xd = torch.from_numpy(X).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, rp, col, val = hts.build_affinities(ctx, Xd, 30.0, 90, p_dtype=torch.float32, want_knn=False)
    torch.cuda.synchronize()
    aff_s = time.perf_counter() - t0
    nnz = int(col.numel())
    del Xd
    print("bench: affinities nnz=%d in %.2fs" % (nnz, aff_s), file=sys.stderr, flush=True)

    Y0d = torch.from_numpy(Y0).to(dev)
    hs = args.hsne_lambda
    if hs is not None and hs < 0:
        raise SystemExit("bench.py: --hsne-lambda must be >= 0")
    K = hts.STATS_BLOCK
    nst = 2 * K if hs is None else 4 * K

    def run_pass(events, stats):
        """Warm-up + the timed iterations from the same start; the iteration
        is deterministic, so every pass follows the same trajectory."""
        emb = Embedding(ctx, rp, col, val, Y0d, theta=args.theta, split_rule=args.split_rule,
                        hsne_lambda=hs)
        for _ in range(args.warmup):
            emb.iterate()
        torch.cuda.synchronize()
        if ctx.check() != 0:
            raise RuntimeError("device error word set during warm-up")
        ctx.timing(events)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        e0.record()
        for _ in range(args.steps):
            emb.iterate(stats)
        e1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        kt = ctx.timing_read()
        ctx.timing(False)
        bits = ctx.check()
        if bits:
            raise RuntimeError("device error word 0x%x in the timed region" % bits)
        return emb, e0.elapsed_time(e1), wall, kt

    # pass 1: the headline, nothing but the iterations on the stream
    emb, ms_total, wall, _ = run_pass(False, None)
    ms_step = ms_total / args.steps
    value = 1000.0 / ms_step
    rmax = float(torch.linalg.vector_norm(emb.Y.double(), dim=1).max())
    print("bench: BH %d steps %.3f ms/step (wall %.2fs) rmax=%.6f"
          % (args.steps, ms_step, wall, rmax), file=sys.stderr, flush=True)
    # pass 2: per-kernel durations from HIP events around each launch
    kt = {}
    if not args.no_kernel_events:
        e2, _, _, kt = run_pass(True, None)
        e2.close()
        print("bench: kernel events %s" % {k: round(v[0] / args.steps, 4) for k, v in kt.items() if v[1]},
              file=sys.stderr, flush=True)
    # pass 3: traversal counters (the kernels' counting variants)
    st = [0] * nst
    if not args.no_stats:
        stats = torch.zeros(nst, dtype=torch.int64, device=dev)
        e3, _, _, _ = run_pass(False, stats)
        e3.close()
        st = stats.cpu().numpy().tolist()
        print("bench: traversal counts %s" % st, file=sys.stderr, flush=True)

    # exact O(N^2) gradient + step at the same N, from the same state
    exact_ips = None
    if args.exact_steps > 0 and hs is None:
        ex = Embedding(ctx, rp, col, val, emb.Y, exact=True)
        ex.update.copy_(emb.update)
        ex.gains.copy_(emb.gains)
        ex.it = emb.it
        ex.iterate()
        torch.cuda.synchronize()
        f0, f1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        f0.record()
        for _ in range(args.exact_steps):
            ex.iterate()
        f1.record()
        torch.cuda.synchronize()
        exact_ips = 1000.0 * args.exact_steps / f0.elapsed_time(f1)
        ex.close()
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

    # roofline of the dominant kernel of the timed region
    launches = {k: v[1] for k, v in kt.items()}
    kms = {k: v[0] for k, v in kt.items()}
    names = {"tree": "tree build (7 kernels)", "attract": "k_attract", "traverse": "k_bh_top (with the attractive rows)",
             "items": "k_bh_items", "finalize": "k_bh_gather + k_bh_finalize", "step": "k_step"}
    dom = max(names, key=lambda k: kms.get(k, 0.0))
    roof = None
    if launches.get(dom, 0) > 0:
        avg_s = kms[dom] / launches[dom] / 1000.0
        if dom in ("traverse", "items"):
            def part(c):  # the kernel's share of one traversal's counters
                return c[K:2 * K] if dom == "items" else [a - b for a, b in zip(c[:K], c[K:2 * K])]
            if hs is None:
                share = part(st[:2 * K])
                flops = (share[0] * F_TEST + (share[1] + share[2]) * F_PAIR) / launches[dom]
            else:  # two launches per iteration: the Euclidean walk, then the hyperbolic one
                se, sh = part(st[:2 * K]), part(st[2 * K:4 * K])
                flops = (se[0] * F_TEST_E + (se[1] + se[2]) * F_PAIR_E + sh[0] * F_TEST
                         + (sh[1] + sh[2]) * F_PAIR) / launches[dom]
            ach = flops / avg_s / 1e12
            roof = {"bound": "alu", "achieved": round(ach, 3), "peak": VALU_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": round(ach / VALU_PEAK_TFLOPS, 4),
                    "traffic": _traffic(dom), "kernel": names[dom],
                    "avg_launch_us": round(avg_s * 1e6, 2),
                    "flops_per_launch": round(flops)}
        else:
            if dom == "attract":
                byts = 8.0 * nnz + 8.0 * (n + 1) + 16.0 * n + 8.0 * n
            else:  # tree build, combine, step: bytes they must move
                byts = {"tree": 8.0 * n + 16 * n + 2 * 5 * 12.0 * n + 16 * n + 48.0 * 2 * n,
                        "finalize": 24.0 * n, "step": 56.0 * n}[dom]
            ach = byts / avg_s / 1e9
            roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                    "traffic": _traffic(dom) if dom in KERNEL_SOURCES else None,
                    "kernel": names[dom], "avg_launch_us": round(avg_s * 1e6, 2)}

    cpu = None
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle for ~%.0fs" % args.cpu_seconds, file=sys.stderr, flush=True)
        cpu = cpu_baseline(n, args.cpu_seconds, args.theta, hs)

    def counts(c):
        return {"tests": c[0] // max(1, args.steps),
                "accepted_cells": c[1] // max(1, args.steps),
                "leaf_pairs": c[2] // max(1, args.steps),
                "wave_node_visits": c[3] // max(1, args.steps),
                "wave_visits_with_work": c[4] // max(1, args.steps),
                "points_covered": c[5] // max(1, args.steps),
                "share_of_item_walks": [round(b / a, 3) if a else 0.0 for a, b in zip(c[:K], c[K:2 * K])]}

    workload = ("hyperbolic t-SNE Barnes-Hut iteration" if hs is None else
                "h-SNE Barnes-Hut iteration (Euclidean term + %g x hyperbolic term)" % hs)
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
        "config": {"workload": "%s, N=%d D=%d sigmoid factor "
                               "mixture, perplexity 30, k=90, theta=%.2f, iterations %d-%d of the "
                               "1000-iteration schedule" % (workload, n, d, args.theta, args.warmup,
                                                            args.warmup + args.steps - 1),
                   "n": n, "d": d, "theta": args.theta, "perplexity": 30, "k": 90, "nnz": nnz,
                   "split_rule": "equal lengths, eq. (10)" if args.split_rule == 0
                   else "equal areas, eq. (9)", "hsne_lambda": hs, "item_list": ctx.item_list,
                   "item_points": ctx.item_points},
        "exact_iters_per_s": round(exact_ips, 3) if exact_ips else None,
        "speedup_vs_exact": round(value / exact_ips, 1) if exact_ips else None,
        "kernel_ms_per_step": {k: round(v[0] / max(1, args.steps), 4) for k, v in kt.items() if v[1]},
        "bh_counts_per_step": counts(st[:2 * K]) if hs is None else
        {"euclidean": counts(st[:2 * K]), "hyperbolic": counts(st[2 * K:4 * K])},
        "setup_s": {"generate": round(gen_s, 2), "affinities_gpu": round(aff_s, 3)},
        "roofline": roof,
        "cpu_baseline": cpu,
        "paper_context": {"accelerated_s_per_iter": 4.57, "exact_s_per_iter": 191.0,
                          "dataset": "MNIST 70000x784", "hardware": "CPU, unstated"},
    }
    emb.close()
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
