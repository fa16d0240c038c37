"""Continuous-batching server for hyperbolic t-SNE jobs on one GPU.

Requests (a data matrix X and an iteration count) arrive over time.  A
request waits until its device footprint fits the HBM budget next to the
running jobs, then is admitted: its affinities P are built on the GPU by a
worker thread, on a second stream (default priority) with a context of its
own (so its workspaces are its own), while the running jobs keep iterating;
once P is ready the job joins the running job layout (`batch.JobBatch`),
where every iteration advances all admitted jobs in the same launches, each
at its own point of the schedule of Sec. 5.  A job leaves the layout after exactly its iteration
count; its result is copied to the host at that moment.  P, tree and
positions stay on the device for the job's whole life.

The layout is rebuilt only when jobs join or leave (state is carried over,
the tree storage is reused while it is large enough).  Each job's result is
bit for bit the one it gets alone (`embed.Embedding`), whatever else runs
beside it.

`FifoServer` is the comparison: the same requests served one at a time with
the single-job calls.
"""
from __future__ import annotations

import concurrent.futures
import dataclasses
import time

import numpy as np
import torch

from . import hts
from .batch import Job, JobBatch
from .embed import Embedding, Schedule


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float          # seconds after the start of the run
    X: np.ndarray           # n x d data (float32)
    iters: int = 500
    seed: int = 0           # of the start embedding (uniform in a disk of radius 1e-4)


@dataclasses.dataclass
class Result:
    rid: int
    n: int
    arrival: float
    admitted: float
    finished: float
    Y: np.ndarray

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def footprint_bytes(n: int, k: int = 90, max_depth: int = 20,
                    item_list: int = hts.DEFAULT_ITEM_LIST) -> int:
    """Device bytes a job of n points holds while it runs: P (at most 2nk
    entries of column + value, and row pointers), the state and gradient
    arrays, its share of the tree storage (60 bytes per node slot, n (depth
    + 1) slots, and 142 bytes per point of keys, sort buffers, prefix sums and
    point records), the per-point buffers of the gradient call, its share of
    the traversal workspace (four phase-A waves per 64 queries, each with
    item_list item records of 40 bytes and 64-lane single-precision partials,
    plus per-slot partials of every query), and 8 MiB for allocation
    granularity."""
    p = 2 * n * k * 8 + (n + 1) * 8
    state = n * 2 * 4 * 4
    tree = n * (max_depth + 1) * 60 + n * 142
    grad = n * 40
    waves = 4 * (n // 64 + 1)
    trav = waves * (item_list * (64 * 2 * 4 + 40) + 16) + n * (4 * 2 * 4 + 2 * 4)
    return p + state + tree + grad + trav + (8 << 20)


def _start_embedding(n: int, seed: int, dev) -> torch.Tensor:
    from . import synth
    return torch.from_numpy(synth.disk_uniform(n, 1e-4, seed=seed)).to(dev)


class Server:
    """Admission by footprint, one running job layout, continuous batching."""

    def __init__(self, ctx: hts.Context, hbm_budget: int, theta: float = 0.5,
                 perplexity: float = 30.0, k: int = 90, schedule: Schedule | None = None,
                 max_depth: int = 20):
        self.ctx, self.budget, self.theta = ctx, int(hbm_budget), theta
        self.perplexity, self.k = perplexity, k
        self.sched = schedule or Schedule()
        self.max_depth = max_depth
        self.dev = torch.device("cuda", ctx.device)
        self.max_active = 0
        self.relayouts = 0
        self.setup_overlap_s = 0.0   # setup time spent while jobs were iterating

    def _prepare(self, req: Request, setup_ctx: hts.Context, stream: torch.cuda.Stream):
        """Worker thread: P of a request on the setup stream and context; returns
        the device tensors and an event recorded after them."""
        with torch.cuda.device(self.dev), torch.cuda.stream(stream):
            X = torch.from_numpy(np.ascontiguousarray(req.X, dtype=np.float32)).to(self.dev)
            n = X.shape[0]
            _, rp, col, val = hts.build_affinities(setup_ctx, X, self.perplexity, min(self.k, n - 1),
                                                   p_dtype=torch.float32, want_knn=False)
            ev = torch.cuda.Event()
            ev.record(stream)
        return rp, col, val, ev

    def _join(self, req: Request, prepared) -> dict:
        """Main thread: the prepared P becomes a job of the layout on the
        current stream (which waits for the setup stream's work)."""
        rp, col, val, ev = prepared
        main = torch.cuda.current_stream(self.dev)
        main.wait_event(ev)
        for t in (rp, col, val):
            t.record_stream(main)   # allocated on the setup stream, used on this one
        job = Job(rp, col, val, _start_embedding(rp.numel() - 1, req.seed, self.dev),
                  name=str(req.rid))
        return {"req": req, "job": job, "done": 0, "admitted": None, "state": None}

    def _layout(self, active, old: JobBatch | None) -> JobBatch | None:
        tree = old.release_tree() if old is not None else None
        if not active:
            if tree is not None:
                tree.close()
            return None
        carry = [a["state"] for a in active]
        b = JobBatch(self.ctx, [a["job"] for a in active], theta=self.theta,
                     max_depth=self.max_depth, schedule=self.sched,
                     start_iter=[a["done"] for a in active], carry=carry, tree=tree)
        self.relayouts += 1
        return b

    def run(self, requests: list[Request]) -> list[Result]:
        setup_ctx = hts.Context(self.ctx.device)
        stream = torch.cuda.Stream(self.dev)   # default priority
        pool = concurrent.futures.ThreadPoolExecutor(max_workers=1)
        try:
            return self._run(requests, setup_ctx, stream, pool)
        finally:
            pool.shutdown(wait=True)
            stream.synchronize()
            setup_ctx.close()

    def _run(self, requests, setup_ctx, stream, pool) -> list[Result]:
        pending = sorted(requests, key=lambda r: r.arrival)
        waiting, preparing, active, results = [], [], [], []
        batch = None
        used = 0
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0
        while pending or waiting or preparing or active:
            t = now()
            while pending and pending[0].arrival <= t:
                waiting.append(pending.pop(0))
            changed = False
            # admission in arrival order while the footprint fits (a job
            # larger than the whole budget runs alone): its setup starts on
            # the worker, its footprint counts from now
            while waiting:
                fp = footprint_bytes(waiting[0].X.shape[0], self.k, self.max_depth, self.ctx.item_list)
                if (active or preparing) and used + fp > self.budget:
                    break
                req = waiting.pop(0)
                used += fp
                preparing.append((req, fp, pool.submit(self._prepare, req, setup_ctx, stream), now()))
            # jobs whose P is ready join the layout, in admission order
            while preparing and preparing[0][2].done():
                req, fp, fut, ts = preparing.pop(0)
                a = self._join(req, fut.result())
                if active:
                    self.setup_overlap_s += now() - ts
                a["admitted"] = now()
                a["fp"] = fp
                active.append(a)
                changed = True
            if not active:
                if preparing:
                    concurrent.futures.wait([preparing[0][2]], timeout=0.01)
                elif pending:
                    time.sleep(max(0.0, min(pending[0].arrival - now(), 0.01)))
                continue
            if changed:
                if batch is not None:
                    for j, a in enumerate(active[:len(batch.jobs)]):
                        a["state"] = batch.state(j)
                batch = self._layout(active, batch)
                for a in active:
                    a["state"] = None
                self.max_active = max(self.max_active, len(active))
            # iterate until the next job completes, a new request arrives or
            # a setup finishes
            left = min(a["req"].iters - a["done"] for a in active)
            steps = 0
            while steps < left:
                batch.iterate()
                steps += 1
                if steps % 8 == 0 and ((pending and pending[0].arrival <= now()) or
                                       (preparing and preparing[0][2].done())):
                    break
            for a in active:
                a["done"] += steps
            finished = [i for i, a in enumerate(active) if a["done"] >= a["req"].iters]
            if finished:
                # this stream only: a setup running beside it is not waited for
                torch.cuda.current_stream(self.dev).synchronize()
                tf = now()
                keep = []
                for i, a in enumerate(active):
                    if i in finished:
                        Y = batch.state(i)[0].cpu().numpy()
                        results.append(Result(a["req"].rid, a["job"].n, a["req"].arrival,
                                              a["admitted"], tf, Y))
                        used -= a["fp"]
                    else:
                        a["state"] = batch.state(i)
                        keep.append(a)
                active = keep
                batch = self._layout(active, batch)
                for a in active:
                    a["state"] = None
        if batch is not None:
            batch.close()
        if self.ctx.check() != 0:
            raise RuntimeError("device error word set")
        return results


class FifoServer:
    """The same requests, one job at a time with the single-job calls."""

    def __init__(self, ctx: hts.Context, theta: float = 0.5, perplexity: float = 30.0, k: int = 90,
                 schedule: Schedule | None = None, max_depth: int = 20):
        self.ctx, self.theta, self.perplexity, self.k = ctx, theta, perplexity, k
        self.sched = schedule or Schedule()
        self.max_depth = max_depth
        self.dev = torch.device("cuda", ctx.device)

    def run(self, requests: list[Request]) -> list[Result]:
        results = []
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0
        for req in sorted(requests, key=lambda r: r.arrival):
            while now() < req.arrival:
                time.sleep(min(req.arrival - now(), 0.01))
            ta = now()
            X = torch.from_numpy(np.ascontiguousarray(req.X, dtype=np.float32)).to(self.dev)
            n = X.shape[0]
            _, rp, col, val = hts.build_affinities(self.ctx, X, self.perplexity, min(self.k, n - 1),
                                                   p_dtype=torch.float32, want_knn=False)
            e = Embedding(self.ctx, rp, col, val, _start_embedding(n, req.seed, self.dev),
                          theta=self.theta, max_depth=self.max_depth, schedule=self.sched)
            e.run(req.iters)
            Y = e.Y.cpu().numpy()
            e.close()
            results.append(Result(req.rid, n, req.arrival, ta, now(), Y))
        if self.ctx.check() != 0:
            raise RuntimeError("device error word set")
        return results


def summarize(results: list[Result], skip: int = 0) -> dict:
    """jobs/s over the measured window and p50/p99 completion latency,
    leaving out the first `skip` requests (by id) as warm-up."""
    rs = sorted(results, key=lambda r: r.rid)[skip:]
    if not rs:
        return {}
    lat = np.array([r.latency for r in rs])
    t_first = min(r.arrival for r in rs)
    t_last = max(r.finished for r in rs)
    return {"jobs": len(rs), "jobs_per_s": len(rs) / max(t_last - t_first, 1e-9),
            "p50_latency_s": float(np.percentile(lat, 50)),
            "p99_latency_s": float(np.percentile(lat, 99)),
            "mean_latency_s": float(lat.mean())}
