"""Many hyperbolic t-SNE embeddings advancing together on one GPU.

The jobs are laid side by side: one concatenated Y (with update, gains,
gradient), one CSR of P whose column indices are global, and one tree whose
job layout (`hts_tree_set_jobs`) keeps every job in its own subtree range.
An iteration of all jobs is then the same four library calls as for one job
(schedule, tree, Barnes-Hut gradient, step), whatever the number of jobs, and
each job's result is bit for bit the one it gets alone.

Jobs may be at different iterations of the schedule of Sec. 5 (per-job
iteration counters on the device), which the serving loop uses when it
admits new jobs next to running ones.
"""
from __future__ import annotations

import numpy as np
import torch

from . import hts
from .embed import Schedule


class Job:
    """One embedding job: its P (CSR, local column indices) and start Y on the device."""

    def __init__(self, row_ptr, col_idx, p_val, Y0, name: str = ""):
        self.rp, self.col, self.val, self.Y0 = row_ptr, col_idx, p_val, Y0
        self.n = int(Y0.shape[0])
        self.name = name


class JobBatch:
    """Device-resident state of several jobs in one layout.

    `start_iter[j]` gives the iteration job j is at (0 for a fresh job); state
    (Y, update, gains) may be handed over from a previous layout with
    `carry`, a list of (Y, update, gains) or None per job."""

    def __init__(self, ctx: hts.Context, jobs: list[Job], theta: float = 0.5, max_depth: int = 20,
                 schedule: Schedule | None = None, start_iter=None, carry=None,
                 n_max: int | None = None, tree: hts.Tree | None = None):
        if not jobs:
            raise ValueError("a batch needs at least one job")
        self.ctx, self.jobs, self.theta = ctx, jobs, theta
        self.sched = schedule or Schedule()
        dev = jobs[0].Y0.device
        dt = jobs[0].Y0.dtype
        sizes = [j.n for j in jobs]
        self.sizes = sizes
        self.off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        N = int(self.off[-1])
        self.N = N
        # concatenated CSR with global columns
        rps, cols, vals, nnz0 = [], [], [], 0
        for j, job in enumerate(jobs):
            rps.append(job.rp[:-1] + nnz0)
            cols.append(job.col + int(self.off[j]))
            vals.append(job.val)
            nnz0 += int(job.col.numel())
        rps.append(torch.tensor([nnz0], dtype=torch.int64, device=dev))
        self.rp = torch.cat(rps).contiguous()
        self.col = torch.cat(cols).to(torch.int32).contiguous()
        self.val = torch.cat(vals).contiguous()
        # state
        self.Y = torch.empty((N, 2), dtype=dt, device=dev)
        self.update = torch.zeros_like(self.Y)
        self.gains = torch.ones_like(self.Y)
        for j, job in enumerate(jobs):
            a, b = int(self.off[j]), int(self.off[j + 1])
            c = carry[j] if carry is not None else None
            if c is None:
                self.Y[a:b] = job.Y0
            else:
                self.Y[a:b], self.update[a:b], self.gains[a:b] = c
        self.grad = torch.empty_like(self.Y)
        J = len(jobs)
        self.z = torch.zeros(J, dtype=torch.float64, device=dev)
        it0 = [0] * J if start_iter is None else list(start_iter)
        self.it = torch.tensor(it0, dtype=torch.int32, device=dev)
        self.ex = torch.empty(J, dtype=torch.float64, device=dev)
        self.mu = torch.empty(J, dtype=torch.float64, device=dev)
        s = self.sched
        self.eta = torch.tensor([s.eta if s.eta is not None else n / 12000.0 for n in sizes],
                                dtype=torch.float64, device=dev)
        # a tree of a previous layout is reused when it is large enough
        if tree is not None and tree.n_max >= N and tree.max_depth == max_depth:
            self.tree = tree
        else:
            if tree is not None:
                tree.close()
            self.tree = hts.Tree(ctx, max(N, n_max or 0), max_depth)
        self.tree.set_jobs(sizes)
        self.iters_done = 0
        self.graph = None
        self.graph_gen = -1

    def _launch(self, stats=None):
        s = self.sched
        hts.jobs_schedule(self.ctx, self.it, s.ee_iters, s.exaggeration, s.momentum_early,
                          s.momentum_late, self.ex, self.mu)
        hts.build_polar_tree(self.ctx, self.Y, self.tree)
        hts.gradient_bh_jobs(self.ctx, self.Y, self.rp, self.col, self.val, self.tree, self.ex,
                             self.theta, self.grad, self.z, stats)
        hts.step_jobs(self.ctx, self.tree, self.Y, self.update, self.gains, self.grad, self.eta,
                      self.mu, s.min_gain, s.boundary_eps, s.metric_power)

    def iterate(self, stats=None):
        if self.graph is not None and stats is None and self.ctx.generation() == self.graph_gen:
            self.graph.replay()
        else:
            self._launch(stats)
            if self.graph is not None and stats is None:
                # a workspace the graph points into was reallocated since the
                # capture (another call on the context needed more): record
                # the iteration again against the current workspaces
                self._record()
        self.iters_done += 1

    def _record(self):
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self._launch()
        self.graph, self.graph_gen = g, self.ctx.generation()

    def capture(self):
        """Records one iteration of all jobs (schedule, tree, gradient, step:
        every kernel of it, no memory clears or allocations) as a HIP graph,
        which `iterate` then replays.  The iteration before the capture runs
        eagerly so that the library's workspaces exist; the per-job iteration
        counters live on the device, so every replay is the next iteration.
        A replay is skipped in favour of a new capture when the context's
        workspaces were reallocated after the graph was recorded."""
        self.iterate()
        self._record()
        return self

    def run(self, iters: int):
        for _ in range(iters):
            self.iterate()
        return self

    def job_slice(self, j: int) -> slice:
        return slice(int(self.off[j]), int(self.off[j + 1]))

    def state(self, j: int):
        sl = self.job_slice(j)
        return self.Y[sl], self.update[sl], self.gains[sl]

    def release_tree(self) -> hts.Tree:
        """Hands the tree to the next layout."""
        t, self.tree = self.tree, None
        self.graph = None
        return t

    def close(self):
        self.graph = None
        if self.tree is not None:
            self.tree.close()
            self.tree = None


def pick_setting(times: dict, default, margin: float):
    """The fastest of the timed settings ({setting: ms}), or `default` unless
    the fastest beats it by more than the fraction `margin`."""
    if not times:
        return default
    best = min(times, key=times.get)
    if default in times and times[best] > (1.0 - margin) * times[default]:
        return default
    return best


# launch shapes of the traversal's second kernel: (workgroups, waves per workgroup)
TRAVERSAL_LAUNCHES = ((0, 1), (16384, 4), (65536, 2), (32768, 1), (65536, 1), (131072, 1),
                      (262144, 1))


def autotune_traversal(ctx: hts.Context, jobs: list[Job], candidates=(128, 256, 288, 512, 1024, 2048),
                       launches=TRAVERSAL_LAUNCHES, warm: int = 100, reps: int = 8,
                       theta: float = 0.5, margin: float = 0.02
                       ) -> tuple[tuple[int, tuple[int, int], int], dict]:
    """Picks the Barnes-Hut traversal's tile and launch shapes for a batch of
    jobs by timing: the work-item size S (the walks handed to the second
    kernel hold at most S points), then, at the best S, the second kernel's
    workgroup count (0: the library's automatic count) and waves per
    workgroup, then the launch that computes the attractive term (0:
    automatic, 1: beside phase A, 2: at the end of phase B).

    A scratch copy of the batch is advanced `warm` iterations (the embedding
    spreads out, which changes the traversal), then every candidate times
    `reps` iterations from that same state.  The fastest setting is left on
    ctx and returned with the milliseconds per iteration of every candidate
    ({"S=..": ms, "grid=..x..": ms, "attract=..": ms}); a setting replaces the library's
    default only when it is faster by more than `margin` (a fraction), so
    that timing noise does not pick it.  S changes only the order of
    floating-point sums; the launch shapes change nothing in the result."""
    b = JobBatch(ctx, jobs, theta=theta)
    ctx.set_item_points(hts.DEFAULT_ITEM_POINTS)
    ctx.set_traversal_launch(hts.DEFAULT_ITEMS_GRID, hts.DEFAULT_ITEMS_WAVES)
    ctx.set_attract_launch(hts.DEFAULT_ATTRACT_LAUNCH)
    b.run(warm)
    saved = [t.clone() for t in (b.Y, b.update, b.gains, b.it)]

    def timed():
        for t, v in zip((b.Y, b.update, b.gains, b.it), saved):
            t.copy_(v)
        b.iterate()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            b.iterate()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    times = {}
    by_s = {}
    for S in sorted(set(candidates) | {hts.DEFAULT_ITEM_POINTS}):  # the default is always timed
        ctx.set_item_points(S)
        by_s[S] = times["S=%d" % S] = timed()
    best_s = pick_setting(by_s, hts.DEFAULT_ITEM_POINTS, margin)
    ctx.set_item_points(best_s)
    by_l = {}
    for g, w in launches:
        ctx.set_traversal_launch(g, w)
        by_l[(g, w)] = times["grid=%dx%d" % (g, w)] = timed()
    best_l = pick_setting(by_l, (hts.DEFAULT_ITEMS_GRID, hts.DEFAULT_ITEMS_WAVES), margin)
    ctx.set_traversal_launch(*best_l)
    by_a = {}
    for where in (0, 1, 2):
        ctx.set_attract_launch(where)
        by_a[where] = times["attract=%d" % where] = timed()
    best_a = pick_setting(by_a, hts.DEFAULT_ATTRACT_LAUNCH, margin)
    ctx.set_attract_launch(best_a)
    b.close()
    return (best_s, best_l, best_a), times
