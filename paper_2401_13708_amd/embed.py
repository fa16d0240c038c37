"""Optimisation driver for one hyperbolic t-SNE job on the GPU.

Runs the schedule of Sec. 5: early exaggeration 12 with momentum 0.5 for the
first 250 iterations, then no exaggeration with momentum 0.8; learning rate
eta = n / (12 * 1000); gains as in the Euclidean case.  Every iteration is
(polar quadtree + Barnes-Hut gradient, or the exact gradient) followed by the
Riemannian step, all through libhts on one stream with no host
synchronisation.  The optional stopping rule (a point within 1e-4 of the rim,
Sec. 5) needs a host read and is off unless asked for.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import torch

from . import hts


@dataclasses.dataclass
class Schedule:
    ee_iters: int = 250
    exaggeration: float = 12.0
    momentum_early: float = 0.5
    momentum_late: float = 0.8
    eta: float | None = None           # default n / 12000
    min_gain: float = 0.01
    boundary_eps: float = 1e-5
    metric_power: int = 2

    def at(self, it: int, n: int):
        early = it < self.ee_iters
        ex = self.exaggeration if early else 1.0
        mu = self.momentum_early if early else self.momentum_late
        eta = self.eta if self.eta is not None else n / 12000.0
        return ex, mu, eta


class Embedding:
    """Device-resident state (Y, update, gains, P, tree) of one job."""

    def __init__(self, ctx: hts.Context, row_ptr, col_idx, p_val, Y0, theta: float = 0.5,
                 exact: bool = False, max_depth: int = 20, schedule: Schedule | None = None,
                 split_rule: int = 0, hsne_lambda: float | None = None, fused: bool = True):
        self.ctx = ctx
        # the Barnes-Hut iteration through hts_iteration_bh (False: the three
        # separate calls; the same results bit for bit)
        self.fused = fused
        self.rp, self.col, self.val = row_ptr, col_idx, p_val
        self.Y = Y0.clone()
        self.update = torch.zeros_like(self.Y)
        self.gains = torch.ones_like(self.Y)
        self.grad = torch.empty_like(self.Y)
        # h-SNE (Sec. 4-C): Euclidean term plus hsne_lambda times the hyperbolic
        # one (Barnes-Hut only); z then holds Z^E and Z^H
        self.hsne_lambda = hsne_lambda
        if hsne_lambda is not None and exact:
            raise ValueError("the h-SNE gradient is Barnes-Hut only")
        self.z = torch.zeros(1 if hsne_lambda is None else 2, dtype=torch.float64,
                             device=self.Y.device)
        self.n = self.Y.shape[0]
        self.theta = theta
        self.exact = exact
        self.sched = schedule or Schedule()
        self.tree = None if exact else hts.Tree(ctx, self.n, max_depth)
        if self.tree is not None and split_rule:
            self.tree.set_split(split_rule)
        self.it = 0

    def iterate(self, stats=None):
        ex, mu, eta = self.sched.at(self.it, self.n)
        s = self.sched
        if self.fused and not self.exact and self.hsne_lambda is None and stats is None:
            # tree, gradient and step in one call; bit for bit the three
            # calls below
            hts.iteration_bh(self.ctx, self.Y, self.update, self.gains, self.rp, self.col, self.val,
                             self.tree, self.theta, ex, eta, mu, self.grad, self.z, s.min_gain,
                             s.boundary_eps, s.metric_power)
            self.it += 1
            return
        if self.exact:
            hts.gradient_exact(self.ctx, self.Y, self.rp, self.col, self.val, ex, self.grad, self.z)
        else:
            hts.build_polar_tree(self.ctx, self.Y, self.tree)
            if self.hsne_lambda is None:
                hts.gradient_bh(self.ctx, self.Y, self.rp, self.col, self.val, self.tree,
                                self.theta, ex, self.grad, self.z, stats)
            else:
                hts.gradient_hsne(self.ctx, self.Y, self.rp, self.col, self.val, self.tree,
                                  self.hsne_lambda, self.theta, ex, self.grad, self.z, stats)
        s = self.sched
        hts.step(self.ctx, self.Y, self.update, self.gains, self.grad, eta, mu, s.min_gain,
                 s.boundary_eps, s.metric_power)
        self.it += 1

    def run(self, iters: int, stop_at_rim: bool = False, check_every: int = 10):
        for _ in range(iters):
            self.iterate()
            if stop_at_rim and self.it % check_every == 0:
                r = torch.linalg.vector_norm(self.Y.double(), dim=1).max().item()
                if r > 1.0 - 1e-4:
                    break
        return self

    def snapshot(self):
        """Device copies of the optimiser state (Y, update, gains) and the
        iteration counter, to restart the schedule from later."""
        return (self.Y.clone(), self.update.clone(), self.gains.clone(), self.it)

    def restore(self, snap):
        Y, U, G, it = snap
        self.Y.copy_(Y)
        self.update.copy_(U)
        self.gains.copy_(G)
        self.it = int(it)

    def state_dict(self) -> dict:
        return {"Y": self.Y.cpu().numpy(), "update": self.update.cpu().numpy(),
                "gains": self.gains.cpu().numpy(), "it": self.it}

    def load_state_dict(self, st: dict):
        dev = self.Y.device
        self.Y.copy_(torch.from_numpy(np.asarray(st["Y"])).to(dev))
        self.update.copy_(torch.from_numpy(np.asarray(st["update"])).to(dev))
        self.gains.copy_(torch.from_numpy(np.asarray(st["gains"])).to(dev))
        self.it = int(st["it"])

    def close(self):
        if self.tree is not None:
            self.tree.close()
            self.tree = None
