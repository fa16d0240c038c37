"""Seeded synthetic inputs for hyperbolic t-SNE workloads.

This module is shared by the CPU oracle tests and the GPU path, so it holds no
arithmetic of the method itself: only random draws shaped like the workloads of
the paper's evaluation (Sec. 5, Table 1) and of the benchmark configurations.
Every generator takes an explicit seed and uses numpy's PCG64 generator.

Workload recipes (each stands in for a dataset of Table 1, none of whose items
is reproduced here):

* ``gaussian_mixture``   -- N=1000, D=32: 10 isotropic unit-variance Gaussians
  with means ~ N(0, 4 I), point i in cluster i mod 10.
* ``sigmoid_factor_mixture`` -- N=70000, D=784 in (0, 1): 10 classes, each a
  rank-20 Gaussian factor model passed through a sigmoid (an image-like
  stand-in for the 70k x 784 digit data of Table 1).
* ``branching_walk``     -- N=200000, D=50: binary branching random walk of
  depth 10 (hierarchical data), leaves sampled with sigma = 0.05.
* ``disk_uniform``       -- the embedding initialisation: uniform in a disk
  of radius 1e-4 around the origin of the Poincare disk.
* ``disk_state``         -- synthetic embedding states (clusters in the disk
  at increasing radii, down to 1e-4 from the boundary) that stand in for the
  states an optimisation passes through; used as shared parity inputs.
* ``random_csr``         -- a sparse row structure with the row lengths of a
  symmetrised k-NN graph, for timing-only inputs.
* ``near_split_rays``    -- adversarial tree inputs: single-precision points a
  few units in the last place either side of the rays that halve the angular
  range of the polar quadtree's cells (angles 2 pi (2j + 1) / 2^(l + 1) at
  level l), where an angle computed by a math library could fall on either
  side.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "rng",
    "gaussian_mixture",
    "sigmoid_factor_mixture",
    "branching_walk",
    "disk_uniform",
    "disk_state",
    "random_csr",
    "subsample",
    "near_split_rays",
]


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def gaussian_mixture(n: int = 1000, d: int = 32, n_clusters: int = 10,
                     mean_std: float = 2.0, seed: int = 1,
                     dtype=np.float64) -> np.ndarray:
    """Isotropic Gaussian mixture: mu_c ~ N(0, mean_std^2 I), x = mu_c(i) + N(0, I)."""
    g = rng(seed)
    mu = g.normal(0.0, mean_std, size=(n_clusters, d))
    c = np.arange(n) % n_clusters
    x = mu[c] + g.normal(0.0, 1.0, size=(n, d))
    return np.ascontiguousarray(x.astype(dtype))


def sigmoid_factor_mixture(n: int = 70000, d: int = 784, n_classes: int = 10,
                           rank: int = 20, load_std: float = 1.5,
                           seed: int = 2) -> np.ndarray:
    """x = sigmoid(mu_c + W_c z), mu_c ~ N(-1, 1)^d, W_c entries ~ N(0, load_std^2/rank),
    z ~ N(0, I_rank); class of point i is i mod n_classes.  Returns float32 in (0, 1)."""
    g = rng(seed)
    mu = g.normal(-1.0, 1.0, size=(n_classes, d))
    w = g.normal(0.0, load_std / np.sqrt(rank), size=(n_classes, d, rank))
    z = g.normal(0.0, 1.0, size=(n, rank))
    out = np.empty((n, d), dtype=np.float32)
    cls = np.arange(n) % n_classes
    for c in range(n_classes):
        rows = np.nonzero(cls == c)[0]
        a = mu[c][None, :] + z[rows] @ w[c].T
        out[rows] = (1.0 / (1.0 + np.exp(-a))).astype(np.float32)
    return out


def branching_walk(n: int = 200000, d: int = 50, depth: int = 10,
                   leaf_sigma: float = 0.05, seed: int = 3) -> np.ndarray:
    """Binary branching random walk: a child at depth l has mean parent + N(0, 0.5^l I);
    2^depth leaves; point i is drawn around leaf i mod 2^depth with std leaf_sigma."""
    g = rng(seed)
    means = np.zeros((1, d))
    for lvl in range(1, depth + 1):
        step = g.normal(0.0, np.sqrt(0.5 ** lvl), size=(means.shape[0] * 2, d))
        means = np.repeat(means, 2, axis=0) + step
    leaf = np.arange(n) % means.shape[0]
    x = means[leaf] + g.normal(0.0, leaf_sigma, size=(n, d))
    return np.ascontiguousarray(x.astype(np.float32))


def disk_uniform(n: int, radius: float = 1e-4, seed: int = 1000001,
                 dtype=np.float32) -> np.ndarray:
    """Uniform in a Euclidean disk of the given radius: r = radius sqrt(U), phi = 2 pi U'."""
    g = rng(seed)
    r = radius * np.sqrt(g.random(n))
    phi = 2.0 * np.pi * g.random(n)
    y = np.stack([r * np.cos(phi), r * np.sin(phi)], axis=1)
    return np.ascontiguousarray(y.astype(dtype))


_STAGES = {
    # stage: (centre radius range, relative cluster spread)
    "init": None,
    "early": ((0.0, 0.05), 0.08),
    "mid": ((0.2, 0.8), 0.05),
    "late": ((0.85, 0.999), 0.02),
    "edge": ((0.99, 0.9999), 0.01),
}


def disk_state(n: int, stage: str = "mid", n_clusters: int = 10,
               seed: int = 7, dtype=np.float32) -> np.ndarray:
    """Clustered points inside the unit disk.

    Cluster centres are drawn at radii in the stage's range and uniform angles;
    the spread of a cluster shrinks with (1 - |c|^2) so that clusters near the
    rim look as small in the disk as the conformal factor makes them.  Points
    are redrawn until they lie at least 1e-4 inside the unit circle."""
    if stage == "init":
        return disk_uniform(n, 1e-4, seed, dtype)
    (rlo, rhi), spread = _STAGES[stage]
    g = rng(seed)
    cr = g.uniform(rlo, rhi, size=n_clusters)
    cphi = g.uniform(0.0, 2.0 * np.pi, size=n_clusters)
    cen = np.stack([cr * np.cos(cphi), cr * np.sin(cphi)], axis=1)
    lab = np.arange(n) % n_clusters
    out = np.empty((n, 2))
    todo = np.arange(n)
    while todo.size:
        c = cen[lab[todo]]
        s = spread * (1.0 - np.sum(c * c, axis=1, keepdims=True)) + 1e-6
        cand = c + s * g.normal(size=(todo.size, 2))
        ok = np.sum(cand * cand, axis=1) < (1.0 - 1e-4) ** 2
        out[todo[ok]] = cand[ok]
        todo = todo[~ok]
    return np.ascontiguousarray(out.astype(dtype))


def random_csr(n: int, k: int = 90, seed: int = 11, dtype=np.float32):
    """Row structure of a symmetrised k-NN graph (about k to 2k entries per
    row, columns ascending, no diagonal), random positive values normalised
    to sum 1.  For inputs whose only role is their sparsity shape."""
    g = rng(seed)
    lens = k + g.integers(0, k + 1, size=n)
    rows = np.repeat(np.arange(n, dtype=np.int64), lens)
    cols = g.integers(0, n - 1, size=rows.size)
    cols = cols + (cols >= rows)                    # skip the diagonal
    key = np.unique(rows * n + cols)                # sorted, duplicates removed
    rows, cols = key // n, key % n
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=row_ptr[1:])
    val = g.random(cols.size)
    val /= val.sum()
    return row_ptr, cols.astype(np.int32), val.astype(dtype)


def subsample(n: int, m: int, seed: int = 99) -> np.ndarray:
    """Sorted uniform sample of m distinct row indices out of n."""
    g = rng(seed)
    return np.sort(g.choice(n, size=min(m, n), replace=False)).astype(np.int64)


def near_split_rays(levels=range(1, 20), rays_per_level: int = 3, ulps=(-2, -1, 0, 1, 2),
                    seed: int = 61, background: int = 300) -> np.ndarray:
    """Single-precision points straddling the angular split rays.

    For every level l and a few random cells j of that level, the ray at
    angle 2 pi (2j + 1) / 2^(l + 1) (the middle of the cell's angular range)
    gets a point at a random radius rounded to single precision, and copies
    of it moved by the given numbers of units in the last place along x;
    such a family shares every cell above level l and is split by the ray.
    A uniform background keeps the root annulus and the upper levels busy."""
    g = rng(seed)
    pts = []
    for lvl in levels:
        for _ in range(rays_per_level):
            j = int(g.integers(0, 2 ** lvl))
            a = 2.0 * np.pi * (2 * j + 1) / 2.0 ** (lvl + 1)
            r = g.uniform(0.05, 0.95)
            x = np.float32(r * np.cos(a))
            y = np.float32(r * np.sin(a))
            for u in ulps:
                xu = x
                step = np.float32(np.inf) if u > 0 else np.float32(-np.inf)
                for _ in range(abs(u)):
                    xu = np.nextafter(xu, step)
                pts.append((xu, y))
    r = 0.95 * np.sqrt(g.random(background))
    phi = 2.0 * np.pi * g.random(background)
    bg = np.stack([r * np.cos(phi), r * np.sin(phi)], axis=1).astype(np.float32)
    out = np.concatenate([np.array(pts, dtype=np.float32), bg])
    return np.ascontiguousarray(out[g.permutation(out.shape[0])])
