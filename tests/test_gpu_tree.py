"""GPU polar quadtree against the oracle's insertion-built tree: node counts,
depths, pre-order links and the point order bit-exact; midpoints and cell
diameters within rounding."""
import numpy as np
import pytest
import torch

import oracle
from paper_2401_13708_amd import hts, synth
from gpu_inputs import STAGES, embedding

pytestmark = pytest.mark.gpu


def _gpu_tree(ctx, Y, max_depth=20, split=0):
    t = hts.Tree(ctx, Y.shape[0], max_depth)
    if split:
        t.set_split(split)
    hts.build_polar_tree(ctx, torch.from_numpy(Y).cuda(), t)
    out = hts.tree_export(ctx, t, Y.shape[0])
    t.close()
    return out


def _compare(ctx, Y, max_depth=20, mid_rtol=1e-12, split=0, g=None):
    if g is None:
        g = _gpu_tree(ctx, Y, max_depth, split)
    o = oracle.Tree(Y.astype(np.float64), max_depth, split_rule=split).export()
    assert g["count"].size == o["count"].size
    for key in ("count", "depth", "first", "next"):
        assert np.array_equal(g[key], o[key]), key
    assert np.array_equal(g["perm"], o["perm"].astype(np.int32))
    # a single-point leaf carries the point itself (the midpoint of one point)
    leaf1 = (o["next"] == np.arange(o["next"].size) + 1) & (o["count"] == 1)
    pts = Y[o["perm"][o["first"][leaf1]]].astype(np.float64)
    assert np.array_equal(g["mid"][leaf1], pts)
    # other midpoints: rounding of eq. (11), relative to the disk scale
    # (an absolute floor for midpoints that cancel to ~0, like a symmetric root)
    # The Klein-to-disk map m = K / (1 + s), s = sqrt(1 - |K|^2) ~ (1 - |m|^2) / 2,
    # amplifies the summation error of K (up to count * eps for the oracle's
    # plain sums) by 1 / s for midpoints near the rim.
    scale = max(float(np.abs(Y).max()), 1e-300)
    mo = o["mid"][~leaf1]
    m2 = np.sum(mo * mo, 1)
    s = (1 - m2) / (1 + m2)
    rtol = mid_rtol + o["count"][~leaf1] * 1.2e-16 / s
    assert np.all(np.abs(g["mid"][~leaf1] - mo) <= rtol[:, None] * np.abs(mo) + 1e-14 * scale)
    # diameters: the oracle evaluates eq. (8) at corners (r cos phi, r sin phi);
    # 1 - |c|^2 carries a relative error of about eps / (1 - r_hi^2) and the
    # corner differences one of about eps r_hi / (cell extent)
    rlo, rhi = o["bounds"][:, 0], o["bounds"][:, 1]
    extent = np.maximum(rhi - rlo, rhi * np.minimum(np.pi, o["bounds"][:, 3] - o["bounds"][:, 2]))
    tol = 2e-12 + 2e-15 / (1.0 - rhi * rhi) + 2e-15 * rhi / np.maximum(extent, 1e-300)
    assert np.all(np.abs(g["r_cell"] - o["r_cell"]) <= tol * o["r_cell"] + 1e-300)


@pytest.mark.parametrize("stage", STAGES)
@pytest.mark.parametrize("n", [2, 3, 257, 4099])
def test_tree_f64(ctx, stage, n):
    _compare(ctx, embedding(n, stage, np.float64), mid_rtol=1e-11)


@pytest.mark.parametrize("stage", STAGES)
def test_tree_f32(ctx, stage):
    # midpoints are stored in single precision
    _compare(ctx, embedding(5000, stage, np.float32), mid_rtol=1.2e-7)


def test_tree_duplicates_and_caps(ctx):
    Y = embedding(3000, "mid", np.float64)
    Y[100:160] = Y[7]
    Y[500] = Y[501] = Y[502]
    for depth in (20, 8, 3, 1):
        _compare(ctx, Y, depth, mid_rtol=1e-11)


def test_tree_same_radius_and_axis_points(ctx):
    k = np.arange(512)
    ring = np.stack([0.5 * np.cos(k * 2 * np.pi / 512), 0.5 * np.sin(k * 2 * np.pi / 512)], 1)
    axis = np.array([[0.3, 0.0], [-0.3, 0.0], [0.0, 0.3], [0.0, -0.3], [0.0, 0.0], [1e-30, -1e-30]])
    _compare(ctx, np.concatenate([ring, axis]).astype(np.float64), mid_rtol=1e-11)


@pytest.mark.parametrize("stage", STAGES)
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_tree_equal_area_split(ctx, stage, dtype):
    # eq. (9): the split radius is reproduced to the bit, so the node set is
    # the oracle's
    _compare(ctx, embedding(4099, stage, dtype), mid_rtol=1.2e-7 if dtype == np.float32 else 1e-11,
             split=1)


def test_tree_equal_area_duplicates_and_caps(ctx):
    Y = embedding(3000, "late", np.float64)
    Y[100:160] = Y[7]
    for depth in (20, 5):
        _compare(ctx, Y, depth, mid_rtol=1e-11, split=1)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("max_depth,split", [(20, 0), (24, 0), (20, 1)])
def test_tree_points_straddling_the_split_rays(ctx, dtype, max_depth, split):
    # families of points a few units in the last place either side of the
    # rays that halve the cells' angular ranges at levels 1-19 (and 20-23
    # for the deeper cap): the angular decision is an exact sign test on both
    # sides, so the trees agree node for node even there
    levels = range(1, min(max_depth, 24))
    Y = synth.near_split_rays(levels=levels, seed=61 + max_depth).astype(dtype)
    # midpoints of the single-precision tree are stored in single precision
    _compare(ctx, Y, max_depth, mid_rtol=1.2e-7 if dtype == np.float32 else 1e-11, split=split)


def test_tree_destroyed_after_its_context():
    # destroying a tree after its context touches nothing of the context, and
    # leaves no HIP error behind for the next call
    c = hts.Context(0)
    t = hts.Tree(c, 1000, 20)
    hts.build_polar_tree(c, torch.from_numpy(embedding(1000, "mid", np.float32)).cuda(), t)
    torch.cuda.synchronize()
    c.close()
    t.close()
    c2 = hts.Context(0)
    Y = torch.from_numpy(embedding(300, "mid", np.float32)).cuda()
    t2 = hts.Tree(c2, 300, 20)
    hts.build_polar_tree(c2, Y, t2)
    torch.cuda.synchronize()
    assert c2.check() == 0
    t2.close()
    c2.close()


def test_tree_build_replayed_from_a_graph_on_new_points(ctx):
    # a tree build captured as a HIP graph and replayed on other points of
    # the same size gives their tree: every buffer the build reads is written
    # earlier in the same build, so no replay depends on what an earlier one
    # left (40 sort tiles, 5 digit passes, other GPU work between the replays)
    n = 20000
    t = hts.Tree(ctx, n, 20)
    Ybuf = torch.from_numpy(embedding(n, "mid", np.float32)).cuda()
    hts.build_polar_tree(ctx, Ybuf, t)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        hts.build_polar_tree(ctx, Ybuf, t)
    scratch = torch.ones(1 << 20, device="cuda")
    for k, stage in enumerate(STAGES + STAGES[::-1]):
        Y = embedding(n, stage, np.float32, seed=200 + k)
        Ybuf.copy_(torch.from_numpy(Y))
        g.replay()
        scratch.mul_(1.0001)
        torch.cuda.synchronize()
        print("replay", k, stage, flush=True)
        _compare(ctx, Y, mid_rtol=1.2e-7, g=hts.tree_export(ctx, t, n))
    assert ctx.check() == 0
    t.close()
