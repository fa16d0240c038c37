"""Pins of the oracle's h-SNE terms (Sec. 4-C): the Euclidean Student-t cost of
the disk coordinates and its exact gradient against finite differences and a
two-point closed form; the combined h-SNE gradient against finite differences
of KL(P||Q^E) + lambda KL(P||Q^H); the Barnes-Hut Euclidean gradient over the
polar quadtree against the exact one (theta = 0, error band, Newton's third
law); the per-cell centres of mass and Euclidean diameters against brute
force."""
import numpy as np
import pytest

import oracle
from paper_2401_13708_amd import synth


def _problem(n=40, seed=0, stage="mid", perplexity=5.0, k=15):
    X = synth.gaussian_mixture(n, 8, n_clusters=4, seed=seed)
    _, rp, col, val = oracle.build_affinities(X, perplexity, k)
    Y = synth.disk_state(n, stage, n_clusters=4, seed=seed + 100).astype(np.float64)
    return Y, rp, col, val


def _fd(fun, Y):
    g = np.zeros_like(Y)
    for i in range(Y.shape[0]):
        h = 1e-6 * (1 - Y[i] @ Y[i])
        for c in range(2):
            Yp, Ym = Y.copy(), Y.copy()
            Yp[i, c] += h
            Ym[i, c] -= h
            g[i, c] = (fun(Yp) - fun(Ym)) / (2 * h)
    return g


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("stage,ex", [("mid", 1.0), ("early", 1.0), ("late", 1.0), ("mid", 12.0)])
def test_euclid_gradient_is_the_cost_derivative(stage, ex):
    Y, rp, col, val = _problem(36, seed=3, stage=stage)
    g, _ = oracle.gradient_euclid_exact(Y, rp, col, val, ex)
    fd = _fd(lambda Z: oracle.euclid_cost(Z, rp, col, val, ex), Y)
    assert _rel(g, fd) < 1e-6


def test_euclid_two_points_closed_form():
    # n = 2, p_12 = p_21 = 1/2: q is 1/2 whatever the distance, so the cost is
    # 0 at a = 1 and the gradient is 2 w (a - 1) (y_1 - y_2), w = 1 / (1 + s^2)
    Y = np.array([[0.3, -0.2], [-0.1, 0.45]])
    rp = np.array([0, 1, 2], np.int64)
    col = np.array([1, 0], np.int32)
    val = np.array([0.5, 0.5])
    diff = Y[0] - Y[1]
    w = 1.0 / (1.0 + diff @ diff)
    for a in (1.0, 4.0):
        g, z = oracle.gradient_euclid_exact(Y, rp, col, val, a)
        assert z == pytest.approx(2 * w, rel=1e-15)
        assert np.allclose(g[0], 2 * w * (a - 1) * diff, rtol=1e-14, atol=1e-14)
        assert np.allclose(g[1], -g[0], rtol=1e-14, atol=1e-14)
    assert oracle.euclid_cost(Y, rp, col, val, 1.0) == pytest.approx(0.0, abs=1e-15)


@pytest.mark.parametrize("lam", [0.5, 2.0])
def test_hsne_gradient_is_the_cost_derivative(lam):
    Y, rp, col, val = _problem(32, seed=5, stage="mid")
    t = oracle.Tree(Y)
    g, ze, zh = oracle.hsne_gradient_bh(Y, rp, col, val, t, 0.0, lam)
    fd = _fd(lambda Z: oracle.hsne_cost(Z, rp, col, val, lam), Y)
    assert _rel(g, fd) < 1e-6
    assert ze == pytest.approx(oracle.gradient_euclid_exact(Y, rp, col, val)[1], rel=1e-13)
    assert zh == pytest.approx(oracle.z_exact(Y), rel=1e-13)


def test_printed_minus_sign_fails_fd():
    # the printed second part has a minus sign: that form is not the
    # derivative of the stated cost
    Y, rp, col, val = _problem(28, seed=6)
    ge, _ = oracle.gradient_euclid_exact(Y, rp, col, val)
    gh, _ = oracle.gradient_exact(Y, rp, col, val)
    fd = _fd(lambda Z: oracle.hsne_cost(Z, rp, col, val, 1.0), Y)
    assert _rel(ge - gh, fd) > 0.05
    assert _rel(ge + gh, fd) < 1e-6


@pytest.mark.parametrize("stage", ["init", "early", "mid", "late", "edge"])
def test_euclid_bh_theta_zero_equals_exact(stage):
    Y, rp, col, val = _problem(300, seed=7, stage=stage)
    t = oracle.Tree(Y)
    gb, zb, cnt = oracle.gradient_euclid_bh(Y, rp, col, val, t, 0.0, 3.0)
    ge, zx = oracle.gradient_euclid_exact(Y, rp, col, val, 3.0)
    assert cnt["accepts"] == 0
    assert cnt["pairs"] == Y.shape[0] * (Y.shape[0] - 1)
    assert _rel(gb, ge) < 1e-12
    assert zb == pytest.approx(zx, rel=1e-12)


def test_euclid_bh_error_band_and_newton():
    Y, rp, col, val = _problem(800, seed=8, stage="mid")
    t = oracle.Tree(Y)
    ge, zx = oracle.gradient_euclid_exact(Y, rp, col, val)
    # exact forces cancel in pairs (P symmetric): the total is zero
    assert np.abs(ge.sum(axis=0)).max() < 1e-12 * np.abs(ge).sum()
    errs = []
    for theta in (0.2, 0.5, 0.8):
        gb, zb, cnt = oracle.gradient_euclid_bh(Y, rp, col, val, t, theta)
        errs.append(_rel(gb, ge))
        assert cnt["accepts"] > 0
        assert abs(zb / zx - 1) < 0.02
    assert errs[0] < errs[1] < errs[2]
    assert errs[1] < 0.05, errs


def test_euclid_cell_summaries_brute_force():
    Y = synth.disk_state(500, "mid", n_clusters=4, seed=9).astype(np.float64)
    t = oracle.Tree(Y)
    e = t.export()
    cent, diam = t.export_euclid()
    Ys = Y.astype(np.float32).astype(np.float64)  # the tree places the single-precision points
    for k in range(t.n_nodes):
        f, c = e["first"][k], e["count"][k]
        pts = Y[e["perm"][f:f + c]]
        assert np.allclose(cent[k], pts.mean(axis=0), rtol=0, atol=1e-15)
        r_lo, r_hi, p_lo, p_hi = e["bounds"][k]
        if c > 1:
            # no two points of the cell are farther apart than its diameter
            q = Ys[e["perm"][f:f + c]]
            far = np.sqrt(((q[:, None, :] - q[None, :, :]) ** 2).sum(-1)).max()
            assert far <= diam[k] * (1 + 1e-12)
        # the boundary of the cell, sampled densely with its corners: the
        # largest distance is the diameter (angular widths >= pi read as pi)
        w = min(p_hi - p_lo, np.pi)
        rs = np.linspace(r_lo, r_hi, 40)
        ps = np.linspace(p_lo, p_lo + w, 200)
        bx = np.concatenate([r_lo * np.cos(ps), r_hi * np.cos(ps), rs * np.cos(p_lo),
                             rs * np.cos(p_lo + w)])
        by = np.concatenate([r_lo * np.sin(ps), r_hi * np.sin(ps), rs * np.sin(p_lo),
                             rs * np.sin(p_lo + w)])
        b = np.stack([bx, by], 1)
        far_b = np.sqrt(((b[:, None, :] - b[None, :, :]) ** 2).sum(-1)).max()
        assert far_b == pytest.approx(diam[k], rel=1e-12, abs=1e-15)
        if e["depth"][k] == 0:
            assert diam[k] == pytest.approx(2 * r_hi, rel=1e-12)
