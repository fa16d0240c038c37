"""Pins of the oracle's cost, exact gradient and Barnes-Hut gradient
(eqs. (3), (12)-(15), (19)) against finite differences, brute force, symmetry,
the Euclidean limit (eq. (4)) and the theta = 0 reduction (Sec. 5)."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_2401_13708_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _problem(n=48, seed=0, stage="mid", perplexity=5.0, k=15):
    X = synth.gaussian_mixture(n, 8, n_clusters=4, seed=seed)
    _, rp, col, val = oracle.build_affinities(X, perplexity, k)
    Y = synth.disk_state(n, stage, n_clusters=4, seed=seed + 100).astype(np.float64)
    return Y, rp, col, val


@pytest.mark.parametrize("stage,ex", [("mid", 1.0), ("early", 1.0), ("late", 1.0), ("mid", 12.0)])
def test_exact_gradient_is_the_cost_derivative(stage, ex):
    Y, rp, col, val = _problem(40, seed=1, stage=stage)
    g, _ = oracle.gradient_exact(Y, rp, col, val, ex)
    # central differences of the cost, step scaled to the local metric
    fd = np.zeros_like(Y)
    for i in range(Y.shape[0]):
        h = 1e-6 * (1 - Y[i] @ Y[i])
        for c in range(2):
            Yp, Ym = Y.copy(), Y.copy()
            Yp[i, c] += h
            Ym[i, c] -= h
            fd[i, c] = (oracle.kl_cost(Yp, rp, col, val, ex) - oracle.kl_cost(Ym, rp, col, val, ex)) / (2 * h)
    err = np.linalg.norm(g - fd) / np.linalg.norm(g)
    assert err < 1e-6, err


def test_printed_gradient_without_distance_factor_fails_fd():
    # eq. (14) as printed omits the factor d_ij; that form is not the derivative
    Y, rp, col, val = _problem(24, seed=2)
    g, z = oracle.gradient_exact(Y, rp, col, val, 1.0)
    n = Y.shape[0]
    lit = np.zeros_like(Y)
    P = np.zeros((n, n))
    for i in range(n):
        P[i, col[rp[i]:rp[i + 1]]] = val[rp[i]:rp[i + 1]]
    for i in range(n):
        for j in range(n):
            if i == j:
                continue
            d = oracle.dist(Y[i], Y[j])
            w = 1 / (1 + d * d)
            lit[i] += 4 * (P[i, j] - w / z) * w * oracle.dist_grad(Y[i], Y[j])
    assert np.linalg.norm(lit - g) / np.linalg.norm(g) > 0.05


def test_z_brute_force():
    Y, rp, col, val = _problem(30, seed=3)
    _, z = oracle.gradient_exact(Y, rp, col, val)
    # independent evaluation: arccosh of the eq. (8) argument, ordered pairs
    n = Y.shape[0]
    s = 0.0
    for i in range(n):
        for j in range(n):
            if i != j:
                a, b = Y[i], Y[j]
                gam = 1 + 2 * (a - b) @ (a - b) / ((1 - a @ a) * (1 - b @ b))
                s += 1 / (1 + np.arccosh(gam) ** 2)
    assert z == pytest.approx(s, rel=1e-12)
    assert oracle.z_exact(Y) == pytest.approx(s, rel=1e-12)


def test_rotation_covariance():
    Y, rp, col, val = _problem(36, seed=4)
    th = 1.234
    R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    g0, z0 = oracle.gradient_exact(Y, rp, col, val, 4.0)
    g1, z1 = oracle.gradient_exact(Y @ R.T, rp, col, val, 4.0)
    assert np.allclose(g1, g0 @ R.T, rtol=1e-10, atol=1e-12 * np.abs(g0).max())
    assert z1 == pytest.approx(z0, rel=1e-12)


def _euclid_grad(Y, P):
    # textbook Euclidean t-SNE gradient, eq. (4)
    D = Y[:, None, :] - Y[None, :, :]
    W = 1 / (1 + np.sum(D * D, -1))
    np.fill_diagonal(W, 0)
    Q = W / W.sum()
    return 4 * np.sum(((P - Q) * W)[:, :, None] * D, axis=1)


@pytest.mark.parametrize("scale,tol", [(1e-2, 3e-3), (1e-4, 1e-6)])
def test_near_origin_limit_is_euclidean_tsne(scale, tol):
    # near the origin d^H ~ 2 |y_i - y_j|, so g_H(Y) ~ 2 g_E(2 Y) with the error O(|y|^2)
    n = 40
    X = synth.gaussian_mixture(n, 6, n_clusters=4, seed=5)
    _, rp, col, val = oracle.build_affinities(X, 5.0, 15)
    P = np.zeros((n, n))
    for i in range(n):
        P[i, col[rp[i]:rp[i + 1]]] = val[rp[i]:rp[i + 1]]
    Y = synth.rng(6).normal(size=(n, 2)) * scale
    gh, _ = oracle.gradient_exact(Y, rp, col, val)
    ge = 2 * _euclid_grad(2 * Y, P)
    assert np.linalg.norm(gh - ge) / np.linalg.norm(ge) < tol


@pytest.mark.parametrize("stage", ["init", "early", "mid", "late", "edge"])
def test_bh_theta_zero_equals_exact(stage):
    Y, rp, col, val = _problem(60, seed=7, stage=stage)
    t = oracle.Tree(Y)
    gb, zb, cnt = oracle.gradient_bh(Y, rp, col, val, t, 0.0, 12.0)
    ge, ze = oracle.gradient_exact(Y, rp, col, val, 12.0)
    assert cnt["accepts"] == 0
    assert cnt["pairs"] == 60 * 59
    assert zb == pytest.approx(ze, rel=1e-12)
    assert np.allclose(gb, ge, rtol=1e-10, atol=1e-12 * np.abs(ge).max())


def test_bh_theta_zero_with_duplicates():
    Y, rp, col, val = _problem(50, seed=8)
    Y[10] = Y[11] = Y[12]
    Y[20] = Y[3]
    t = oracle.Tree(Y)
    gb, zb, _ = oracle.gradient_bh(Y, rp, col, val, t, 0.0)
    ge, ze = oracle.gradient_exact(Y, rp, col, val)
    assert zb == pytest.approx(ze, rel=1e-12)
    assert np.allclose(gb, ge, rtol=1e-10, atol=1e-12 * np.abs(ge).max())


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_bh_error_band_and_growth():
    # the gradient error of Table 3 (theta = 0.5) is about 1e-3 to 2.7e-3; on
    # synthetic data of the same kind the error must be of that order, and
    # it must grow with theta (Sec. 5, effect of theta)
    with open(os.path.join(GOLDEN, "paper_table3_gradient_error.json")) as f:
        band = json.load(f)
    lo, hi = min(band["gradient_error_theta_0_5"].values()), max(band["gradient_error_theta_0_5"].values())
    n = 1500
    X = synth.gaussian_mixture(n, 16, seed=9)
    _, rp, col, val = oracle.build_affinities(X, 30.0, 90)
    Y = synth.disk_state(n, "mid", seed=10).astype(np.float64)
    ge, ze = oracle.gradient_exact(Y, rp, col, val)
    t = oracle.Tree(Y)
    errs = {}
    for th in (0.3, 0.5, 0.8):
        gb, zb, _ = oracle.gradient_bh(Y, rp, col, val, t, th)
        errs[th] = _rel(gb, ge)
    assert errs[0.3] < errs[0.5] < errs[0.8]
    assert lo / 30 < errs[0.5] < hi * 10, (errs, lo, hi)


# ---------------------------------------------------------------- CO-SNE (Sec. 4-C)
def _fd(fun, Y):
    fd = np.zeros_like(Y)
    for i in range(Y.shape[0]):
        h = 1e-6 * (1 - Y[i] @ Y[i])
        for c in range(2):
            Yp, Ym = Y.copy(), Y.copy()
            Yp[i, c] += h
            Ym[i, c] -= h
            fd[i, c] = (fun(Yp) - fun(Ym)) / (2 * h)
    return fd


@pytest.mark.parametrize("lam1,lam2", [(1.0, 0.5), (0.3, 4.0), (1.0, 0.0)])
def test_cosne_gradient_is_the_cost_derivative(lam1, lam2):
    Y, rp, col, val = _problem(36, seed=3, stage="late")
    g = synth.rng(4)
    xn2 = g.uniform(0.0, 0.9, size=Y.shape[0])
    gk, _ = oracle.gradient_exact(Y, rp, col, val, 1.0)
    got = oracle.cosne_gradient(Y, xn2, lam1, lam2, gk)
    fd = _fd(lambda Z: oracle.cosne_cost(Z, rp, col, val, xn2, lam1, lam2), Y)
    assert np.linalg.norm(got - fd) / np.linalg.norm(fd) < 1e-6


def test_cosne_printed_sign_fails_fd():
    # the variation as printed, +(4 lambda2 / n)(|x|^2 - |y|^2) y, is not the
    # derivative of the stated cost
    Y, rp, col, val = _problem(36, seed=5, stage="mid")
    xn2 = synth.rng(6).uniform(0.0, 0.9, size=Y.shape[0])
    gk, _ = oracle.gradient_exact(Y, rp, col, val, 1.0)
    n, lam2 = Y.shape[0], 3.0
    printed = gk + (4 * lam2 / n) * (xn2 - np.sum(Y * Y, 1))[:, None] * Y
    fd = _fd(lambda Z: oracle.cosne_cost(Z, rp, col, val, xn2, 1.0, lam2), Y)
    assert np.linalg.norm(printed - fd) / np.linalg.norm(fd) > 1e-2
    # the norm term alone: at |y_i|^2 = |x_i|^2 it vanishes
    Z = Y.copy()
    xs = np.sum(Z * Z, 1)
    zero = oracle.cosne_gradient(Z, xs, 0.0, lam2, gk)
    assert np.abs(zero).max() < 1e-15


# ---------------------------------------------------------------- further pins
@pytest.mark.parametrize("stage,ex", [("early", 12.0), ("mid", 1.0), ("edge", 1.0)])
def test_exact_rows_equal_the_whole_gradient(stage, ex):
    # the row-subset routine (used where the whole O(n^2) gradient is too
    # slow) against the whole gradient, all rows, at three stages
    Y, rp, col, val = _problem(53, seed=21, stage=stage)
    g, z = oracle.gradient_exact(Y, rp, col, val, ex)
    rows = np.arange(Y.shape[0])
    gr = oracle.gradient_exact_rows(Y, rp, col, val, rows, z, ex)
    assert np.allclose(gr, g, rtol=1e-13, atol=1e-15 * np.abs(g).max())
    # and on a shuffled subset, each row where it belongs
    sub = synth.rng(22).permutation(Y.shape[0])[:17]
    gs = oracle.gradient_exact_rows(Y, rp, col, val, sub, z, ex)
    assert np.allclose(gs, g[sub], rtol=1e-13, atol=1e-15 * np.abs(g).max())


def _two_point_csr():
    rp = np.array([0, 1, 2], dtype=np.int64)
    col = np.array([1, 0], dtype=np.int32)
    val = np.array([0.5, 0.5])
    return rp, col, val


@pytest.mark.parametrize("a", [0.1, 0.5, 0.9])
@pytest.mark.parametrize("ex", [1.0, 2.0, 12.0])
def test_kl_cost_two_point_closed_form(a, ex):
    # two points at (a, 0) and (-a, 0): by symmetry about the origin their
    # distance is twice d(0, (a, 0)) = 2 artanh a, so d = 4 artanh a (eq. (8)),
    # w = (1 + d^2)^-1, Z = 2 w and q_12 = q_21 = 1/2 = p_12 = p_21.  The cost
    # sum ex p ln(ex p) - sum ex p ln w + ln Z is then
    # ex ln ex - (ex - 1)(ln 2 + ln w), which vanishes at ex = 1 (Q = P)
    Y = np.array([[a, 0.0], [-a, 0.0]])
    rp, col, val = _two_point_csr()
    d = 4.0 * np.arctanh(a)
    w = 1.0 / (1.0 + d * d)
    want = ex * np.log(ex) - (ex - 1.0) * (np.log(2.0) + np.log(w))
    got = oracle.kl_cost(Y, rp, col, val, ex)
    assert got == pytest.approx(want, rel=1e-13, abs=1e-14)
    if ex == 1.0:
        assert abs(got) < 1e-14


@pytest.mark.parametrize("stage", ["early", "mid", "late"])
@pytest.mark.parametrize("ex", [1.0, 12.0])
def test_kl_cost_dense_definition(stage, ex):
    # eq. (3) written out over dense matrices with numpy: q_ij = w_ij / Z from
    # arccosh of the eq. (8) argument, KL = sum p ln(p / q) for ex = 1, and in
    # general sum ex p ln(ex p) - sum ex p ln w + ln Z
    Y, rp, col, val = _problem(40, seed=23, stage=stage)
    n = Y.shape[0]
    P = np.zeros((n, n))
    for i in range(n):
        P[i, col[rp[i]:rp[i + 1]]] = val[rp[i]:rp[i + 1]]
    sq = np.sum(Y * Y, axis=1)
    D2 = np.sum((Y[:, None, :] - Y[None, :, :]) ** 2, axis=-1)
    gam = 1.0 + 2.0 * D2 / ((1.0 - sq)[:, None] * (1.0 - sq)[None, :])
    W = 1.0 / (1.0 + np.arccosh(gam) ** 2)
    np.fill_diagonal(W, 0.0)
    Z = W.sum()
    nz = P > 0
    if ex == 1.0:
        want = np.sum(P[nz] * np.log(P[nz] / (W[nz] / Z)))
    else:
        A = ex * P[nz]
        want = np.sum(A * np.log(A)) - np.sum(A * np.log(W[nz])) + np.log(Z)
    assert oracle.kl_cost(Y, rp, col, val, ex) == pytest.approx(want, rel=1e-11)


@pytest.mark.parametrize("stage", ["init", "early", "mid", "late", "edge"])
@pytest.mark.parametrize("theta", [0.3, 0.5, 0.8, 0.99, 1.5])
def test_bh_accounts_for_every_point_once(stage, theta):
    # whichever cells the criterion accepts, every query stands for each other
    # point exactly once: sum of N_cell over accepted cells + leaf pairs =
    # n (n - 1).  A cell counted twice, a skipped child or a leaf that keeps
    # the query itself breaks the identity.  Below theta = 1 no cell holding
    # the query can be accepted (its distance to the cell's midpoint or centre
    # of mass is at most the cell's diameter); from theta = 1 on such a cell
    # may stand for the query too, once per level at most.
    Y, rp, col, val = _problem(97, seed=31, stage=stage)
    n = Y.shape[0]
    t = oracle.Tree(Y)
    _, _, cnt = oracle.gradient_bh(Y, rp, col, val, t, theta, 1.0)
    _, _, ce = oracle.gradient_euclid_bh(Y, rp, col, val, t, theta, 1.0)
    if theta >= 0.5 and stage != "init":
        assert cnt["accepts"] > 0
    for c in (cnt, ce):
        if theta < 1.0:
            assert c["covered"] == n * (n - 1)
        else:
            assert n * (n - 1) <= c["covered"] <= n * (n - 1) + n * 20


def test_bh_accounts_for_every_point_once_with_duplicates_and_depth_cap():
    # duplicate points end in depth-capped leaves holding several points
    Y, rp, col, val = _problem(64, seed=33, stage="mid")
    Y[10:20] = Y[3]
    n = Y.shape[0]
    for depth in (3, 20):
        t = oracle.Tree(Y, max_depth=depth)
        _, _, cnt = oracle.gradient_bh(Y, rp, col, val, t, 0.5, 1.0)
        assert cnt["covered"] == n * (n - 1)


@pytest.mark.parametrize("stage,theta", [("mid", 0.5), ("edge", 0.3), ("early", 0.0)])
def test_bh_rows_equal_the_whole_bh_gradient(stage, theta):
    # the row-subset traversal (used to time a bounded sample of queries)
    # gives each sampled row of the whole Barnes-Hut gradient, and its
    # counters are those rows' share
    Y, rp, col, val = _problem(70, seed=41, stage=stage)
    t = oracle.Tree(Y)
    g, z, cnt = oracle.gradient_bh(Y, rp, col, val, t, theta, 12.0)
    rows = np.arange(Y.shape[0])
    gr, cr = oracle.gradient_bh_rows(Y, rp, col, val, t, theta, rows, z, 12.0)
    assert np.array_equal(gr, g)
    assert cr == cnt
    sub = synth.rng(42).permutation(Y.shape[0])[:9]
    gs, cs = oracle.gradient_bh_rows(Y, rp, col, val, t, theta, sub, z, 12.0)
    assert np.array_equal(gs, g[sub])
    assert cs["covered"] == 9 * (Y.shape[0] - 1)
