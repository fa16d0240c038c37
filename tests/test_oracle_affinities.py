"""Pins of the oracle's input affinities (Sec. 2-A eq. (1), truncated to k
nearest neighbours and symmetrised): brute-force k-NN, achieved perplexity,
and the structure of the symmetric P."""
import numpy as np
import pytest

import oracle
from paper_2401_13708_amd import synth


def _np_knn(X, k):
    n = X.shape[0]
    D = np.sum((X[:, None, :] - X[None, :, :]) ** 2, -1)
    out = np.zeros((n, k), dtype=np.int64)
    for i in range(n):
        js = np.array([j for j in range(n) if j != i])
        order = np.lexsort((js, D[i, js]))
        out[i] = js[order[:k]]
    return out, D


@pytest.mark.parametrize("n,d,k", [(64, 8, 10), (50, 32, 20), (40, 3, 39)])
def test_knn_brute_force(n, d, k):
    X = synth.gaussian_mixture(n, d, seed=n + d)
    idx, d2 = oracle.knn_rows(X, k)
    ref, D = _np_knn(X, k)
    assert np.array_equal(idx, ref)
    assert np.allclose(d2, np.take_along_axis(D, ref, 1), rtol=1e-13)
    assert np.all(np.diff(d2, axis=1) >= 0)


def test_knn_ties_break_by_index():
    X = np.zeros((12, 4))
    X[5:] = 1.0                       # 7 identical points and 5 identical points
    idx, d2 = oracle.knn_rows(X, 6)
    assert idx[0].tolist() == [1, 2, 3, 4, 5, 6]
    assert idx[7].tolist() == [5, 6, 8, 9, 10, 11]
    assert np.all(d2[7] == 0)


def test_knn_subset_rows_match_full():
    X = synth.gaussian_mixture(120, 16, seed=3)
    full, dfull = oracle.knn_rows(X, 30)
    rows = np.array([0, 17, 64, 119])
    sub, dsub = oracle.knn_rows(X, 30, rows)
    assert np.array_equal(sub, full[rows]) and np.array_equal(dsub, dfull[rows])


@pytest.mark.parametrize("perp,k", [(30.0, 90), (5.0, 15), (10.0, 11)])
def test_perplexity_is_reached(perp, k):
    X = synth.gaussian_mixture(300, 10, seed=4)
    _, d2 = oracle.knn_rows(X, k)
    p, beta = oracle.cond_p(d2, perp)
    H = -np.sum(np.where(p > 0, p * np.log(np.where(p > 0, p, 1)), 0), 1)
    assert np.allclose(H, np.log(perp), atol=1e-10)
    assert np.allclose(p.sum(1), 1, atol=1e-14)
    assert np.all(beta > 0)
    # the Gaussian shape of eq. (1): log p is affine in the squared distance with slope -beta
    for i in range(0, 300, 37):
        sl = np.polyfit(d2[i], np.log(p[i]), 1)[0]
        assert sl == pytest.approx(-beta[i], rel=1e-8)


def test_symmetric_p_structure():
    n, k = 200, 30
    X = synth.gaussian_mixture(n, 12, seed=5)
    knn, rp, col, val = oracle.build_affinities(X, 10.0, k)
    P = np.zeros((n, n))
    for i in range(n):
        cs = col[rp[i]:rp[i + 1]]
        assert np.all(np.diff(cs) > 0)              # sorted, no duplicates
        P[i, cs] = val[rp[i]:rp[i + 1]]
    assert np.allclose(P, P.T, rtol=0, atol=1e-18)
    assert np.sum(P) == pytest.approx(1.0, abs=1e-14)
    assert np.all(val > 0) and np.all(np.diag(P) == 0)
    pattern = np.zeros((n, n), bool)
    for i in range(n):
        pattern[i, knn[i]] = True
    pattern |= pattern.T
    assert np.array_equal(P > 0, pattern)
    # p_ij = (p_{j|i} + p_{i|j}) / (2 n)
    _, d2 = oracle.knn_rows(X, k)
    pc, _ = oracle.cond_p(d2, 10.0)
    C = np.zeros((n, n))
    for i in range(n):
        C[i, knn[i]] = pc[i]
    assert np.allclose(P, (C + C.T) / (2 * n), rtol=1e-14, atol=0)


def test_invalid_arguments():
    X = synth.gaussian_mixture(20, 4, seed=6)
    with pytest.raises(RuntimeError):
        oracle.build_affinities(X, 30.0, 19)   # perplexity >= k
    with pytest.raises(RuntimeError):
        oracle.build_affinities(X, 5.0, 20)    # k >= n
