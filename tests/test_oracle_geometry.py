"""Pins of the oracle's Poincare-disk geometry against closed forms and invariants
(Sec. 2-C eqs. (7)-(8), Sec. 4-A eq. (11), Sec. 4-B eqs. (13), (16)-(17))."""
import numpy as np
import pytest

import oracle


def _rand_disk(g, n, rmax=0.95):
    r = rmax * np.sqrt(g.random(n))
    p = 2 * np.pi * g.random(n)
    return np.stack([r * np.cos(p), r * np.sin(p)], 1)


def test_distance_from_origin_closed_form():
    # d(0, y) = 2 artanh |y|: the radial geodesic of the metric of eq. (7)
    g = np.random.default_rng(0)
    for y in _rand_disk(g, 200, 0.999):
        r = np.hypot(*y)
        assert oracle.dist([0, 0], y) == pytest.approx(2 * np.arctanh(r), rel=1e-13, abs=1e-300)


def test_distance_symmetry_and_triangle():
    g = np.random.default_rng(1)
    P = _rand_disk(g, 300)
    for a, b, c in zip(P[0::3], P[1::3], P[2::3]):
        dab, dba = oracle.dist(a, b), oracle.dist(b, a)
        assert dab == pytest.approx(dba, rel=1e-14)
        assert dab <= oracle.dist(a, c) + oracle.dist(c, b) + 1e-12


def test_mobius_translation_is_an_isometry():
    g = np.random.default_rng(2)
    P = _rand_disk(g, 300, 0.9)
    for a, x, y in zip(P[0::3], P[1::3], P[2::3]):
        d0 = oracle.dist(x, y)
        d1 = oracle.dist(oracle.mobius_add(a, x), oracle.mobius_add(a, y))
        assert d1 == pytest.approx(d0, rel=1e-10)


def test_boundary_example_closed_form():
    # Sec. 5 prints d((-1+1e-4, 0), (1-1e-4, 0)) as "about 80"; eq. (8) gives
    # 2 ln((1+r)/(1-r)) for r = 1-1e-4, i.e. 2 ln(19999) = 19.807...  The
    # closed form decides (the printed figure is not reproducible from eq. (8)).
    d = oracle.dist([-1 + 1e-4, 0.0], [1 - 1e-4, 0.0])
    assert d == pytest.approx(2 * np.log(19999.0), rel=1e-10)
    assert 19.80 < d < 19.81


def test_distance_tiny_separation_keeps_relative_accuracy():
    # near the origin d ~ 2 |a - b| (lambda_0 = 2); the log1p form keeps digits
    a = np.array([3e-7, -1e-7])
    b = np.array([3.5e-7, 0.5e-7])
    assert oracle.dist(a, b) == pytest.approx(2 * np.hypot(*(a - b)), rel=1e-12)


def test_distance_gradient_matches_finite_differences():
    g = np.random.default_rng(3)
    P = _rand_disk(g, 100, 0.9)
    h = 1e-7
    for a, b in zip(P[0::2], P[1::2]):
        gr = oracle.dist_grad(a, b)
        fd = np.zeros(2)
        for c in range(2):
            e = np.zeros(2)
            e[c] = h
            fd[c] = (oracle.dist(a + e, b) - oracle.dist(a - e, b)) / (2 * h)
        assert np.allclose(gr, fd, rtol=1e-6, atol=1e-7)


def test_distance_gradient_matches_printed_form():
    # eq. (13) in its printed arrangement, at well-separated points
    g = np.random.default_rng(4)
    P = _rand_disk(g, 100, 0.9)
    for a, b in zip(P[0::2], P[1::2]):
        al = 1 - a @ a
        be = 1 - b @ b
        gam = 1 + 2 * (a - b) @ (a - b) / (al * be)
        lit = 4 * ((b @ b - 2 * a @ b + 1) * a / al - b) / (al * be * np.sqrt(gam * gam - 1))
        assert np.allclose(oracle.dist_grad(a, b), lit, rtol=1e-9, atol=1e-12)


def test_distance_force_euclidean_limit():
    # d * dd/dy_i -> 4 (y_i - y_j) as both points approach the origin
    a = np.array([2e-6, 1e-6])
    b = np.array([-1e-6, 3e-6])
    f = oracle.dist(a, b) * oracle.dist_grad(a, b)
    assert np.allclose(f, 4 * (a - b), rtol=1e-9)


def test_exp_map_identities():
    g = np.random.default_rng(5)
    P = _rand_disk(g, 60, 0.9)
    for y, v in zip(P[0::2], P[1::2] * 0.7):
        # exp_y(0) = y
        assert np.array_equal(oracle.exp_map(y, [0.0, 0.0]), y)
        # geodesic length: d(y, exp_y(v)) = lambda_y |v|
        lam = 2 / (1 - y @ y)
        z = oracle.exp_map(y, v)
        if lam * np.hypot(*v) < 15:
            assert oracle.dist(y, z) == pytest.approx(lam * np.hypot(*v), rel=1e-8)
        assert z @ z < 1
        # exp_0(v) = tanh(|v|) v / |v|
        nv = np.hypot(*v)
        assert np.allclose(oracle.exp_map([0, 0], v), np.tanh(nv) * v / nv, rtol=1e-14)


def test_mobius_identities():
    g = np.random.default_rng(6)
    for y in _rand_disk(g, 50, 0.99):
        assert np.allclose(oracle.mobius_add([0, 0], y), y, rtol=0, atol=1e-16)
        assert np.allclose(oracle.mobius_add(y, [0, 0]), y, rtol=0, atol=1e-16)
        assert np.allclose(oracle.mobius_add(-y, y), 0, atol=1e-15)


def test_einstein_midpoint_properties():
    g = np.random.default_rng(7)
    for _ in range(20):
        y = _rand_disk(g, 1, 0.99)[0]
        assert np.allclose(oracle.einstein_midpoint(y[None]), y, rtol=1e-13, atol=1e-16)
        assert np.allclose(oracle.einstein_midpoint(np.stack([y, -y])), 0, atol=1e-15)
    # rotation equivariance
    P = _rand_disk(g, 17, 0.95)
    th = 0.731
    R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    assert np.allclose(oracle.einstein_midpoint(P @ R.T), oracle.einstein_midpoint(P) @ R.T,
                       atol=1e-14)
    # gyro-covariance under Mobius translation: m(a (+) y_j) = a (+) m(y_j)
    a = np.array([0.3, -0.4])
    moved = np.stack([oracle.mobius_add(a, y) for y in P])
    assert np.allclose(oracle.einstein_midpoint(moved),
                       oracle.mobius_add(a, oracle.einstein_midpoint(P)), atol=1e-12)
    # two points: the midpoint lies on their geodesic, equidistant from both
    x, y = np.array([0.5, 0.1]), np.array([-0.2, 0.6])
    m = oracle.einstein_midpoint(np.stack([x, y]))
    assert oracle.dist(x, m) == pytest.approx(oracle.dist(m, y), rel=1e-10)
    assert oracle.dist(x, m) + oracle.dist(m, y) == pytest.approx(oracle.dist(x, y), rel=1e-10)
