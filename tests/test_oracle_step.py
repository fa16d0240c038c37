"""Pins of the oracle's Riemannian step (eqs. (7), (16)-(18) and the optimiser
of Sec. 5: momentum, gains, learning rate)."""
import numpy as np
import pytest

import oracle
from paper_2401_13708_amd import synth


def test_step_matches_independent_update_rule():
    n = 300
    g = synth.rng(1)
    Y = synth.disk_state(n, "mid", seed=2).astype(np.float64)
    U = g.normal(size=(n, 2)) * 1e-3
    G = g.uniform(0.5, 2.0, size=(n, 2))
    grad = g.normal(size=(n, 2))
    eta, mu = n / 12000.0, 0.8
    Y1, U1, G1 = oracle.step(Y, U, G, grad, eta, mu)
    # independent: delta-bar-delta gains, momentum, metric rescale, exp map
    s = (1 - np.sum(Y * Y, 1, keepdims=True)) ** 2 / 4
    gh = s * grad
    Gr = np.where((gh > 0) != (U > 0), G + 0.2, G * 0.8)
    Gr = np.maximum(Gr, 0.01)
    Ur = mu * U - eta * Gr * gh
    assert np.array_equal(G1, Gr)
    assert np.allclose(U1, Ur, rtol=1e-15, atol=0)
    lam = 2 / (1 - np.sum(Y * Y, 1))
    for i in range(n):
        # the new point is on the geodesic from y in direction u, at distance lambda |u|
        assert oracle.dist(Y[i], Y1[i]) == pytest.approx(lam[i] * np.hypot(*Ur[i]), rel=1e-7)
        assert Y1[i] @ Y1[i] < 1


def test_zero_gradient_and_update_keeps_points():
    Y = synth.disk_state(50, "late", seed=3).astype(np.float64)
    Z = np.zeros_like(Y)
    Y1, U1, G1 = oracle.step(Y, Z, np.ones_like(Y), Z, 1.0, 0.5)
    assert np.array_equal(Y1, Y) and np.array_equal(U1, Z)
    assert np.allclose(G1, 0.8)


def test_gain_floor():
    Y = np.array([[0.1, 0.2]])
    G = np.array([[0.011, 0.011]])
    U = np.array([[1e-4, -1e-4]])
    grad = np.array([[1.0, -1.0]])          # same sign as u -> gains x0.8
    _, _, G1 = oracle.step(Y, U, G, grad, 1.0, 0.5, min_gain=0.01)
    assert np.array_equal(G1, [[0.01, 0.01]])


def test_projection_back_into_the_disk():
    # a huge step saturates tanh; the projection of eq. (18) keeps 1 - eps
    Y = np.array([[0.999, 0.0], [0.0, -0.9999]])
    U = np.zeros((2, 2))
    grad = np.array([[-1e12, 0.0], [0.0, 1e12]])
    Y1, _, _ = oracle.step(Y, U, np.ones((2, 2)), grad, 1e6, 0.5, boundary_eps=1e-5)
    r = np.hypot(Y1[:, 0], Y1[:, 1])
    assert np.all(r < 1)
    assert np.all(r >= 1 - 1e-5 - 1e-15)


def test_metric_power_one_uses_lambda_inverse():
    Y = np.array([[0.5, 0.0]])
    grad = np.array([[1.0, 0.0]])
    _, U2, _ = oracle.step(Y, np.zeros((1, 2)), np.ones((1, 2)), grad, 1.0, 0.0, metric_power=2)
    _, U1, _ = oracle.step(Y, np.zeros((1, 2)), np.ones((1, 2)), grad, 1.0, 0.0, metric_power=1)
    a = 1 - 0.25
    assert U2[0, 0] == pytest.approx(-1.2 * a * a / 4)
    assert U1[0, 0] == pytest.approx(-1.2 * a / 2)
