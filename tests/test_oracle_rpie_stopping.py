"""Pins of the oracle's rPIE regularisation vector (Section 2.1, the u^rPIE choice)
and of the stopping statistic of Section 5 ("Stopping criterion"), on values worked
out by hand.

u^rPIE = alpha (max|Q|^2 J - |Q|^2): zero where the probe is brightest, alpha max|Q|^2
where it vanishes, and u + |Q|^2 >= alpha max|Q|^2 > 0 (the positivity the paper states
right after the definition).

The statistic is (1 / (N m)) sum_k ||grad_k||_2 with m the probe side, the plain
(unsquared) 2-norm per position, and N the number of positions.  The worked example
uses m = 2 and flat patches, for which every transform is a single DC term.
"""

import numpy as np
import pytest

import oracle


def test_u_rpie_hand_values():
    Q = np.array([[2.0, 1j], [0.0, 1 + 1j]])
    # |Q|^2 = [[4, 1], [0, 2]], max 4
    u = oracle.u_rpie(Q, 0.3)
    np.testing.assert_allclose(u, [[0.0, 0.9], [1.2, 0.6]], rtol=0, atol=1e-15)
    w0 = u + np.abs(Q) ** 2
    np.testing.assert_allclose(w0, [[4.0, 1.9], [1.2, 2.6]], rtol=0, atol=1e-15)
    # the smallest precision alpha max|Q|^2 sits where Q = 0
    assert w0.min() == pytest.approx(0.3 * 4.0, abs=1e-15)
    assert np.argmin(w0) == 2


def test_u_rpie_scaling_and_limits(rng):
    m = 8
    Q = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
    u = oracle.u_rpie(Q, 0.7)
    A = np.abs(Q) ** 2
    assert u.min() == 0.0 and u[np.unravel_index(np.argmax(A), A.shape)] == 0.0
    assert np.all(u >= 0)
    # u(c Q) = |c|^2 u(Q); u is linear in alpha; alpha = 0 gives PIE's u = 0
    c = 0.3 - 1.7j
    np.testing.assert_allclose(oracle.u_rpie(c * Q, 0.7), abs(c) ** 2 * u, rtol=1e-13)
    np.testing.assert_allclose(oracle.u_rpie(Q, 1.4), 2 * u, rtol=1e-15)
    assert np.all(oracle.u_rpie(Q, 0.0) == 0)
    # positivity of the rPIE denominator for alpha > 0 even where Q vanishes
    Q[3, 4] = 0
    w0 = oracle.u_rpie(Q, 0.05) + np.abs(Q) ** 2
    assert w0.min() >= 0.05 * (np.abs(Q) ** 2).max() * (1 - 1e-15)


def _two_flat_patches():
    """2 x 4 object, probe Q = 1 (2 x 2), positions (0, 0) and (0, 2) that do not overlap.
    Patch 0 is 3 everywhere with sqrt(d) = 4 at DC (0 elsewhere): F(Q z_0) = 12 at DC, so
    R_0 = F^{-1}(4 delta) = 1 everywhere and grad_0 = 3 - 1 = 2 at each of 4 pixels:
    ||grad_0|| = 4.  Patch 1 is a = 5 e^{i pi/3} with sqrt(d) = 8 at DC: R_1 = 2 e^{i pi/3},
    grad_1 = 3 e^{i pi/3} per pixel, ||grad_1|| = 6."""
    a = 5 * np.exp(1j * np.pi / 3)
    z = np.array([[3, 3, a, a], [3, 3, a, a]], dtype=np.complex128)
    Q = np.ones((2, 2), dtype=np.complex128)
    offs = np.array([[0, 0], [0, 2]], dtype=np.int32)
    sd = np.zeros((2, 2, 2))
    sd[0, 0, 0] = 4.0
    sd[1, 0, 0] = 8.0
    return z, Q, offs, sd


def test_stopping_statistic_hand_example():
    z, Q, offs, sd = _two_flat_patches()
    g0 = oracle.grad_k(oracle.extract(z, offs[0], 2), Q, sd[0])
    g1 = oracle.grad_k(oracle.extract(z, offs[1], 2), Q, sd[1])
    np.testing.assert_allclose(g0, 2 * np.ones((2, 2)), atol=1e-14)
    np.testing.assert_allclose(g1, 3 * np.exp(1j * np.pi / 3) * np.ones((2, 2)), atol=1e-14)
    # (1 / (N m)) (4 + 6) with N = 2, m = 2; a squared norm would give 13, 1/(N m^2) 1.25
    assert oracle.stopping_statistic(z, Q, offs, sd) == pytest.approx(2.5, rel=1e-14)


def test_stopping_statistic_vanishes_at_noiseless_truth(rng):
    m, n = 8, 20
    z = np.exp(1j * rng.uniform(-1, 1, (n, n))) * (0.8 + 0.2 * rng.random((n, n)))
    Q = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
    offs = np.array([(r, c) for r in range(0, n - m + 1, 4) for c in range(0, n - m + 1, 4)], np.int32)
    sd = np.sqrt(oracle.forward_model(z, Q, offs))
    assert oracle.stopping_statistic(z, Q, offs, sd) <= 1e-13
    assert oracle.stopping_statistic(1.1 * z, Q, offs, sd) > 1e-3
