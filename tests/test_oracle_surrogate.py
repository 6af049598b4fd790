"""Pins of the surrogate model (Section 3): Lemma C.1, Prop 3.1, Prop 3.2, Prop 3.3.

Prop 3.3 as printed, (1/L) sum_j ||grad Phi(z^(j))||^2 <= Phi(z^(0)), fails on a
one-pixel example (test below); its proof replaces (1/2) sum_k P_k^T grad Phi_k
by grad Phi.  Redoing the last step with the minimiser of the quadratic bound
gives Phi(z^(j)) - Phi(z^(j+1)) >= ||grad Phi(z^(j))||^2 / (4 L), i.e. the bound
with 4 L in place of L, which is what is pinned.
"""

import numpy as np
import pytest

import oracle
from helpers import crandn, random_probe, tiny_problem


def test_lemma_c1_pointwise(rng):
    x = crandn(rng, 2000)
    y = crandn(rng, 2000)
    d = rng.random(2000) * 3
    lhs = np.abs(x - d * np.exp(1j * np.angle(x))) ** 2
    rhs = np.abs(x - d * np.exp(1j * np.angle(y))) ** 2
    assert np.all(lhs <= rhs + 1e-12)
    # closed form of the left side: (|x| - d)^2
    np.testing.assert_allclose(lhs, (np.abs(x) - d) ** 2, atol=1e-12)


def test_prop31_majorisation(rng):
    z_true, Q, offs, sd = tiny_problem(rng, noiseless=False)
    n = z_true.shape[0]
    zj = z_true + 0.3 * crandn(rng, n, n)
    # agree at z^(j)
    assert np.isclose(oracle.objective(zj, Q, offs, sd), oracle.surrogate(zj, zj, Q, offs, sd), rtol=1e-13)
    # dominated everywhere
    for _ in range(5):
        z = zj + 0.5 * crandn(rng, n, n)
        assert oracle.objective(z, Q, offs, sd) <= oracle.surrogate(z, zj, Q, offs, sd) + 1e-12
    # gradients agree at z^(j): directional derivatives by central differences
    for _ in range(3):
        dirn = crandn(rng, n, n)
        h = 1e-6
        dphi = (oracle.objective(zj + h * dirn, Q, offs, sd) - oracle.objective(zj - h * dirn, Q, offs, sd)) / (2 * h)
        dsur = (oracle.surrogate(zj + h * dirn, zj, Q, offs, sd) - oracle.surrogate(zj - h * dirn, zj, Q, offs, sd)) / (2 * h)
        assert abs(dphi - dsur) <= 1e-6 * max(1.0, abs(dphi))


def test_prop32_monotone_full_batch(rng):
    """Exact minimisation of eq. (3.1) never increases Phi (Prop 3.2)."""
    z_true, Q, offs, sd = tiny_problem(rng, noiseless=False)
    n = z_true.shape[0]
    z = np.ones((n, n), dtype=complex)
    prev = oracle.objective(z, Q, offs, sd)
    for _ in range(15):
        z = oracle.full_batch_surrogate_minimiser(z, Q, offs, sd)
        cur = oracle.objective(z, Q, offs, sd)
        assert cur <= prev * (1 + 1e-12)
        prev = cur


def test_full_batch_minimiser_is_stationary_for_surrogate(rng):
    """The closed form is the minimiser of Phi~(.; z^(j)) with u = 0: directional derivative 0."""
    z_true, Q, offs, sd = tiny_problem(rng, noiseless=False)
    n = z_true.shape[0]
    zj = np.ones((n, n), dtype=complex)
    zp = oracle.full_batch_surrogate_minimiser(zj, Q, offs, sd)
    f = lambda v: oracle.surrogate(v, zj, Q, offs, sd)  # noqa: E731
    f0 = f(zp)
    for _ in range(4):
        dirn = crandn(rng, n, n)
        h = 1e-5
        dd = (f(zp + h * dirn) - f(zp - h * dirn)) / (2 * h)
        assert abs(dd) < 1e-6 * max(1.0, f0)
        assert f(zp + 1e-2 * dirn) >= f0


def test_prop33_printed_constant_fails_on_one_pixel():
    """m = n = 1, Q = 1, d = 1, z0 = 2: printed bound gives 2 <= 0.5 (false); 4L version holds with equality."""
    Q = np.ones((1, 1), dtype=complex)
    offs = np.zeros((1, 2), dtype=np.int32)
    sd = np.ones((1, 1, 1))
    z = np.full((1, 1), 2.0 + 0j)
    L = 0.5 * np.max(oracle.illumination(z.shape, Q, offs))
    phi0 = oracle.objective(z, Q, offs, sd)
    gs = []
    for _ in range(3):
        gs.append(np.linalg.norm(oracle.full_gradient(z, Q, offs, sd)) ** 2)
        z = oracle.full_batch_surrogate_minimiser(z, Q, offs, sd)
    printed = sum(gs) / L
    assert printed > phi0            # the printed inequality is violated
    assert np.isclose(sum(gs), 4 * L * phi0)  # the corrected bound is tight here


def test_prop33_sublinear_bound_corrected(rng):
    z_true, Q, offs, sd = tiny_problem(rng, noiseless=False)
    n = z_true.shape[0]
    z = np.ones((n, n), dtype=complex)
    L = 0.5 * np.max(oracle.illumination(z.shape, Q, offs))
    phi0 = oracle.objective(z, Q, offs, sd)
    acc = 0.0
    for j in range(25):
        phi = oracle.objective(z, Q, offs, sd)
        g2 = np.linalg.norm(oracle.full_gradient(z, Q, offs, sd)) ** 2
        znext = oracle.full_batch_surrogate_minimiser(z, Q, offs, sd)
        # per-step decrease bound
        assert phi - oracle.objective(znext, Q, offs, sd) >= g2 / (4 * L) * (1 - 1e-9)
        acc += g2
        z = znext
    assert acc <= 4 * L * phi0


def test_minibatch_L1_is_proximal_minimiser(rng):
    """L = 1: the minibatch step minimises sum_{k in B} Phi~_k + 1/2 u^T |z_k - z_k^(j)|^2 (eqs. 3.4-3.5)."""
    z_true, Q, offs, sd = tiny_problem(rng, noiseless=False)
    n = z_true.shape[0]
    u = oracle.u_rpie(Q, 0.3)
    zj = z_true + 0.4 * crandn(rng, n, n)
    batch = [0, 3, 4, 7, 8]
    m = Q.shape[0]

    def prox_obj(v):
        return sum(oracle.pie_surrogate_k(oracle.extract(v, offs[k], m), oracle.extract(zj, offs[k], m),
                                          Q, sd[k], u) for k in batch)

    zp = oracle.minibatch_step(zj, Q, offs, sd, u, 1, batch)
    f0 = prox_obj(zp)
    for _ in range(4):
        dirn = crandn(rng, n, n)
        h = 1e-5
        dd = (prox_obj(zp + h * dirn) - prox_obj(zp - h * dirn)) / (2 * h)
        assert abs(dd) < 1e-6 * max(1.0, f0)
    # and the minibatch partial objective does not increase
    part = lambda v: sum(oracle.phi_k(oracle.extract(v, offs[k], m), Q, sd[k]) for k in batch)  # noqa: E731
    assert part(zp) <= part(zj) + 1e-12


def test_full_batch_L1_u0_equals_closed_form(rng):
    """B = N, L = 1, u = 0: the minibatch combination is the closed-form minimiser of eq. (3.1)."""
    z_true, Q, offs, sd = tiny_problem(rng, noiseless=False)
    n = z_true.shape[0]
    z0 = z_true + 0.2 * crandn(rng, n, n)
    u = np.zeros(Q.shape)
    a = oracle.minibatch_step(z0, Q, offs, sd, u, 1, list(range(len(offs))))
    b = oracle.full_batch_surrogate_minimiser(z0, Q, offs, sd)
    np.testing.assert_allclose(a, b, atol=1e-12)
