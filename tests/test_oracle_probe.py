"""Pins of the probe step (beyond the paper: blind ptychography is named as
future work in its Conclusion).  For one minibatch the probe step is the exact
minimiser, in Q, of sum_k 1/2 ||Q z_k - R_k||^2 + 1/2 sum_k beta max|z_k|^2 |Q - Q^j|^2
with R_k = R_k(z_k; Q^j) fixed; hence it does not increase the minibatch's
partial objective (majorisation, Lemma C.1, applied in Q).  Taken alternately
after the object step (at the new object), both half steps keep the minibatch's
partial objective from increasing with one grid.  With the probe unknown, z is
determined only up to a complex scale: the scaled error removes it."""

import numpy as np

import oracle
from helpers import crandn, tiny_problem


def test_probe_step_is_proximal_minimiser(rng):
    z_true, Q, offs, sd = tiny_problem(rng, noiseless=False)
    m = Q.shape[0]
    n = z_true.shape[0]
    z = z_true + 0.2 * crandn(rng, n, n)
    Qj = Q * (1 + 0.2 * crandn(rng, m, m))
    batch = [0, 2, 5, 7]
    beta = 0.3
    Qn = oracle.probe_update_step(z, Qj, offs, sd, batch, beta)
    R = {k: oracle.revised_exit_wave(oracle.extract(z, offs[k], m), Qj, sd[k]) for k in batch}
    mx = sum(np.max(np.abs(oracle.extract(z, offs[k], m)) ** 2) for k in batch)

    def f(Qv):
        tot = 0.5 * beta * mx * np.sum(np.abs(Qv - Qj) ** 2)
        for k in batch:
            tot += 0.5 * np.sum(np.abs(Qv * oracle.extract(z, offs[k], m) - R[k]) ** 2)
        return tot

    f0 = f(Qn)
    for _ in range(4):
        dirn = crandn(rng, m, m)
        h = 1e-5
        dd = (f(Qn + h * dirn) - f(Qn - h * dirn)) / (2 * h)
        assert abs(dd) < 1e-6 * max(1.0, f0)
        assert f(Qn + 1e-2 * dirn) >= f0
    part = lambda QQ: sum(oracle.phi_k(oracle.extract(z, offs[k], m), QQ, sd[k]) for k in batch)  # noqa: E731
    assert part(Qn) <= part(Qj) + 1e-12


def test_probe_fixed_point_at_truth(rng):
    z_true, Q, offs, sd = tiny_problem(rng)
    Qn = oracle.probe_update_step(z_true, Q, offs, sd, list(range(len(offs))), 0.5)
    assert np.linalg.norm(Qn - Q) <= 1e-12 * np.linalg.norm(Q)


def test_blind_step_keeps_truth(rng):
    z_true, Q, offs, sd = tiny_problem(rng)
    z, Qn = oracle.run_epochs_blind(z_true, Q, offs, sd, 0.5, 2, [rng.permutation(len(offs))], 4, 0.5)
    assert np.linalg.norm(z - z_true) <= 1e-12 * np.linalg.norm(z_true)
    assert np.linalg.norm(Qn - Q) <= 1e-12 * np.linalg.norm(Q)


def test_alternating_steps_never_raise_the_minibatch_objective(rng):
    """One grid, noisy data: the object half step (proximal minimiser of the minibatch
    surrogate in z) and then the probe half step at the new object (the same in Q) each
    keep sum_{k in B} Phi_k from increasing."""
    z_true, Q, offs, sd = tiny_problem(rng, noiseless=False)
    m = Q.shape[0]
    n = z_true.shape[0]
    z = z_true + 0.3 * crandn(rng, n, n)
    Qj = Q * (1 + 0.2 * crandn(rng, m, m))
    part = lambda zz, QQ, B: sum(oracle.phi_k(oracle.extract(zz, offs[k], m), QQ, sd[k]) for k in B)  # noqa: E731
    for _ in range(6):
        B = list(rng.choice(len(offs), 4, replace=False))
        u = oracle.u_rpie(Qj, 0.5)
        zn = oracle.minibatch_step(z, Qj, offs, sd, u, 1, B)
        zn2, Qn = oracle.blind_minibatch_step(z, Qj, offs, sd, 0.5, 1, B, 0.3, alternate=True)
        np.testing.assert_array_equal(zn, zn2)
        assert part(zn, Qj, B) <= part(z, Qj, B) + 1e-12
        assert part(zn, Qn, B) <= part(zn, Qj, B) + 1e-12
        z, Qj = zn, Qn


def test_alternating_probe_step_uses_the_new_object(rng):
    """The alternating probe step equals probe_update_step at the updated object, and it
    differs from the simultaneous one (which uses the old object)."""
    z_true, Q, offs, sd = tiny_problem(rng, noiseless=False)
    n = z_true.shape[0]
    z = z_true + 0.3 * crandn(rng, n, n)
    B = [1, 3, 4]
    zn, Qa = oracle.blind_minibatch_step(z, Q, offs, sd, 0.5, 2, B, 0.2, alternate=True)
    _, Qs = oracle.blind_minibatch_step(z, Q, offs, sd, 0.5, 2, B, 0.2)
    np.testing.assert_array_equal(Qa, oracle.probe_update_step(zn, Q, offs, sd, B, 0.2))
    assert np.linalg.norm(Qa - Qs) > 1e-3 * np.linalg.norm(Q)


def test_alternating_blind_keeps_truth(rng):
    z_true, Q, offs, sd = tiny_problem(rng)
    z, Qn = oracle.run_epochs_blind(z_true, Q, offs, sd, 0.5, 3, [rng.permutation(len(offs))], 4, 0.5,
                                    alternate=True)
    assert np.linalg.norm(z - z_true) <= 1e-12 * np.linalg.norm(z_true)
    assert np.linalg.norm(Qn - Q) <= 1e-12 * np.linalg.norm(Q)


def test_scaled_error_removes_the_blind_ambiguity(rng):
    """(c z, Q / c) give the same data: the scaled error is 0 for any complex multiple of
    the truth, never exceeds the phase-only error, and sees a genuine difference."""
    z_true, Q, offs, sd = tiny_problem(rng)
    mask = np.ones(z_true.shape, bool)
    c = 0.7 * np.exp(0.4j)
    np.testing.assert_allclose(oracle.forward_model(c * z_true, Q / c, offs), sd ** 2, rtol=1e-12)
    assert oracle.error_scaled(c * z_true, z_true, mask) < 1e-14
    assert oracle.error_relative(c * z_true, z_true, mask) > 0.29
    zb = z_true + 0.1 * crandn(rng, *z_true.shape)
    assert 0 < oracle.error_scaled(zb, z_true, mask) <= oracle.error_relative(zb, z_true, mask) + 1e-15
