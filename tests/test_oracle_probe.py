"""Pins of the probe step (beyond the paper: blind ptychography is named as
future work in its Conclusion).  For one minibatch the probe step is the exact
minimiser, in Q, of sum_k 1/2 ||Q z_k - R_k||^2 + 1/2 sum_k beta max|z_k|^2 |Q - Q^j|^2
with R_k = R_k(z_k; Q^j) fixed; hence it does not increase the minibatch's
partial objective (majorisation, Lemma C.1, applied in Q)."""

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
