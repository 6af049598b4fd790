"""Pins of the stochastic driver (Alg 1, Alg 3, Alg 4 and the minibatch reading).

* one position per minibatch == Alg 4 (sequential MAGPIE);
* one grid == Alg 1 (rPIE) with eq. (2.3);
* the truth (and any global phase of it) is a fixed point for noiseless data;
* near-truth starts converge on the 128 x 128 workload's geometry (noiseless);
* the library's splitmix64 permutation generator reproduces the published
  splitmix64 test vector and yields permutations;
* phase recycling (eq. 3.2): no effect without exact zeros, theta = 0 on the first
  visit, and recycled phases of a visit at the truth recover the truth from a zeroed
  patch (where theta = 0 does not).
"""

import os

import numpy as np
import pytest

import oracle
from helpers import crandn, tiny_problem

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_b1_minibatch_equals_alg4(rng):
    z_true, Q, offs, sd = tiny_problem(rng, n=20, m=8, step=3, noiseless=False)
    n = z_true.shape[0]
    u = oracle.u_rpie(Q, 0.5)
    z0 = z_true + 0.3 * crandn(rng, n, n)
    orders = [rng.permutation(len(offs)) for _ in range(2)]
    for L in (1, 2, 3):
        a = oracle.run_epochs(z0, Q, offs, sd, u, L, orders, 1)
        b = oracle.magpie_sequential(z0, Q, offs, sd, u, L, orders)
        np.testing.assert_allclose(a, b, atol=1e-12)


def test_one_level_is_rpie_alg1(rng):
    z_true, Q, offs, sd = tiny_problem(rng, n=20, m=8, step=3, noiseless=False)
    n = z_true.shape[0]
    z0 = z_true + 0.3 * crandn(rng, n, n)
    orders = [rng.permutation(len(offs)) for _ in range(2)]
    a = oracle.magpie_sequential(z0, Q, offs, sd, oracle.u_rpie(Q, 0.5), 1, orders)
    b = oracle.rpie_sequential(z0, Q, offs, sd, 0.5, orders)
    np.testing.assert_allclose(a, b, atol=1e-13)


def test_gradient_form_driver_equals_literal(rng):
    z_true, Q, offs, sd = tiny_problem(rng, n=24, m=8, step=4, noiseless=False)
    n = z_true.shape[0]
    u = oracle.u_rpie(Q, 0.5)
    z0 = z_true + 0.3 * crandn(rng, n, n)
    orders = [rng.permutation(len(offs))]
    for L in (1, 2, 3):
        a = oracle.run_epochs(z0, Q, offs, sd, u, L, orders, 4)
        b = oracle.run_epochs(z0, Q, offs, sd, u, L, orders, 4, use_gradient_form=True)
        np.testing.assert_allclose(a, b, atol=1e-12)


@pytest.mark.parametrize("L,B", [(1, 1), (2, 5), (3, 64)])
def test_truth_is_fixed_point(rng, L, B):
    z_true, Q, offs, sd = tiny_problem(rng, n=24, m=8, step=4)
    u = oracle.u_rpie(Q, 0.5)
    for phase in (0.0, 1.234):
        zs = z_true * np.exp(1j * phase)
        z1 = oracle.run_epochs(zs, Q, offs, sd, u, L, [rng.permutation(len(offs))], B)
        assert np.linalg.norm(z1 - zs) <= 1e-13 * np.linalg.norm(zs)


def _problem_128x128():
    from synth import WORKLOADS, make_problem_inputs
    cfg = WORKLOADS["128x128"]
    z_true, Q, offs, _, r_perm = make_problem_inputs(cfg)
    zt = z_true.astype(np.complex64).astype(np.complex128)
    Qf = Q.astype(np.complex64).astype(np.complex128)
    sd = np.sqrt(oracle.forward_model(zt, Qf, offs)).astype(np.float32).astype(np.float64)
    return cfg, zt, Qf, offs, sd, r_perm


@pytest.mark.slow
@pytest.mark.parametrize("L,B", [(1, 1), (2, 8), (3, 1)])
def test_recovery_near_truth_128x128(L, B):
    """Noiseless 128 x 128 workload from z* (1 + 0.05 CN(0,1)): the masked relative error falls >= 20x in 60 epochs."""
    cfg, zt, Q, offs, sd, r_perm = _problem_128x128()
    rng = np.random.default_rng(7)
    z0 = zt * (1 + 0.05 * (rng.standard_normal(zt.shape) + 1j * rng.standard_normal(zt.shape)) / np.sqrt(2))
    mask = oracle.illumination(zt.shape, Q, offs) >= 0.1 * oracle.illumination(zt.shape, Q, offs).max()
    e0 = oracle.error_relative(z0, zt, mask)
    orders = [r_perm.permutation(len(offs)) for _ in range(60)]
    z = oracle.run_epochs(z0, Q, offs, sd, oracle.u_rpie(Q, cfg.alpha), L, orders, B,
                          use_gradient_form=True)
    e1 = oracle.error_relative(z, zt, mask)
    assert e1 <= e0 / 20, (e0, e1)


def test_splitmix64_published_vector():
    with open(os.path.join(GOLDEN, "splitmix64_seed1234567.txt")) as f:
        want = [int(x) for x in f.read().split("\n") if x and not x.startswith("#")]
    gen = oracle.splitmix64(1234567)
    got = [next(gen) for _ in range(5)]
    assert got == want


def test_library_permutation_is_permutation():
    for n in (1, 2, 7, 64, 1600):
        p = oracle.library_permutation(42, 3, n)
        assert sorted(p.tolist()) == list(range(n))
    assert not np.array_equal(oracle.library_permutation(42, 0, 64), oracle.library_permutation(42, 1, 64))


def test_error_metrics():
    z = np.array([[1 + 0j, 2j], [3.0, 0.5]])
    mask = np.ones(z.shape, bool)
    assert oracle.error_relative(z * np.exp(0.7j), z, mask) < 1e-15
    assert np.isclose(oracle.error_paper(2 * z, z), np.linalg.norm(np.abs(z)))


# --------------------------------------------------------------------------
# Phase recycling, eq. (3.2)
# --------------------------------------------------------------------------
def test_phase_recycling_without_zeros_changes_nothing(rng):
    """Generic data never make F(Q z_k) vanish, so eq. (3.2) reduces to Definition 2.1."""
    z_true, Q, offs, sd = tiny_problem(rng, n=24, m=8, step=4, noiseless=False)
    u = oracle.u_rpie(Q, 0.5)
    z0 = z_true + 0.3 * crandn(rng, 24, 24)
    orders = [rng.permutation(len(offs)) for _ in range(2)]
    ph = oracle.initial_phases(len(offs), 8)
    a = oracle.run_epochs(z0, Q, offs, sd, u, 2, orders, 3, phases=ph)
    b = oracle.run_epochs(z0, Q, offs, sd, u, 2, orders, 3)
    np.testing.assert_array_equal(a, b)
    assert np.allclose(np.abs(ph), 1.0)


def test_phase_recycling_first_visit_is_theta_zero(rng):
    """j = 0: a vanishing exit wave takes theta = 0, as Definition 2.1's footnote."""
    m = 8
    Q = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
    sd = rng.random((1, m, m)) + 0.5
    zk = np.zeros((m, m), dtype=np.complex128)
    R0 = oracle.revised_exit_wave(zk, Q, sd[0])
    R1, ph = oracle.revised_exit_wave_recycled(zk, Q, sd[0], oracle.initial_phases(1, m)[0])
    np.testing.assert_array_equal(R0, R1)
    np.testing.assert_allclose(R1, oracle.ifft2(sd[0]), atol=1e-15)
    np.testing.assert_array_equal(ph, np.ones((m, m)))


def test_phase_recycling_recovers_truth_after_zeroing():
    """One position, noiseless data.  A visit at z* stores the phases of F(Q z*); zero the
    patch and visit again with one grid and u = 0: the recycled phases give back the true
    exit wave (|F(Q z*)| e^{i arg F(Q z*)} = F(Q z*)), so the update returns z* wherever Q is
    nonzero.  theta(0) = 0 instead leaves the real-valued F^{-1}(sqrt d) and misses z*."""
    rng = np.random.default_rng(32)
    m = 8
    Q = rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))
    z_true = (0.8 + 0.2 * rng.random((m, m))) * np.exp(1j * rng.uniform(-1.5, 1.5, (m, m)))
    offs = np.zeros((1, 2), dtype=np.int32)
    sd = np.sqrt(oracle.forward_model(z_true, Q, offs))
    u = np.zeros((m, m))
    ph = oracle.initial_phases(1, m)
    z1 = oracle.run_epochs(z_true, Q, offs, sd, u, 1, [[0]], 1, phases=ph)
    np.testing.assert_allclose(z1, z_true, atol=1e-13)            # z* is a fixed point
    z2 = oracle.run_epochs(np.zeros((m, m)), Q, offs, sd, u, 1, [[0]], 1, phases=ph)
    np.testing.assert_allclose(z2, z_true, atol=1e-12)
    z3 = oracle.run_epochs(np.zeros((m, m)), Q, offs, sd, u, 1, [[0]], 1)
    assert np.linalg.norm(z3 - z_true) > 0.1 * np.linalg.norm(z_true)
