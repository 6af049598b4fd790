"""Pins of the multigrid part (Section 4, Appendices E-I).

Lemma E.1-E.4 (restriction/prolongation), Prop 4.1 (weight bounds), Prop 4.2
(consistency), Thm 4.3 with eq. (4.6), Prop 4.4 (read as an inequality: the
proof equates I(1/w) with 1/I(w), which holds only when w = u + |Q|^2 is
constant on each bin; AM-HM gives <=), eq. (2.3) as the one-level case, and
the equality of Alg 3 with the gradient form the GPU evaluates.
"""

import numpy as np
import pytest

import oracle
from helpers import crandn, random_probe


def restriction_matrix(mh):
    """Eq. (2.5) written out: row (I, J) has 1/4 at fine (2I+a, 2J+b), a, b in {0, 1}."""
    mH = mh // 2
    Mx = np.zeros((mH * mH, mh * mh))
    for I in range(mH):
        for J in range(mH):
            for a in range(2):
                for b in range(2):
                    Mx[I * mH + J, (2 * I + a) * mh + (2 * J + b)] = 0.25
    return Mx


def test_restrict_prolong_match_matrices(rng):
    mh = 8
    Mx = restriction_matrix(mh)
    a = crandn(rng, mh, mh)
    np.testing.assert_allclose(oracle.restrict(a).ravel(), Mx @ a.ravel(), atol=1e-15)
    b = crandn(rng, mh // 2, mh // 2)
    np.testing.assert_allclose(oracle.prolong(b).ravel(), (4 * Mx.T) @ b.ravel(), atol=1e-15)


def test_lemma_e1_to_e4(rng):
    mh = 8
    A = crandn(rng, mh, mh)
    B = crandn(rng, mh // 2, mh // 2)
    # E.1: B * I A = I((I_H^h B) * A), and I_h^H I_H^h = Id
    np.testing.assert_allclose(B * oracle.restrict(A), oracle.restrict(oracle.prolong(B) * A), atol=1e-14)
    np.testing.assert_allclose(oracle.restrict(oracle.prolong(B)), B, atol=0)
    # E.2 / E.3: elementwise maps commute with prolongation
    C = crandn(rng, mh // 2, mh // 2)
    np.testing.assert_allclose(np.exp(oracle.prolong(B)), oracle.prolong(np.exp(B)), atol=1e-14)
    np.testing.assert_allclose(oracle.prolong(B) * oracle.prolong(C), oracle.prolong(B * C), atol=1e-14)
    # E.4: operator norms
    Mx = restriction_matrix(mh)
    assert np.isclose(np.linalg.norm(Mx, 2), 0.5)
    assert np.isclose(np.linalg.norm(4 * Mx.T, 2), 2.0)
    assert np.isclose(np.linalg.norm(Mx, np.inf), 1.0)
    assert np.isclose(np.linalg.norm(4 * Mx.T, np.inf), 1.0)


@pytest.mark.parametrize("zeros", [False, True])
def test_prop41_weight_bounds(rng, zeros):
    for _ in range(20):
        Q = random_probe(rng, 16, zeros=zeros)
        QH, Wz, WR, Wu = oracle.weights(Q)
        S = oracle.restrict(np.abs(Q) ** 2)
        # I_h^H W_z = J on bins with nonzero illumination
        IWz = oracle.restrict(Wz)
        np.testing.assert_allclose(IWz[S > 0], 1.0, atol=1e-14)
        assert Wz.min() >= 0 and Wz.max() <= 4 + 1e-14
        assert np.abs(WR).max() <= 1.5 + 1e-14      # the sharp bound stated after Prop 4.1
        assert Wu.min() >= 0 and Wu.max() <= 1 + 1e-14


def test_wr_sharp_bound_attained():
    """A bin (3, 1, 1, 1) attains |W_R| = 3/2 at the bright pixel."""
    Q = np.array([[3.0, 1.0], [1.0, 1.0]], dtype=complex)
    _, _, WR, _ = oracle.weights(Q)
    assert np.isclose(np.abs(WR[0, 0]), 1.5)


def test_weights_cancelled_form_equals_printed(rng):
    Q = random_probe(rng, 16)
    for a, b in zip(oracle.weights(Q), oracle.weights_literal(Q)):
        np.testing.assert_allclose(a, b, rtol=1e-13, atol=1e-15)


def test_prop42_consistency(rng):
    m = 16
    for _ in range(10):
        Q = random_probe(rng, m)
        z = crandn(rng, m, m)
        R = crandn(rng, m, m)
        QH, Wz, WR, Wu = oracle.weights(Q)
        zH = oracle.restrict(Wz * z)
        RH = oracle.restrict(WR * R)
        phiH = 0.5 * np.sum(np.abs(QH * zH - RH) ** 2)
        phi = 0.5 * np.sum(np.abs(Q * z - R) ** 2)
        assert phiH <= 0.25 * np.abs(WR).max() ** 2 * phi * (1 + 1e-12)
        gH = np.conj(QH) * (QH * zH - RH)
        g = np.conj(Q) * (Q * z - R)
        assert np.linalg.norm(gH) <= 0.5 * Wu.max() * np.linalg.norm(g) * (1 + 1e-12)


def test_thm43_closed_form_and_descent(rng):
    m = 16
    for _ in range(10):
        Q = random_probe(rng, m)
        u = oracle.u_rpie(Q, rng.uniform(0.05, 1.0))
        zp = crandn(rng, m, m)
        R = crandn(rng, m, m)
        QH, Wz, WR, Wu = oracle.weights(Q)
        zH = oracle.restrict(Wz * zp)
        RH = oracle.restrict(WR * R)
        uH = Wu * oracle.restrict(u)
        # coarse proximal step (eq. 4.5) as the one-level MAGPS on the coarse grid
        eH = oracle.magps(zH, QH, RH, uH, 1) - zH
        g = np.conj(Q) * (Q * zp - R)
        S = oracle.restrict(np.abs(Q) ** 2)
        eq46 = -(np.abs(QH) ** 2) / S / (uH + np.abs(QH) ** 2) * oracle.restrict(g)
        np.testing.assert_allclose(eH, eq46, rtol=1e-12, atol=1e-14)
        # descent direction: Re <g, I_H^h e_H> <= 0
        assert np.real(np.vdot(g, oracle.prolong(eH))) <= 1e-12


def test_prop44_inequality(rng):
    m = 16
    for _ in range(10):
        Q = random_probe(rng, m)
        u = oracle.u_rpie(Q, rng.uniform(0.05, 1.0))
        w = u + np.abs(Q) ** 2
        QH, _, _, Wu = oracle.weights(Q)
        uH = Wu * oracle.restrict(u)
        S = oracle.restrict(np.abs(Q) ** 2)
        coarse = 1.0 / (uH + np.abs(QH) ** 2) * np.abs(QH) ** 2 / S     # max |e_H(g)|_r
        fine = oracle.restrict(1.0 / w)                                  # max |I e_k(g)|_r
        assert np.all(coarse <= fine * (1 + 1e-12))
    # equality when w is constant on each bin (a bin-constant probe)
    Qc = oracle.prolong(crandn(rng, m // 2, m // 2))
    u = oracle.u_rpie(Qc, 0.3)
    w = u + np.abs(Qc) ** 2
    QH, _, _, Wu = oracle.weights(Qc)
    uH = Wu * oracle.restrict(u)
    S = oracle.restrict(np.abs(Qc) ** 2)
    np.testing.assert_allclose(np.abs(QH) ** 2 / S / (uH + np.abs(QH) ** 2), oracle.restrict(1.0 / w), rtol=1e-12)


def test_one_level_is_rpie(rng):
    """Alg 3 with a single grid is the rPIE update eq. (2.3)."""
    m = 16
    Q = random_probe(rng, m)
    u = oracle.u_rpie(Q, 0.2)
    z, R = crandn(rng, m, m), crandn(rng, m, m)
    expect = z + np.conj(Q) / (u + np.abs(Q) ** 2) * (R - Q * z)
    np.testing.assert_allclose(oracle.magps(z, Q, R, u, 1), expect, atol=1e-14)


def test_two_level_matches_section_41(rng):
    """Two-level MAGPS written as Section 4.1 prints it: coarse prox step, prolong, fine prox step."""
    m = 16
    Q = random_probe(rng, m)
    u = oracle.u_rpie(Q, 0.4)
    z, R = crandn(rng, m, m), crandn(rng, m, m)
    QH, Wz, WR, Wu = oracle.weights_literal(Q)
    zH = oracle.restrict(Wz * z)
    RH = oracle.restrict(WR * R)
    uH = Wu * oracle.restrict(u)
    zH_hat = zH + np.conj(QH) / (uH + np.abs(QH) ** 2) * (RH - QH * zH)
    zt = z + oracle.prolong(zH_hat - zH)
    zp = zt + np.conj(Q) / (u + np.abs(Q) ** 2) * (R - Q * zt)
    np.testing.assert_allclose(oracle.magps(z, Q, R, u, 2), zp, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("levels", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("probe", ["random", "zeros", "synthetic"])
def test_gradient_form_equals_alg3(rng, levels, probe):
    from synth import make_probe
    m = 32
    if probe == "synthetic":
        Q = make_probe(m)
    else:
        Q = random_probe(rng, m, zeros=(probe == "zeros"))
    u = oracle.u_rpie(Q, rng.uniform(0.05, 1.0))
    w0 = u + np.abs(Q) ** 2
    consts = oracle.level_constants(Q, u, levels)
    for _ in range(3):
        z, R = crandn(rng, m, m), crandn(rng, m, m)
        lit = w0 * (oracle.magps(z, Q, R, u, levels) - z)
        gf = oracle.magps_gradient_form(z, Q, R, consts)
        scale = np.abs(lit).max()
        np.testing.assert_allclose(gf, lit, rtol=0, atol=1e-12 * scale)


def test_two_level_step_lowers_patch_objective(rng):
    """L = 2: Phi~_k(z + dz) <= Phi~_k(z) and Phi_k(z^+) <= Phi_k(z) for one patch."""
    from synth import make_probe
    m = 32
    Q = make_probe(m)
    for _ in range(10):
        z_true = crandn(rng, m, m)
        sd = np.abs(oracle.fft2(Q * z_true)) * (1 + 0.05 * rng.random((m, m)))
        z = z_true + 0.7 * crandn(rng, m, m)
        u = oracle.u_rpie(Q, rng.uniform(0.05, 1.0))
        R = oracle.revised_exit_wave(z, Q, sd)
        zp = oracle.magps(z, Q, R, u, 2)
        assert oracle.surrogate_k(zp, z, Q, sd) <= oracle.surrogate_k(z, z, Q, sd) + 1e-12
        assert oracle.phi_k(zp, Q, sd) <= oracle.phi_k(z, Q, sd) + 1e-12


def test_deepest_level_is_scalar():
    """With log2(m)+1 grids the coarsest grid of the patch is a single value (Section 5 cost remark)."""
    m = 16
    Q = np.ones((m, m), dtype=complex)
    consts = oracle.level_constants(Q, oracle.u_rpie(Q, 0.1), 5)
    assert consts["levels"][-1][0].shape == (1, 1)
