"""Pins of the oracle's DFT, revised exit wave, objective and gradient.

Section 2.1 (forward model, eq. 2.1, Definition 2.1, eq. 2.2), Appendix A
(Parseval, F^{-1} = F^* / m^2) and Appendix B.1 (objective identity).
"""

import numpy as np
import pytest

import oracle
from helpers import crandn, random_probe


def brute_dft2(v):
    """O(m^4) double sum: X[a, b] = sum_{x, y} v[x, y] exp(-2 pi i (a x + b y) / m)."""
    m0, m1 = v.shape
    X = np.zeros((m0, m1), dtype=np.complex128)
    for a in range(m0):
        for b in range(m1):
            s = 0j
            for x in range(m0):
                for y in range(m1):
                    s += v[x, y] * np.exp(-2j * np.pi * (a * x / m0 + b * y / m1))
            X[a, b] = s
    return X


@pytest.mark.parametrize("m", [2, 4, 8])
def test_fft_matches_bruteforce_dft(rng, m):
    v = crandn(rng, m, m)
    np.testing.assert_allclose(oracle.fft2(v), brute_dft2(v), rtol=0, atol=1e-12 * m * m)


@pytest.mark.parametrize("m", [4, 8, 32])
def test_parseval_and_inverse(rng, m):
    v = crandn(rng, m, m)
    F = oracle.fft2(v)
    assert np.isclose(np.sum(np.abs(F) ** 2), m * m * np.sum(np.abs(v) ** 2), rtol=1e-13)
    # F^{-1} = F^* / m^2: the inverse equals the conjugate-kernel sum divided by m^2
    np.testing.assert_allclose(oracle.ifft2(F), v, atol=1e-13)
    np.testing.assert_allclose(oracle.ifft2(v), np.conj(oracle.fft2(np.conj(v))) / (m * m), atol=1e-14)


def test_revised_exit_wave_definition(rng):
    m = 8
    zk, Q = crandn(rng, m, m), random_probe(rng, m)
    sd = rng.random((m, m))
    R = oracle.revised_exit_wave(zk, Q, sd)
    FR = oracle.fft2(R)
    Psi = brute_dft2(Q * zk)
    # modulus of F(R) is sqrt(d); phase equals that of F(Q z_k)
    np.testing.assert_allclose(np.abs(FR), sd, atol=1e-12)
    np.testing.assert_allclose(FR * np.abs(Psi), sd * Psi, atol=1e-10)


def test_theta_zero_convention():
    # Psi = 0 at every frequency when Q z = 0: R = F^{-1}(sqrt d) (theta(0) = 0)
    m = 4
    sd = np.arange(m * m, dtype=float).reshape(m, m)
    R = oracle.revised_exit_wave(np.zeros((m, m)), np.ones((m, m)), sd)
    np.testing.assert_allclose(oracle.fft2(R), sd, atol=1e-12)


def test_objective_identity(rng):
    """1/2 ||Q z_k - R_k||^2 = (1 / (2 m^2)) || |F(Q z_k)| - sqrt(d_k) ||^2 (Appendix B.1)."""
    m, n = 8, 16
    z = crandn(rng, n, n)
    Q = random_probe(rng, m)
    offs = np.array([[0, 0], [4, 4], [8, 8], [8, 0]], dtype=np.int32)
    sd = rng.random((4, m, m)) * 3
    phi = oracle.objective(z, Q, offs, sd)
    amp = oracle.objective_amplitude(z, Q, offs, sd)
    assert np.isclose(phi, amp / (m * m), rtol=1e-12)
    # and with brute-force DFT for one patch
    zk = oracle.extract(z, offs[1], m)
    brute = 0.5 * np.sum((np.abs(brute_dft2(Q * zk)) - sd[1]) ** 2) / (m * m)
    assert np.isclose(oracle.phi_k(zk, Q, sd[1]), brute, rtol=1e-11)


def _fd_complex_grad(f, z, idx, h=1e-6):
    e = np.zeros_like(z)
    e[idx] = 1.0
    gx = (f(z + h * e) - f(z - h * e)) / (2 * h)
    gy = (f(z + 1j * h * e) - f(z - 1j * h * e)) / (2 * h)
    return gx + 1j * gy


def test_gradient_finite_differences(rng):
    """eq. (2.2): nabla Phi_k = conj(Q)(Q z_k - R_k(z_k)) vs central differences in x and y."""
    m = 8
    zk, Q = crandn(rng, m, m), random_probe(rng, m)
    sd = rng.random((m, m)) * 4
    g = oracle.grad_k(zk, Q, sd)
    f = lambda v: oracle.phi_k(v, Q, sd)  # noqa: E731
    for idx in [(0, 0), (3, 5), (7, 7), (4, 1)]:
        fd = _fd_complex_grad(f, zk, idx)
        assert abs(fd - g[idx]) <= 1e-6 * max(1.0, abs(g[idx])), (idx, fd, g[idx])


def test_full_gradient_finite_differences(rng):
    """nabla Phi(z) = sum_k P_k^T nabla Phi_k (Section 2.1), FD on the whole object."""
    m, n = 4, 10
    z = crandn(rng, n, n)
    Q = random_probe(rng, m)
    offs = np.array([[0, 0], [2, 3], [6, 6], [3, 0]], dtype=np.int32)
    sd = rng.random((4, m, m)) * 3
    g = oracle.full_gradient(z, Q, offs, sd)
    f = lambda v: oracle.objective(v, Q, offs, sd)  # noqa: E731
    for idx in [(2, 3), (3, 4), (9, 9), (0, 0), (5, 1)]:
        fd = _fd_complex_grad(f, z, idx)
        assert abs(fd - g[idx]) <= 1e-6 * max(1.0, abs(g[idx])), (idx, fd, g[idx])
    # pixels that no scan covers have zero gradient
    assert g[0, 9] == 0


def test_forward_model_is_squared_modulus(rng):
    m, n = 4, 8
    z = crandn(rng, n, n)
    Q = random_probe(rng, m)
    offs = np.array([[1, 2], [4, 4]], dtype=np.int32)
    d = oracle.forward_model(z, Q, offs)
    for k, (r, c) in enumerate(offs):
        np.testing.assert_allclose(d[k], np.abs(brute_dft2(Q * z[r:r + m, c:c + m])) ** 2, rtol=1e-11)
