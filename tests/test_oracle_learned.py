"""Pins of the learned-start oracle (CPU only).

Each test checks the oracle against something other than itself: SciPy's
correlation, central finite differences, Adam's closed-form first steps, the
Fourier shift theorem, adjointness and exact identities of the pyramid.
"""

import numpy as np
import pytest
from scipy import signal

from oracle import learned as ol
from oracle import core as oc

CIN, WIDTH = 3, 4


def _params(rng, cin=CIN, width=WIDTH, scale=0.25):
    return rng.normal(0.0, scale, ol.n_params(cin, width))


def test_param_count_of_the_fixed_architecture():
    # 3 input channels, 32 wide: 896 + 3 * 9248 + 578
    assert ol.n_params(3, 32) == 29218
    assert ol.n_params(1, 32) == 32 * 9 + 32 + 3 * 9248 + 578


def test_conv_equals_scipy_correlation():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(2, 3, 7, 9))
    w = rng.normal(size=(5, 3, 3, 3))
    b = rng.normal(size=5)
    out = ol.conv3x3(x, w, b)
    for n in range(2):
        for o in range(5):
            ref = b[o] + sum(signal.correlate2d(x[n, c], w[o, c], mode="same", boundary="fill")
                             for c in range(3))
            assert np.allclose(out[n, o], ref, rtol=1e-13, atol=1e-13)


def test_conv_backward_is_adjoint_and_matches_finite_differences():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(2, 3, 5, 6))
    w = rng.normal(size=(4, 3, 3, 3))
    b = rng.normal(size=4)
    dout = rng.normal(size=(2, 4, 5, 6))
    dx, dw, db = ol.conv3x3_backward(x, w, dout)
    # linear in x: <conv(x) - b, dout> = <x, dx>
    lhs = ((ol.conv3x3(x, w, b) - b[None, :, None, None]) * dout).sum()
    assert np.isclose(lhs, (x * dx).sum(), rtol=1e-12)
    f = lambda ww, bb: (ol.conv3x3(x, ww, bb) * dout).sum()  # noqa: E731
    h = 1e-6
    for idx in [(0, 0, 0, 0), (3, 2, 1, 2), (1, 1, 2, 0)]:
        wp, wm = w.copy(), w.copy()
        wp[idx] += h
        wm[idx] -= h
        assert np.isclose((f(wp, b) - f(wm, b)) / (2 * h), dw[idx], rtol=1e-7)
    bp, bm = b.copy(), b.copy()
    bp[2] += h
    bm[2] -= h
    assert np.isclose((f(w, bp) - f(w, bm)) / (2 * h), db[2], rtol=1e-7)


def test_upsample_adjoint():
    rng = np.random.default_rng(3)
    a = rng.normal(size=(2, 3, 4, 5))
    d = rng.normal(size=(2, 3, 8, 10))
    assert np.isclose((ol.upsample2(a) * d).sum(), (a * ol.upsample2_backward(d)).sum(), rtol=1e-13)
    assert np.array_equal(ol.upsample2(a)[..., 1::2, 0::2], a)


def _loss(params, x, target, mask):
    y, _ = ol.net_forward(params, x, CIN, WIDTH)
    return ol.complex_mse(y, target, mask)[0]


def test_network_gradient_matches_finite_differences():
    rng = np.random.default_rng(4)
    p = _params(rng)
    x = rng.normal(size=(2, CIN, 4, 4))
    target = np.exp(1j * rng.uniform(-1, 1, (8, 8))) * rng.uniform(0.5, 1.0, (8, 8))
    mask = (rng.uniform(size=(8, 8)) > 0.2).astype(float)
    y, cache = ol.net_forward(p, x, CIN, WIDTH)
    loss, dy = ol.complex_mse(y, target, mask)
    g, dx = ol.net_backward(p, cache, dy, CIN, WIDTH)
    h = 1e-6
    idx = rng.choice(p.size, 40, replace=False)
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (_loss(pp, x, target, mask) - _loss(pm, x, target, mask)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i])) + 1e-9, (i, fd, g[i])
    for j in [(0, 0, 0, 0), (1, 2, 3, 1), (0, 1, 2, 2)]:
        xp, xm = x.copy(), x.copy()
        xp[j] += h
        xm[j] -= h
        fd = (_loss(p, xp, target, mask) - _loss(p, xm, target, mask)) / (2 * h)
        assert abs(fd - dx[j]) <= 1e-6 * max(1e-3, abs(dx[j])) + 1e-9


def test_complex_mse_value_and_gradient():
    rng = np.random.default_rng(5)
    y = rng.normal(0, 0.3, size=(3, 2, 4, 4))
    t = rng.normal(size=(4, 4)) + 1j * rng.normal(size=(4, 4))
    mask = np.ones((4, 4))
    mask[0, 0] = 0.0
    loss, dy = ol.complex_mse(y, t, mask)
    pred = np.exp(y[:, 0]) * (np.cos(y[:, 1]) + 1j * np.sin(y[:, 1]))
    direct = sum((np.abs(pred[n] - t) ** 2 * mask).sum() for n in range(3)) / (3 * mask.sum())
    assert np.isclose(loss, direct, rtol=1e-14)
    assert np.all(dy[:, :, 0, 0] == 0.0)
    h = 1e-7
    for j in [(0, 0, 1, 2), (2, 1, 3, 3), (1, 1, 0, 1)]:
        yp, ym = y.copy(), y.copy()
        yp[j] += h
        ym[j] -= h
        fd = (ol.complex_mse(yp, t, mask)[0] - ol.complex_mse(ym, t, mask)[0]) / (2 * h)
        assert np.isclose(fd, dy[j], rtol=1e-6, atol=1e-12)


def test_aligned_mse_is_phase_invariant_and_its_gradient_matches_finite_differences():
    rng = np.random.default_rng(10)
    y = rng.normal(0, 0.3, size=(2, 2, 5, 5))
    t = np.exp(1j * rng.uniform(-1, 1, (5, 5))) * rng.uniform(0.6, 1.0, (5, 5))
    mask = (rng.uniform(size=(5, 5)) > 0.3).astype(float)
    loss, dy = ol.complex_mse_aligned(y, t, mask)
    # a global phase added to the prediction changes nothing
    y2 = y.copy()
    y2[:, 1] += 1.234
    assert np.isclose(ol.complex_mse_aligned(y2, t, mask)[0], loss, rtol=1e-12)
    # the aligned loss is the minimum over a fine grid of global phases
    for n in range(2):
        one = y[n:n + 1]
        best = min(ol.complex_mse(one + np.array([0, ph])[None, :, None, None], t, mask)[0]
                   for ph in np.linspace(-np.pi, np.pi, 4001))
        got = ol.complex_mse_aligned(one, t, mask)[0]
        assert got <= best + 1e-12 and best - got < 1e-5
    h = 1e-6
    for j in [(0, 0, 1, 2), (1, 1, 3, 3), (1, 0, 0, 4), (0, 1, 2, 2)]:
        yp, ym = y.copy(), y.copy()
        yp[j] += h
        ym[j] -= h
        fd = (ol.complex_mse_aligned(yp, t, mask)[0] - ol.complex_mse_aligned(ym, t, mask)[0]) / (2 * h)
        assert np.isclose(fd, dy[j], rtol=1e-6, atol=1e-11)


def test_adam_first_steps_closed_form():
    rng = np.random.default_rng(6)
    p0 = rng.normal(size=50)
    g = rng.normal(size=50)
    lr, b1, b2, eps = 1e-3, 0.9, 0.999, 1e-8
    m = np.zeros(50)
    v = np.zeros(50)
    p1, m, v = ol.adam_step(p0, g, m, v, 1, lr, b1, b2, eps)
    # bias correction makes the first step lr * g / (|g| + eps)
    assert np.allclose(p1, p0 - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)
    # with a constant gradient every later step is the same size
    p2, m, v = ol.adam_step(p1, g, m, v, 2, lr, b1, b2, eps)
    assert np.allclose(p2 - p1, p1 - p0, rtol=1e-10, atol=1e-16)


def test_bf16_round_known_values():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 1e-3], dtype=np.float32)
    r = ol.bf16_round(x)
    assert r[0] == 1.0
    assert r[1] == 1.0                      # tie goes to even (mantissa 0)
    assert r[2] == 1.0 + 2 ** -7            # above the tie rounds up
    assert r[3] == -2.5
    assert abs(r[4] - 1e-3) <= 2 ** -9 * 1e-3


def test_position_stats_shift_theorem():
    """A phase ramp of f0 cycles per patch shifts the pattern by f0 bins (centre of mass moves by f0)."""
    m = 32
    yy, xx = np.mgrid[0:m, 0:m].astype(float)
    c = (m - 1) / 2
    Q = np.exp(-((yy - c) ** 2 + (xx - c) ** 2) / (2 * 3.0 ** 2)).astype(np.complex128)
    base = ol.position_stats(np.abs(oc.fft2(Q))[None], Q)[0]
    for fy, fx in [(2, -3), (-1, 5), (0, 0)]:
        z = np.exp(2j * np.pi * (fy * yy + fx * xx) / m)
        sd = np.abs(oc.fft2(Q * z))[None]
        st = ol.position_stats(sd, Q)[0]
        assert abs(st[1] - base[1] - fy) < 1e-9
        assert abs(st[2] - base[2] - fx) < 1e-9
        # Parseval: mean amplitude ratio is unchanged by a pure phase ramp
        assert abs(st[0] - base[0]) < 1e-12
    assert abs(base[1]) < 1e-9 and abs(base[2]) < 1e-9     # symmetric probe: centred pattern


def test_integrate_gradient_recovers_a_periodic_phase():
    """The spectral gradient of a periodic field integrates back to the field (minus its mean);
    a planted sign error or swapped axes fail."""
    S = 32
    yy, xx = np.mgrid[0:S, 0:S].astype(float)
    phi = np.sin(2 * np.pi * 2 * yy / S + 0.3) * np.cos(2 * np.pi * 3 * xx / S) + 0.5 * np.cos(2 * np.pi * xx / S)
    F = np.fft.fft2(phi)
    w = np.fft.fftfreq(S) * 2 * np.pi
    wy, wx = np.meshgrid(w, w, indexing="ij")
    gy = np.real(np.fft.ifft2(1j * wy * F))
    gx = np.real(np.fft.ifft2(1j * wx * F))
    rec = ol.integrate_gradient(gy, gx)
    assert np.allclose(rec, phi - phi.mean(), atol=1e-12)
    assert not np.allclose(ol.integrate_gradient(gx, gy), phi - phi.mean(), atol=1e-3)
    assert not np.allclose(ol.integrate_gradient(-gy, gx), phi - phi.mean(), atol=1e-3)
    # finite-difference gradients of a smooth field integrate to it within the discretisation error
    gyd = (np.roll(phi, -1, 0) - np.roll(phi, 1, 0)) / 2
    gxd = (np.roll(phi, -1, 1) - np.roll(phi, 1, 1)) / 2
    assert np.max(np.abs(ol.integrate_gradient(gyd, gxd) - (phi - phi.mean()))) < 0.08   # sin(w)/w attenuation


def test_input_map_phase_channel_integrates_the_centre_of_mass_channels():
    rng = np.random.default_rng(11)
    n, m = 64, 16
    Q = np.ones((m, m), dtype=np.complex128)
    offs = np.array([[r, c] for r in range(0, n - m + 1, 6) for c in range(0, n - m + 1, 6)], dtype=np.int32)
    sd = rng.uniform(0.5, 2.0, (len(offs), m, m))
    mp = ol.input_map(sd, Q, offs, n, n, 16)
    f = n // 16
    want = ol.integrate_gradient(mp[1] * 2 * np.pi * f / m, mp[2] * 2 * np.pi * f / m)
    assert mp.shape == (4, 16, 16)
    assert np.allclose(mp[3], want, atol=1e-13)


def test_input_map_constant_and_coverage():
    n, m = 64, 16
    Q = np.ones((m, m), dtype=np.complex128)         # flat probe
    offs = np.array([[r, c] for r in range(8, 40, 8) for c in range(8, 40, 8)], dtype=np.int32)
    sd = np.ones((len(offs), m, m)) * 3.0
    mp = ol.input_map(sd, Q, offs, n, n, 16)
    covered = ol.input_map(np.ones_like(sd), Q, offs, n, n, 16)[0] > 0
    # amplitude channel: mean sqrt(d) / ||Q|| = 3 / m on covered blocks, 0 on uncovered ones
    blk = np.zeros((n, n), bool)
    for r, c in offs:
        blk[r:r + m, c:c + m] = True
    full = blk.reshape(16, 4, 16, 4).all(axis=(1, 3))
    none = ~blk.reshape(16, 4, 16, 4).any(axis=(1, 3))
    assert np.allclose(mp[0][full], 3.0 / m, rtol=1e-14)
    assert np.all(mp[0][none] == 0.0) and np.all(covered == blk.reshape(16, 4, 16, 4).any(axis=(1, 3)))
    # counts only at zero frequency: both centre-of-mass channels vanish
    sdz = np.zeros_like(sd)
    sdz[:, 0, 0] = 1.0
    assert np.all(ol.input_map(sdz, Q, offs, n, n, 16)[1:] == 0.0)


def test_input_map_weighted_mean_of_two_positions():
    m = 4
    Q = np.array([[1, 2, 0, 1], [1, 1, 1, 1], [0.5, 1, 1, 2], [1, 1, 3, 1]], dtype=np.complex128)
    offs = np.array([[0, 0], [2, 2]], dtype=np.int32)
    sd = np.stack([np.full((m, m), 2.0), np.full((m, m), 4.0)])
    mp = ol.input_map(sd, Q, offs, 6, 6, 6)[:3]             # no pooling
    A = np.abs(Q) ** 2
    a = np.array([2.0, 4.0]) / np.sqrt(A.sum())
    # pixel (2,2): covered by Q[2,2] of position 0 and Q[0,0] of position 1
    want = (A[2, 2] * a[0] + A[0, 0] * a[1]) / (A[2, 2] + A[0, 0])
    assert np.isclose(mp[0, 2, 2], want, rtol=1e-14)
    assert mp[0, 5, 0] == 0.0


def test_pyramid_identities():
    rng = np.random.default_rng(8)
    z = rng.normal(size=(16, 16)) + 1j * rng.normal(size=(16, 16))
    zc = rng.normal(size=(4, 4)) + 1j * rng.normal(size=(4, 4))
    assert np.allclose(ol.restrict_object(ol.prolong_object(zc, 2), 2), zc, rtol=0, atol=1e-15)
    # restriction twice = 4 x 4 block mean
    assert np.allclose(ol.restrict_object(z, 2), z.reshape(4, 4, 4, 4).mean(axis=(1, 3)), atol=1e-15)
    # adjointness: <R z, c> = (1/16) <z, P c>
    assert np.isclose(np.vdot(ol.restrict_object(z, 2), zc), np.vdot(z, ol.prolong_object(zc, 2)) / 16,
                      rtol=1e-13)


@pytest.mark.parametrize("mistake", ["flip", "no_bias"])
def test_planted_conv_mistakes_are_caught(mistake):
    """A flipped kernel or a dropped bias in the convolution fails the SciPy pin."""
    rng = np.random.default_rng(9)
    x = rng.normal(size=(1, 2, 5, 5))
    w = rng.normal(size=(2, 2, 3, 3))
    b = rng.normal(size=2)
    if mistake == "flip":
        out = ol.conv3x3(x, w[:, :, ::-1, ::-1], b)
    else:
        out = ol.conv3x3(x, w, 0 * b)
    ref = b[0] + sum(signal.correlate2d(x[0, c], w[0, c], mode="same") for c in range(2))
    assert not np.allclose(out[0, 0], ref)
