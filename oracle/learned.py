"""FP64 oracle of the learned start (coarse-object CNN) -- TEST INFRASTRUCTURE ONLY.

The paper starts Alg 4 from an unspecified initial guess and ends with
multigrid ideas for later work; a learned starting guess is beyond it.  What
this module fixes is therefore a definition written from first principles, with
the paper's own pieces where they apply:

* the object pyramid uses the paper's restriction (2x2 average pooling,
  eq. 2.5) and prolongation (copy into the 2x2 bin, eq. 2.6), applied to the
  whole object with bins aligned to pixel 0;
* the network input is built from the measured intensities d_k of Section 2.1
  only: per position k the mean measured amplitude a_k and the centre of mass
  (first moment) of d_k over signed frequency indices, spread back over the
  object with illumination weights |Q(p - o_k)|^2 and average-pooled, plus the
  phase that the centre-of-mass field (a phase gradient) integrates to;
* the network is five 3x3 convolutions (zero padding 1): Cin -> W, ReLU,
  W -> W, ReLU, nearest 2x upsampling, W -> W, ReLU, W -> W, ReLU, W -> 2.
  The two output channels are log-amplitude and phase of the coarse object;
* the loss is the masked complex mean squared error between exp(y0 + i y1)
  and the target coarse object, optionally after removing each sample's
  global phase (the objective of eq. 2.1 does not see it); Adam (Kingma and Ba, 2015) with bias
  correction updates the parameters.

Parity pins (tests/test_oracle_learned.py): the convolution against SciPy's
2-D correlation, all gradients against central finite differences, the Adam
step against its closed form on the first steps, the up/down-sampling
adjointness, the input map on a constant field and a pure phase ramp (Fourier
shift theorem), and restriction/prolongation identities.  The learned start as
a whole has no paper pin.

Parameter layout (flat float vector): for each layer l = 1..5 the weights
W_l[co][ci][ky][kx] followed by the bias b_l[co].
"""

from __future__ import annotations

import numpy as np

from .core import prolong, restrict

__all__ = [
    "layer_shapes", "n_params", "unpack", "conv3x3", "conv3x3_backward", "relu", "upsample2",
    "upsample2_backward", "net_forward", "net_backward", "complex_mse", "complex_mse_aligned", "adam_step",
    "bf16_round",
    "position_stats", "integrate_gradient", "input_map", "restrict_object", "prolong_object",
]


# --------------------------------------------------------------------------
# Parameters
# --------------------------------------------------------------------------
def layer_shapes(cin: int, width: int):
    """(co, ci) of the five convolutions."""
    return [(width, cin), (width, width), (width, width), (width, width), (2, width)]


def n_params(cin: int, width: int) -> int:
    return sum(co * ci * 9 + co for co, ci in layer_shapes(cin, width))


def unpack(params, cin: int, width: int):
    """[(W [co, ci, 3, 3], b [co]) per layer] views of the flat parameter vector."""
    p = np.asarray(params, dtype=np.float64)
    out, off = [], 0
    for co, ci in layer_shapes(cin, width):
        w = p[off:off + co * ci * 9].reshape(co, ci, 3, 3)
        off += co * ci * 9
        b = p[off:off + co]
        off += co
        out.append((w, b))
    assert off == p.size
    return out


# --------------------------------------------------------------------------
# Layers
# --------------------------------------------------------------------------
def conv3x3(x, w, b):
    """out[n, o, y, x] = b[o] + sum_{c, dy, dx} w[o, c, dy + 1, dx + 1] * x[n, c, y + dy, x + dx], zero outside."""
    N, C, H, W = x.shape
    xp = np.zeros((N, C, H + 2, W + 2))
    xp[:, :, 1:-1, 1:-1] = x
    out = np.zeros((N, w.shape[0], H, W)) + np.asarray(b)[None, :, None, None]
    for ky in range(3):
        for kx in range(3):
            out += np.einsum("oc,nchw->nohw", w[:, :, ky, kx], xp[:, :, ky:ky + H, kx:kx + W])
    return out


def conv3x3_backward(x, w, dout):
    """Gradients (dx, dw, db) of sum(dout * conv3x3(x, w, b))."""
    N, C, H, W = x.shape
    xp = np.zeros((N, C, H + 2, W + 2))
    xp[:, :, 1:-1, 1:-1] = x
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for ky in range(3):
        for kx in range(3):
            dw[:, :, ky, kx] = np.einsum("nohw,nchw->oc", dout, xp[:, :, ky:ky + H, kx:kx + W])
            dxp[:, :, ky:ky + H, kx:kx + W] += np.einsum("oc,nohw->nchw", w[:, :, ky, kx], dout)
    db = dout.sum(axis=(0, 2, 3))
    return dxp[:, :, 1:-1, 1:-1], dw, db


def relu(x):
    return np.maximum(x, 0.0)


def upsample2(x):
    """Nearest-neighbour 2x upsampling of the last two axes."""
    return np.repeat(np.repeat(x, 2, axis=-2), 2, axis=-1)


def upsample2_backward(d):
    """Adjoint of upsample2: sum over each 2x2 block."""
    return d[..., 0::2, 0::2] + d[..., 1::2, 0::2] + d[..., 0::2, 1::2] + d[..., 1::2, 1::2]


# --------------------------------------------------------------------------
# Network
# --------------------------------------------------------------------------
def net_forward(params, x, cin: int, width: int):
    """y = conv5(relu(conv4(relu(conv3(up(relu(conv2(relu(conv1(x)))))))))); returns (y, cache)."""
    L = unpack(params, cin, width)
    a0 = np.asarray(x, dtype=np.float64)
    a1 = relu(conv3x3(a0, *L[0]))
    a2 = relu(conv3x3(a1, *L[1]))
    u = upsample2(a2)
    a3 = relu(conv3x3(u, *L[2]))
    a4 = relu(conv3x3(a3, *L[3]))
    y = conv3x3(a4, *L[4])
    return y, (a0, a1, a2, u, a3, a4)


def net_backward(params, cache, dy, cin: int, width: int):
    """Flat gradient of sum(dy * y) with respect to the parameters, and dL/dx."""
    L = unpack(params, cin, width)
    a0, a1, a2, u, a3, a4 = cache
    grads = [None] * 5
    da4, dw, db = conv3x3_backward(a4, L[4][0], dy)
    grads[4] = (dw, db)
    dp4 = da4 * (a4 > 0)
    da3, dw, db = conv3x3_backward(a3, L[3][0], dp4)
    grads[3] = (dw, db)
    dp3 = da3 * (a3 > 0)
    du, dw, db = conv3x3_backward(u, L[2][0], dp3)
    grads[2] = (dw, db)
    dp2 = upsample2_backward(du) * (a2 > 0)
    da1, dw, db = conv3x3_backward(a1, L[1][0], dp2)
    grads[1] = (dw, db)
    dp1 = da1 * (a1 > 0)
    dx, dw, db = conv3x3_backward(a0, L[0][0], dp1)
    grads[0] = (dw, db)
    flat = np.concatenate([np.concatenate([g[0].ravel(), g[1].ravel()]) for g in grads])
    return flat, dx


def complex_mse(y, target, mask):
    """Masked complex MSE of the coarse object exp(y0 + i y1) against target; returns (loss, dL/dy).

    loss = sum_n sum_p mask(p) |exp(y0 + i y1) - t|^2 / (N sum_p mask(p)).
    """
    y = np.asarray(y, dtype=np.float64)
    N = y.shape[0]
    pred = np.exp(y[:, 0] + 1j * y[:, 1])
    r = pred - np.asarray(target, dtype=np.complex128)
    msk = np.asarray(mask, dtype=np.float64)[None]
    norm = N * msk.sum()
    loss = float((msk * np.abs(r) ** 2).sum() / norm)
    g = np.conj(r) * pred                     # d|r|^2 = 2 Re(conj(r) dpred)
    dy = np.empty_like(y)
    dy[:, 0] = 2.0 * msk * np.real(g) / norm             # dpred / dy0 = pred
    dy[:, 1] = -2.0 * msk * np.imag(g) / norm            # dpred / dy1 = i pred
    return loss, dy


def complex_mse_aligned(y, target, mask):
    """complex_mse after removing each sample's global phase: pred is rotated by
    exp(i phi_n), phi_n = arg sum_p mask conj(pred) t (the minimiser over phi), so
    loss = sum_n min_phi sum_p mask |exp(i phi) pred - t|^2 / (N sum_p mask).
    By the envelope theorem the gradient is that of the rotated residual with
    phi_n held fixed.  Returns (loss, dL/dy)."""
    y = np.asarray(y, dtype=np.float64)
    N = y.shape[0]
    pred = np.exp(y[:, 0] + 1j * y[:, 1])
    t = np.asarray(target, dtype=np.complex128)
    msk = np.asarray(mask, dtype=np.float64)[None]
    ip = (msk * np.conj(pred) * t).sum(axis=(1, 2))
    rot = np.where(np.abs(ip) > 0, ip / np.where(np.abs(ip) > 0, np.abs(ip), 1.0), 1.0)
    pr = pred * rot[:, None, None]
    r = pr - t
    norm = N * msk.sum()
    loss = float((msk * np.abs(r) ** 2).sum() / norm)
    g = np.conj(r) * pr
    dy = np.empty_like(y)
    dy[:, 0] = 2.0 * msk * np.real(g) / norm
    dy[:, 1] = -2.0 * msk * np.imag(g) / norm
    return loss, dy


def adam_step(p, g, m, v, t: int, lr: float, b1: float, b2: float, eps: float):
    """One Adam update (bias-corrected, step count t >= 1); returns new (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def bf16_round(x):
    """Round float32 values to the nearest bfloat16 (ties to even), returned as float64."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


# --------------------------------------------------------------------------
# Input map from measured intensities (Section 2.1 data only)
# --------------------------------------------------------------------------
def position_stats(sqrt_d, Q):
    """Per position: (mean_r sqrt(d_k) / ||Q||_2, row-frequency and column-frequency centre of mass of d_k).

    Frequencies are the signed DFT indices r for r < m/2 and r - m otherwise; a
    pattern with no counts has centre of mass 0.
    """
    sd = np.asarray(sqrt_d, dtype=np.float64)
    m = sd.shape[-1]
    f = np.arange(m, dtype=np.float64)
    f[f >= m // 2] -= m
    qn = np.sqrt((np.abs(Q) ** 2).sum())
    out = np.zeros((sd.shape[0], 3))
    for k in range(sd.shape[0]):
        d = sd[k] ** 2
        tot = d.sum()
        out[k, 0] = sd[k].mean() / qn
        if tot > 0:
            out[k, 1] = (d.sum(axis=1) * f).sum() / tot
            out[k, 2] = (d.sum(axis=0) * f).sum() / tot
    return out


def integrate_gradient(gy, gx):
    """Least-squares integration of a periodic gradient field (Frankot and Chellappa, 1988):
    phi = Re F^-1[ -i (w_y G_y + w_x G_x) / (w_y^2 + w_x^2) ], mean 0, with w the angular
    frequencies 2 pi f / S of the S x S grid (signed indices f).  Exact for the spectral
    gradient of a periodic field."""
    gy = np.asarray(gy, dtype=np.float64)
    gx = np.asarray(gx, dtype=np.float64)
    S0, S1 = gy.shape
    f0 = np.fft.fftfreq(S0) * 2 * np.pi
    f1 = np.fft.fftfreq(S1) * 2 * np.pi
    wy, wx = np.meshgrid(f0, f1, indexing="ij")
    den = wy ** 2 + wx ** 2
    num = -1j * (wy * np.fft.fft2(gy) + wx * np.fft.fft2(gx))
    out = np.zeros_like(num)
    nz = den > 0
    out[nz] = num[nz] / den[nz]
    return np.real(np.fft.ifft2(out))


def input_map(sqrt_d, Q, offsets, n_rows: int, n_cols: int, side: int):
    """4 x side x side network input: each channel of position_stats spread over the object with
    weights |Q(p - o_k)|^2 (normalised per pixel; 0 where no position covers p), then averaged
    over (n_rows / side) x (n_cols / side) blocks; channel 3 is the phase whose gradient the two
    centre-of-mass channels measure, integrated over the whole map (a centre of mass of f bins
    is a phase slope of 2 pi f / m per object pixel, i.e. 2 pi f (n / side) / m per map cell)."""
    st = position_stats(sqrt_d, Q)
    m = Q.shape[0]
    A = np.abs(Q) ** 2
    num = np.zeros((3, n_rows, n_cols))
    den = np.zeros((n_rows, n_cols))
    for k, (r, c) in enumerate(np.asarray(offsets)):
        den[r:r + m, c:c + m] += A
        for ch in range(3):
            num[ch, r:r + m, c:c + m] += A * st[k, ch]
    fine = np.zeros_like(num)
    pos = den > 0
    for ch in range(3):
        fine[ch][pos] = num[ch][pos] / den[pos]
    fr, fc = n_rows // side, n_cols // side
    pooled = fine.reshape(3, side, fr, side, fc).mean(axis=(2, 4))
    ph = integrate_gradient(pooled[1] * (2 * np.pi * fr / m), pooled[2] * (2 * np.pi * fc / m))
    return np.concatenate([pooled, ph[None]], axis=0)


# --------------------------------------------------------------------------
# Object pyramid (eqs. 2.5, 2.6 on the whole object)
# --------------------------------------------------------------------------
def restrict_object(z, times: int):
    """I_h^H applied `times` times with bins aligned to pixel 0."""
    out = np.asarray(z)
    for _ in range(times):
        out = restrict(out)
    return out


def prolong_object(zc, times: int):
    """I_H^h applied `times` times."""
    out = np.asarray(zc)
    for _ in range(times):
        out = prolong(out)
    return out
