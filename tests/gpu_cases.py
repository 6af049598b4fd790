"""Problem builders shared by the GPU parity tests.

Inputs are seeded and synthetic; intensities come from the FP64 oracle's
forward model and are rounded to FP32 before either side sees them, so that
parity measures computation error only.
"""

from __future__ import annotations

import numpy as np

import oracle
from synth import make_probe


def raster(n_rows, n_cols, m, step, rng=None, jitter=0):
    pos = []
    for r in range(0, n_rows - m + 1, step):
        for c in range(0, n_cols - m + 1, step):
            pos.append((r, c))
    offs = np.array(pos, dtype=np.int32)
    if rng is not None and jitter:
        offs = offs + rng.integers(-jitter, jitter + 1, size=offs.shape).astype(np.int32)
        offs[:, 0] = np.clip(offs[:, 0], 0, n_rows - m)
        offs[:, 1] = np.clip(offs[:, 1], 0, n_cols - m)
    return offs


def smooth_object(rng, n_rows, n_cols):
    amp = 0.8 + 0.2 * rng.random((n_rows, n_cols))
    yy, xx = np.mgrid[0:n_rows, 0:n_cols]
    ph = 0.9 * np.sin(2 * np.pi * yy / max(8, n_rows / 3) + 1.3) * np.cos(2 * np.pi * xx / max(8, n_cols / 2.5))
    return amp * np.exp(1j * ph)


class Case:
    """A small reconstruction problem with FP32 inputs and their FP64 upcasts."""

    def __init__(self, rng, n_rows, n_cols, m, step, probe="synthetic", noise=0.0, start_noise=0.1,
                 jitter=1, offsets=None):
        self.m = m
        self.n_rows, self.n_cols = n_rows, n_cols
        zt = smooth_object(rng, n_rows, n_cols)
        if probe == "synthetic":
            Q = make_probe(m)
        else:
            Q = (rng.standard_normal((m, m)) + 1j * rng.standard_normal((m, m))) / np.sqrt(2)
        self.Q32 = Q.astype(np.complex64)
        self.Q = self.Q32.astype(np.complex128)
        self.z_true32 = zt.astype(np.complex64)
        self.z_true = self.z_true32.astype(np.complex128)
        self.offs = raster(n_rows, n_cols, m, step, rng, jitter) if offsets is None else np.asarray(offsets, np.int32)
        d = oracle.forward_model(self.z_true, self.Q, self.offs)
        if noise:
            d = d * (1.0 + noise * rng.standard_normal(d.shape)) ** 2
        self.sd32 = np.sqrt(d).astype(np.float32)
        self.sd = self.sd32.astype(np.float64)
        z0 = zt * (1 + start_noise * (rng.standard_normal(zt.shape) + 1j * rng.standard_normal(zt.shape)))
        self.z0_32 = z0.astype(np.complex64)
        self.z0 = self.z0_32.astype(np.complex128)
        ill = oracle.illumination((n_rows, n_cols), self.Q, self.offs)
        self.mask = ill >= 0.1 * ill.max()
        self.covered = covered_pixels((n_rows, n_cols), m, self.offs)

    @property
    def n_pos(self):
        return len(self.offs)

    def gpu(self, levels, alpha, device=0):
        from paper_2504_10118_amd import Magpie
        g = Magpie(self.n_rows, self.n_cols, self.m, levels, alpha, device=device)
        g.set_probe(self.Q32)
        g.set_positions(self.offs)
        g.load_intensities(self.sd32, is_sqrt=True)
        g.set_object(self.z0_32)
        return g

    def oracle_run(self, levels, alpha, orders, batch, z0=None):
        u = oracle.u_rpie(self.Q, alpha)
        return oracle.run_epochs(self.z0 if z0 is None else z0, self.Q, self.offs, self.sd, u, levels,
                                 orders, batch, use_gradient_form=False)

    def rel(self, a, b):
        return float(np.linalg.norm((a - b)[self.mask]) / np.linalg.norm(b[self.mask]))

    def rel_max(self, a, b):
        """Element-wise bound, unmasked: max |a - b| over every pixel any window covers
        (where the update's denominator is positive), relative to max |b| there."""
        return elementwise_rel(a, b, self.covered)


def covered_pixels(shape, m, offs):
    """Pixels inside at least one m x m window."""
    cov = np.zeros(shape, dtype=bool)
    for r, c in offs:
        cov[r:r + m, c:c + m] = True
    return cov


def elementwise_rel(a, b, covered):
    d = np.abs(np.asarray(a) - np.asarray(b))[covered]
    return float(d.max() / np.abs(np.asarray(b)[covered]).max())
