"""Small shared helpers for the tests (random complex arrays, tiny problems)."""

import numpy as np


def crandn(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def random_probe(rng, m, zeros=False):
    q = crandn(rng, m, m)
    if zeros:
        q[rng.random((m, m)) < 0.2] = 0.0
    return q


def tiny_problem(rng, n=24, m=8, step=4, noiseless=True):
    """Random object/probe on a small raster with exact intensities from the oracle."""
    import oracle
    z_true = (0.8 + 0.2 * rng.random((n, n))) * np.exp(1j * rng.uniform(-1.5, 1.5, (n, n)))
    Q = random_probe(rng, m)
    pos = []
    for r in range(0, n - m + 1, step):
        for c in range(0, n - m + 1, step):
            pos.append((r, c))
    offsets = np.array(pos, dtype=np.int32)
    d = oracle.forward_model(z_true, Q, offsets)
    if not noiseless:
        d = d * (1.0 + 0.1 * rng.random(d.shape))
    return z_true, Q, offsets, np.sqrt(d)
