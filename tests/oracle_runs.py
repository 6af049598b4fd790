"""Oracle runs for the GPU tests, in worker processes started with `spawn` (they
inherit no GPU state from the test process).  Everything here calls only the
oracle and the synthetic inputs."""

from __future__ import annotations

import numpy as np

import oracle


def objective_after_epochs(args):
    """Phi (eq. 2.1) after the oracle's epochs from the flat object, optionally
    perturbed by `eps` relative complex Gaussian noise drawn with `seed`."""
    n, Q, offs, sd, alpha, levels, orders, batch, eps, seed = args
    z0 = np.ones((n, n), dtype=np.complex128)
    if eps:
        r = np.random.default_rng(seed)
        z0 = z0 * (1 + eps * (r.standard_normal(z0.shape) + 1j * r.standard_normal(z0.shape)))
    u = oracle.u_rpie(Q, alpha)
    zo = oracle.run_epochs(z0, Q, offs, sd, u, levels, orders, batch)
    return oracle.objective(zo, Q, offs, sd), zo
