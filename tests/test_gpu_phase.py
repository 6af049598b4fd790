"""GPU parity of eq. (3.2) phase recycling (flag MAGPIE_PHASE_RECYCLE) against the FP64
oracle's driver with its phase store.

* generic data (no exact zeros): the flagged step equals the oracle's plain step;
* a patch set to zero between epochs: positions whose window lies inside it see an
  all-zero exit wave, and their revised exit waves come from the phases stored at their
  previous visit (the oracle's phase store, carried the same way); without the flag the
  same epoch differs from that by far more than the tolerance;
* from the flat object with the symmetric probe the exit waves' spectra vanish exactly on
  whole lines at every visit, and the store is consulted there on both sides;
* switching the flag off and on starts the store over (theta = 0), the autotuner's trial
  epochs leave it alone, and multi-context runs refuse flagged contexts.
"""

import numpy as np
import pytest

import oracle
from gpu_cases import Case

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _zeroed_case():
    rng = np.random.default_rng(320)
    c = Case(rng, 72, 68, 16, 4, noise=0.0, start_noise=0.05)
    z = c.z0_32.copy()
    z[20:44, 18:46] = 0                     # windows of 16 x 16 fully inside this block see zeros only
    inside = [k for k, (r, cc) in enumerate(c.offs) if 20 <= r <= 28 and 18 <= cc <= 30]
    assert len(inside) >= 4
    return c, z, inside


def _gpu(c, levels, alpha, flags):
    g = c.gpu(levels, alpha)
    g.set_flags(flags)
    return g


@pytest.mark.parametrize("m,levels", [(16, 2), (64, 3), (128, 4)])
def test_recycling_without_zeros_matches_plain_oracle(m, levels):
    from paper_2504_10118_amd import PHASE_RECYCLE
    rng = np.random.default_rng(330 + m)
    c = Case(rng, 2 * m + 9, 2 * m + 7, m, max(2, m // 3), noise=0.05)
    order = rng.permutation(c.n_pos).astype(np.int32)
    g = _gpu(c, levels, 0.5, PHASE_RECYCLE)
    g.run_epochs(1, 5, order=order[None])
    zg = g.get_object().astype(np.complex128)
    g.close()
    zo = c.oracle_run(levels, 0.5, [order], 5)
    rel = c.rel(zg, zo)
    print("recycle, generic data, m", m, "rel", rel, flush=True)
    assert rel <= TOL


@pytest.mark.parametrize("m,levels", [(32, 3), (64, 3)])
def test_recycling_from_the_flat_object(m, levels):
    """Two epochs, each from the flat object, with the symmetric synthetic probe: every
    exit wave is the probe itself, whose spectrum vanishes exactly on whole lines, so the
    phase store is consulted at those pixels on every visit (and keeps its initial
    theta = 0 there); the flagged GPU epochs equal the oracle's driver with its store."""
    from paper_2504_10118_amd import PHASE_RECYCLE
    rng = np.random.default_rng(340 + m)
    c = Case(rng, 2 * m + 9, 2 * m + 7, m, max(2, m // 3), noise=0.05)
    flat = np.ones((c.n_rows, c.n_cols), dtype=np.complex128)
    orders = [rng.permutation(c.n_pos).astype(np.int32) for _ in range(2)]
    B = max(1, c.n_pos // 3)
    u = oracle.u_rpie(c.Q, 0.5)
    ph = oracle.initial_phases(c.n_pos, c.m)
    oracle.run_epochs(flat, c.Q, c.offs, c.sd, u, levels, [orders[0]], B, phases=ph)
    zo = oracle.run_epochs(flat, c.Q, c.offs, c.sd, u, levels, [orders[1]], B, phases=ph)
    g = _gpu(c, levels, 0.5, PHASE_RECYCLE)
    for o in orders:
        g.set_object(flat.astype(np.complex64))
        g.run_epochs(1, B, order=o[None])
    zg = g.get_object().astype(np.complex128)
    g.close()
    rel, relx = c.rel(zg, zo), c.rel_max(zg, zo)
    print("recycle from flat, m", m, "rel", rel, "element-wise", relx, flush=True)
    assert rel <= TOL and relx <= TOL


@pytest.mark.parametrize("levels,batch", [(1, 210), (2, 210), (3, 64), (4, 105)])
def test_recycled_phases_on_a_zeroed_patch(levels, batch):
    from paper_2504_10118_amd import PHASE_RECYCLE
    c, zz, inside = _zeroed_case()
    rng = np.random.default_rng(331 + levels)
    orders = [rng.permutation(c.n_pos).astype(np.int32) for _ in range(2)]
    u = oracle.u_rpie(c.Q, 0.5)
    # oracle: epoch 0 from z0 fills the phase store, epoch 1 runs on the zeroed object
    ph = oracle.initial_phases(c.n_pos, c.m)
    oracle.run_epochs(c.z0, c.Q, c.offs, c.sd, u, levels, [orders[0]], batch, phases=ph)
    zo = oracle.run_epochs(zz.astype(np.complex128), c.Q, c.offs, c.sd, u, levels, [orders[1]], batch, phases=ph)
    zo_plain = oracle.run_epochs(zz.astype(np.complex128), c.Q, c.offs, c.sd, u, levels, [orders[1]], batch)
    g = _gpu(c, levels, 0.5, PHASE_RECYCLE)
    g.run_epochs(1, batch, order=orders[0][None])
    g.autotune(batch)                       # trial epochs must not touch the store
    g.set_object(zz)
    g.run_epochs(1, batch, order=orders[1][None])
    zg = g.get_object().astype(np.complex128)
    g.close()
    rel = c.rel(zg, zo)
    gap = c.rel(zo_plain, zo)
    print("zeroed patch L", levels, "B", batch, "rel", rel, "recycled vs theta=0", gap, flush=True)
    assert rel <= TOL
    assert gap > 100 * TOL


def test_switching_the_flag_restarts_the_store():
    from paper_2504_10118_amd import PHASE_RECYCLE
    c, zz, _ = _zeroed_case()
    rng = np.random.default_rng(340)
    orders = [rng.permutation(c.n_pos).astype(np.int32) for _ in range(2)]
    B = c.n_pos                             # one minibatch: the zeroed windows see zeros only
    g = _gpu(c, 2, 0.5, PHASE_RECYCLE)
    g.run_epochs(1, B, order=orders[0][None])
    g.set_flags(0)
    g.set_flags(PHASE_RECYCLE)              # theta = 0 everywhere again
    g.set_object(zz)
    g.run_epochs(1, B, order=orders[1][None])
    zg = g.get_object().astype(np.complex128)
    g.close()
    u = oracle.u_rpie(c.Q, 0.5)
    zo = oracle.run_epochs(zz.astype(np.complex128), c.Q, c.offs, c.sd, u, 2, [orders[1]], B,
                           phases=oracle.initial_phases(c.n_pos, c.m))
    ph = oracle.initial_phases(c.n_pos, c.m)
    oracle.run_epochs(c.z0, c.Q, c.offs, c.sd, u, 2, [orders[0]], B, phases=ph)
    zkept = oracle.run_epochs(zz.astype(np.complex128), c.Q, c.offs, c.sd, u, 2, [orders[1]], B, phases=ph)
    rel = c.rel(zg, zo)
    print("restarted store rel", rel, "vs a kept store", c.rel(zg, zkept), flush=True)
    assert rel <= TOL
    assert c.rel(zg, zkept) > 100 * TOL


def test_multi_context_runs_refuse_recycling():
    from paper_2504_10118_amd import PHASE_RECYCLE, MagpieError, run_epochs_multi
    c, _, _ = _zeroed_case()
    a = _gpu(c, 2, 0.5, 0)
    b = _gpu(c, 2, 0.5, PHASE_RECYCLE)
    with pytest.raises(MagpieError):
        run_epochs_multi([a, b], 1, 7)
    a.close()
    b.close()
