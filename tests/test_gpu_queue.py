"""GPU: the work-queue launch of multi-reconstruction runs (flag MAGPIE_PERSISTENT).

The queue takes the same steps and accumulations as the round-by-round launches in a
different schedule (one launch per plan partition and chunk of epochs; each item waits for
the items of its own reconstruction it depends on), so its results must equal theirs
bit for bit; one epoch of each reconstruction is also checked against the FP64 oracle
(masked and element-wise, 1e-5).  The failure path (a wait longer than its bound) is
forced from the host with a zero bound, so every kernel still exits normally.
"""

import os

import numpy as np
import pytest

import oracle
from gpu_cases import Case

pytestmark = pytest.mark.gpu


def _print(*a):
    print(*a, flush=True)


def _cases(seed):
    rng = np.random.default_rng(seed)
    cases = [Case(rng, 120, 100, 16, 6, noise=0.05), Case(rng, 150, 170, 32, 9, noise=0.05),
             Case(rng, 160, 176, 64, 16, noise=0.05), Case(rng, 150, 166, 64, 13, noise=0.05),
             Case(rng, 200, 216, 128, 24, noise=0.05), Case(rng, 180, 196, 128, 21, noise=0.05)]
    levels = [3, 2, 3, 4, 4, 3]
    batches = [7, 25, 9, 6, 5, 4]
    return cases, levels, batches


def _run(cases, levels, batches, epochs, seed, queue, tiles=None):
    from paper_2504_10118_amd import PERSISTENT, run_epochs_multi
    gs = [c.gpu(L, 0.5) for c, L in zip(cases, levels)]
    for g, th in zip(gs, tiles or [None] * len(gs)):
        if th:
            g.set_tuning(0, th)
        if queue:
            g.set_flags(PERSISTENT)
    run_epochs_multi(gs, epochs, batches, seed=seed)
    out = [g.get_object() for g in gs]
    eps = [g.epoch_index for g in gs]
    for g in gs:
        g.close()
    return out, eps


def test_queue_equals_rounds_bitwise():
    """Six reconstructions (probes 16 to 128: five plan partitions on concurrent streams,
    the two 128-point reconstructions' plan split in two), ten epochs (chunks of 1, 8 and 1
    epochs, so both descriptor slots are reused), tile heights 8, 16 and 32 on the
    round-by-round side: the queue's objects are identical."""
    cases, levels, batches = _cases(91)
    ref, _ = _run(cases, levels, batches, 10, 55, queue=False, tiles=[None, 16, 32, None, 16, None])
    got, eps = _run(cases, levels, batches, 10, 55, queue=True)
    for c, a, b, ep in zip(cases, got, ref, eps):
        _print("queue m", c.m, "N", c.n_pos, "identical", np.array_equal(a.view(np.uint64), b.view(np.uint64)))
        assert ep == 10
        assert np.array_equal(a.view(np.uint64), b.view(np.uint64))


def test_queue_matches_oracle():
    """One epoch through the queue, each reconstruction against the oracle's epoch with
    the library's permutation."""
    cases, levels, batches = _cases(92)
    got, _ = _run(cases, levels, batches, 1, 79, queue=True)
    for c, z, L, B in zip(cases, got, levels, batches):
        zg = z.astype(np.complex128)
        zo = c.oracle_run(L, 0.5, [oracle.library_permutation(79, 0, c.n_pos)], B)
        rel, relx = c.rel(zg, zo), c.rel_max(zg, zo)
        _print("queue vs oracle m", c.m, "N", c.n_pos, "B", B, "rel", rel, "element-wise", relx)
        assert rel <= 1e-5 and relx <= 1e-5


def test_queue_single_context_and_full_minibatch():
    """magpie_run_epochs with the flag runs the context through the queue: equal to the
    plain run bit for bit, here with minibatches of 256 positions of a 128 x 128 probe
    (the largest the queue takes) and a short last minibatch."""
    from paper_2504_10118_amd import PERSISTENT
    rng = np.random.default_rng(93)
    c = Case(rng, 420, 420, 128, 14, noise=0.05)
    assert c.n_pos > 256 and c.n_pos % 256 != 0
    g = c.gpu(4, 0.5)
    g.run_epochs(3, 256, seed=5)
    ref = g.get_object()
    g.close()
    g = c.gpu(4, 0.5)
    g.set_flags(PERSISTENT)
    g.run_epochs(3, 256, seed=5)
    got = g.get_object()
    assert g.epoch_index == 3
    g.close()
    assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))


def test_queue_argument_errors():
    """Mixed flags, caller orders, minibatches above 256 and plans of fewer than 64
    threads are refused before anything runs."""
    from paper_2504_10118_amd import PERSISTENT, MagpieError, run_epochs_multi
    rng = np.random.default_rng(94)
    a, b = Case(rng, 90, 90, 32, 9, noise=0.05), Case(rng, 90, 90, 32, 9, noise=0.05)
    ga, gb = a.gpu(2, 0.5), b.gpu(2, 0.5)
    ga.set_flags(PERSISTENT)
    with pytest.raises(MagpieError, match="INVALID_ARG"):
        run_epochs_multi([ga, gb], 1, [5, 5])
    gb.set_flags(PERSISTENT)
    with pytest.raises(MagpieError, match="UNSUPPORTED"):
        ga.run_epochs(1, 5, order=np.arange(a.n_pos, dtype=np.int32)[None, :])
    ga.close()
    gb.close()
    big = Case(rng, 300, 300, 16, 3, noise=0.05)
    assert big.n_pos > 256
    g = big.gpu(2, 0.5)
    g.set_flags(PERSISTENT)
    with pytest.raises(MagpieError, match="UNSUPPORTED"):
        g.run_epochs(1, 300)
    g.close()
    small = Case(rng, 40, 40, 8, 4, noise=0.05)
    g = small.gpu(2, 0.5)
    g.set_flags(PERSISTENT)
    with pytest.raises(MagpieError, match="UNSUPPORTED"):
        g.run_epochs(1, 4)
    g.close()


def test_queue_wait_bound_stops_the_queue():
    """A zero bound on the items' waits (set from the host) makes the first item that
    has to wait stop the queue: every workgroup exits, the call reports the failure,
    and the next run (default bound) is correct again."""
    from paper_2504_10118_amd import PERSISTENT, MagpieError
    rng = np.random.default_rng(95)
    c = Case(rng, 420, 420, 128, 14, noise=0.05)
    g = c.gpu(4, 0.5)
    g.set_flags(PERSISTENT)
    os.environ["MAGPIE_QUEUE_WAIT_US"] = "0"
    try:
        with pytest.raises(MagpieError, match="HIP"):
            g.run_epochs(2, 256, seed=6)
    finally:
        del os.environ["MAGPIE_QUEUE_WAIT_US"]
    g.close()
    g = c.gpu(4, 0.5)
    g.run_epochs(2, 256, seed=6)
    ref = g.get_object()
    g.close()
    g = c.gpu(4, 0.5)
    g.set_flags(PERSISTENT)
    g.run_epochs(2, 256, seed=6)
    assert np.array_equal(g.get_object().view(np.uint64), ref.view(np.uint64))
    g.close()
