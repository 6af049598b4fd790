"""magpie_run_epochs_noalloc (no device allocation, fixed scratch) against
magpie_run_epochs: the same epochs with the library's seeded permutations must give
the same object bit for bit, on consecutive calls whose second input is smaller
(the scratch keeps the previous call's contents), across contexts of different
sizes, and when the epochs are processed in several chunks; one epoch also matches
the FP64 oracle at the per-step tolerance."""

import numpy as np
import pytest

import oracle
from gpu_cases import Case

pytestmark = pytest.mark.gpu


def _same(a, b):
    return np.array_equal(a.view(np.uint64), b.view(np.uint64))


def test_noalloc_equals_run_epochs_on_consecutive_calls():
    rng = np.random.default_rng(91)
    big = Case(rng, 150, 160, 32, 7, noise=0.05)
    small = Case(rng, 70, 76, 16, 5, noise=0.05)
    ga, gb = big.gpu(3, 0.5), big.gpu(3, 0.5)
    ga.run_epochs(3, 16, seed=5)
    gb.run_epochs_noalloc(3, 16, seed=5)
    assert _same(ga.get_object(), gb.get_object())
    assert ga.epoch_index == gb.epoch_index == 3
    # second call on the same contexts with a smaller minibatch and fewer epochs
    ga.run_epochs(1, 5, seed=5)
    gb.run_epochs_noalloc(1, 5, seed=5)
    assert _same(ga.get_object(), gb.get_object())
    ga.close()
    gb.close()
    # a smaller reconstruction next: the scratch still holds the larger call's values
    ha, hb = small.gpu(2, 0.5), small.gpu(2, 0.5)
    ha.run_epochs(1, 4, seed=9)
    hb.run_epochs_noalloc(1, 4, seed=9)
    za, zb = ha.get_object(), hb.get_object()
    ha.close()
    hb.close()
    assert _same(za, zb)
    zo = small.oracle_run(2, 0.5, [oracle.library_permutation(9, 0, small.n_pos)], 4)
    rel, relx = small.rel(zb.astype(np.complex128), zo), small.rel_max(zb.astype(np.complex128), zo)
    print("no-alloc epoch vs oracle: rel", rel, "element-wise", relx, flush=True)
    assert rel <= 1e-5 and relx <= 1e-5


def test_noalloc_chunked_epochs():
    """m = 128, minibatch 127: the staging takes all but 128 KiB of the 16 MiB scratch,
    so the records of 210 positions fit 31 epochs at a time; 40 epochs run in two chunks."""
    rng = np.random.default_rng(92)
    c = Case(rng, 232, 240, 128, 8, noise=0.05, jitter=0)
    assert c.n_pos == 210
    ga, gb = c.gpu(2, 0.5), c.gpu(2, 0.5)
    ga.run_epochs(40, 127, seed=3)
    gb.run_epochs_noalloc(40, 127, seed=3)
    assert _same(ga.get_object(), gb.get_object())
    assert gb.epoch_index == 40
    ga.close()
    gb.close()


def test_noalloc_rejections():
    from paper_2504_10118_amd import UPDATE_PROBE, Magpie, MagpieError
    rng = np.random.default_rng(93)
    c = Case(rng, 232, 240, 128, 8, noise=0.05, jitter=0)
    g = Magpie(c.n_rows, c.n_cols, 128, 2, 0.5)
    with pytest.raises(MagpieError) as e:
        g.run_epochs_noalloc(1, 4)
    assert e.value.name == "BAD_STATE"
    g.close()
    g = c.gpu(2, 0.5)
    with pytest.raises(MagpieError) as e:
        g.run_epochs_noalloc(1, 128)          # 128 x 128 KiB of staging: the whole scratch
    assert e.value.name == "UNSUPPORTED" and "16 MiB" in str(e.value)
    g.set_flags(UPDATE_PROBE, 0.2)
    with pytest.raises(MagpieError) as e:
        g.run_epochs_noalloc(1, 4)
    assert e.value.name == "UNSUPPORTED"
    g.close()
