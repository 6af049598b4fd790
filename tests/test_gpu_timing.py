"""Kernel timing through the C ABI (the figures bench.py's roofline is built from):
one record per launch of the step and the accumulation kernel, with the positions of
each step launch, agreeing with the summed counters, which reading resets."""

import numpy as np
import pytest

from gpu_cases import Case

pytestmark = pytest.mark.gpu


def test_launch_times_follow_the_minibatches():
    from paper_2504_10118_amd.magpie import MagpieError
    rng = np.random.default_rng(77)
    m = 32
    c = Case(rng, 2 * m + 9, 2 * m + 11, m, 10)
    N = c.n_pos
    B = 7                                   # a ragged last minibatch
    nb = -(-N // B)
    assert N % B != 0
    g = c.gpu(2, 0.5)
    g.run_epochs(1, B, seed=4)              # untimed: records start when timing is enabled
    g.set_timing(True)
    epochs = 3
    g.run_epochs(epochs, B, seed=5)
    us0, pos0 = g.launch_times(0)
    us1, pos1 = g.launch_times(1)
    print(f"N {N} B {B}: {len(us0)} step launches, mean {us0.mean():.1f} us; "
          f"{len(us1)} accumulation launches, mean {us1.mean():.1f} us", flush=True)
    assert len(us0) == epochs * nb and len(us1) == epochs * nb
    assert np.all(us0 > 0) and np.all(us1 > 0)
    assert pos0.tolist() == [min(B, N - t * B) for t in range(nb)] * epochs
    assert np.all(pos1 == 0)
    # reading the launches does not reset them; the summed counters do
    assert len(g.launch_times(0)[0]) == epochs * nb
    t = g.get_timing()
    assert t["step_launches"] == epochs * nb and t["accum_launches"] == epochs * nb
    assert t["positions"] == epochs * N
    assert abs(t["step_ms"] * 1e3 - us0.sum()) <= 1e-6 * us0.sum() + 1e-3
    assert abs(t["accum_ms"] * 1e3 - us1.sum()) <= 1e-6 * us1.sum() + 1e-3
    assert len(g.launch_times(0)[0]) == 0
    # enabling again starts the records anew
    g.run_epochs(1, B, seed=6)
    g.set_timing(True)
    assert len(g.launch_times(1)[0]) == 0
    g.set_timing(False)
    g.run_epochs(1, B, seed=7)
    assert len(g.launch_times(0)[0]) == 0
    with pytest.raises(MagpieError):
        g.launch_times(2)
    g.close()
