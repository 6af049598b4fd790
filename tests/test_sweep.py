"""Levels sweep (paper_2504_10118_amd.sweep): host helpers on the CPU, a short sweep on the GPU."""

import numpy as np
import pytest

from paper_2504_10118_amd.sweep import checkpoints, object_errors


def test_checkpoints_log_spaced():
    assert checkpoints(1) == [1]
    assert checkpoints(7) == [1, 2, 3, 5, 7]
    assert checkpoints(200) == [1, 2, 3, 5, 10, 20, 30, 50, 100, 200]


def test_object_errors_global_phase_and_magnitude():
    rng = np.random.default_rng(3)
    z = (rng.uniform(0.8, 1, (16, 16)) * np.exp(1j * rng.uniform(-1, 1, (16, 16))))
    mask = np.ones(z.shape, bool)
    mask[:2] = False
    rel, mag = object_errors(np.exp(0.7j) * z, z, mask)
    assert rel < 1e-14 and mag < 1e-14
    # a pure magnitude change of 1 % everywhere: both errors equal 1 % of ||z*|| / ||z*||
    rel, mag = object_errors(1.01 * z, z, mask)
    assert abs(rel - 0.01) < 1e-12 and abs(mag - 0.01) < 1e-12
    # the conjugate has the right magnitudes but a wrong phase
    rel, mag = object_errors(np.conj(z), z, mask)
    assert mag < 1e-14 and rel > 0.1


@pytest.mark.gpu
def test_short_sweep_runs_every_level():
    from paper_2504_10118_amd import Magpie
    from paper_2504_10118_amd.sweep import illumination_mask, run, run_one
    from synth import CONFIGS, make_problem_inputs
    res = run(config=1, alphas=(0.5,), peaks=(None,), epochs=20, log=lambda s: print(s, flush=True))
    assert [r["levels"] for r in res["runs"]] == [1, 2, 3, 4, 5, 6]
    for r in res["runs"]:
        assert r["finite"] and len(r["phi"]) == 21 and len(r["stat"]) == 21
        assert r["phi"][-1] < 0.5 * r["phi"][0]
        assert [e for e, _, _ in r["errors"]] == [0, 1, 2, 3, 5, 10, 20]
        assert r["errors"][-1][1] < r["errors"][0][1]
    # the sweep's L = 2 trajectory is the context's own: same permutations, same kernels
    cfg = CONFIGS[1]
    z_true, Q, offs, _, _ = make_problem_inputs(cfg)
    with Magpie(cfg.n, cfg.n, cfg.m, 1, 0.5) as fm:
        fm.set_probe(Q.astype(np.complex64))
        fm.set_positions(offs)
        d = fm.forward_model(z_true.astype(np.complex64))
    with Magpie(cfg.n, cfg.n, cfg.m, 2, 0.5) as ctx:
        ctx.set_probe(Q.astype(np.complex64))
        ctx.set_positions(offs)
        ctx.load_intensities(d, is_sqrt=False)
        again = run_one(ctx, z_true.astype(np.complex64), illumination_mask(Q, offs, cfg.n), 20, cfg.batch, 7,
                        1e-4)
    assert again["phi"] == res["runs"][1]["phi"]
