"""Levels sweep (paper_2504_10118_amd.sweep): host helpers on the CPU, a short sweep on the GPU."""

import numpy as np
import pytest

from paper_2504_10118_amd.sweep import checkpoints, object_errors, overlap_geometry, scaled_error


def test_checkpoints_log_spaced():
    assert checkpoints(1) == [1]
    assert checkpoints(7) == [1, 2, 3, 5, 7]
    assert checkpoints(200) == [1, 2, 3, 5, 10, 20, 30, 50, 100, 200]


def test_overlap_geometry_steps():
    """Overlap ratio r of the probe's disc (diameter 20 m / 32) gives step (1 - r) * 2R over
    the workload's own span; None keeps the workload."""
    from synth import WORKLOADS
    cfg = WORKLOADS["512x512"]                      # m = 64: disc diameter 40 px, span 39 * 10 px
    assert overlap_geometry(cfg, None) is cfg
    for r, step, P in ((0.25, 30, 14), (0.5, 20, 20), (0.75, 10, 40)):
        g = overlap_geometry(cfg, r)
        assert (g.step, g.P) == (step, P)
        assert (g.P - 1) * g.step <= (cfg.P - 1) * cfg.step


def test_scaled_error_ignores_a_complex_scale():
    rng = np.random.default_rng(4)
    z = rng.standard_normal((8, 8)) + 1j * rng.standard_normal((8, 8))
    assert scaled_error((0.3 - 2j) * z, z) < 1e-14
    w = z + 0.1 * (rng.standard_normal((8, 8)) + 1j * rng.standard_normal((8, 8)))
    e = scaled_error(w, z)
    assert 0 < e <= np.linalg.norm(w - z) / np.linalg.norm(z)
    mask = np.zeros((8, 8), bool)
    mask[2:6] = True
    assert scaled_error(np.where(mask, 2j * z, 0), z, mask) < 1e-14


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
    from synth import WORKLOADS, make_problem_inputs
    res = run(workload="128x128", alphas=(0.5,), peaks=(None,), epochs=20, log=lambda s: print(s, flush=True))
    assert [r["levels"] for r in res["runs"]] == [1, 2, 3, 4, 5, 6]
    for r in res["runs"]:
        assert r["finite"] and len(r["phi"]) == 21 and len(r["stat"]) == 21
        assert r["phi"][-1] < 0.5 * r["phi"][0]
        assert [e for e, _, _ in r["errors"]] == [0, 1, 2, 3, 5, 10, 20]
        assert r["errors"][-1][1] < r["errors"][0][1]
    # the sweep's L = 2 trajectory is the context's own: same permutations, same kernels
    cfg = WORKLOADS["128x128"]
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


@pytest.mark.gpu
def test_sweep_noise_and_overlap_paths():
    from paper_2504_10118_amd.sweep import run
    res = run(workload="128x128", levels=[1, 2], alphas=(0.5,), peaks=(), etas=(0.05,), overlaps=(None, 0.25), epochs=5,
              log=lambda s: print(s, flush=True))
    assert [(r["overlap"], r["levels"]) for r in res["runs"]] == [(None, 1), (None, 2), (0.25, 1), (0.25, 2)]
    for r in res["runs"]:
        assert r["finite"] and r["eta"] == 0.05 and r["phi"][-1] < r["phi"][0]
    assert res["runs"][2]["positions"] < res["runs"][0]["positions"]


@pytest.mark.gpu
def test_blind_runs():
    from paper_2504_10118_amd.sweep import run_blind
    from synth import WORKLOADS, make_problem_inputs
    res = run_blind(workload="128x128", levels=(2,), epochs=20, log=lambda s: print(s, flush=True))
    assert [r["mode"] for r in res["runs"]] == ["fixed", "simultaneous", "alternating"]
    Q = make_problem_inputs(WORKLOADS["128x128"])[1]
    start = scaled_error(np.abs(Q), Q)
    for r in res["runs"]:
        assert all(np.isfinite(v) for row in r["trace"] for v in row)
    fixed = res["runs"][0]["trace"]
    assert all(abs(q - start) < 1e-6 for _, _, q, _ in fixed)       # the probe never moves
    assert res["runs"][2]["trace"][-1][2] != fixed[-1][2]              # the alternating probe does
