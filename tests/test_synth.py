"""Properties of the seeded synthetic inputs (object, probe, scan, noise, permutations)."""

import numpy as np

from synth import WORKLOADS, make_object, make_probe, make_scan, poisson_counts, epoch_orders, workload_rngs


def test_probe_model():
    for m in (32, 64, 128):
        q = make_probe(m)
        a = np.abs(q)
        assert np.isclose(a.max(), 1.0)
        assert a.min() > 1e-9          # FP32 |Q|^2 never underflows to zero
        # symmetric about the centre
        np.testing.assert_allclose(a, a[::-1, ::-1], atol=1e-14)


def test_object_model():
    r = workload_rngs(2)[0]
    z = make_object(64, r, rectangles=True)
    amp = np.abs(z)
    assert amp.min() >= 0.8 and amp.max() <= 1.0
    ph = np.angle(z)
    assert ph.min() >= -np.pi / 2 - 1e-12


def test_scan_origins_and_bounds():
    for name, origin in (("128x128", 6), ("512x512", 29), ("1024x1024", 53)):
        c = WORKLOADS[name]
        offs = make_scan(c.n, c.m, c.P, c.step, np.random.default_rng(0), jitter=0)
        assert offs[0, 0] == origin and offs[0, 1] == origin
        j = make_scan(c.n, c.m, c.P, c.step, np.random.default_rng(1))
        assert j.shape == (c.P * c.P, 2)
        assert j.min() >= 0 and j.max() <= c.n - c.m
        assert np.abs(j - offs).max() <= 1


def test_poisson_scale():
    rng = np.random.default_rng(3)
    dt = np.linspace(0, 4, 1000)
    d = poisson_counts(dt, 1e4, rng)
    sigma = 1e4 / 4
    # counts are integers in units of 1 / sigma
    np.testing.assert_allclose(d * sigma, np.round(d * sigma), atol=1e-9)
    assert poisson_counts(dt, None, rng) is not dt


def test_epoch_orders():
    o = epoch_orders(3, 50, np.random.default_rng(4))
    for row in o:
        assert sorted(row.tolist()) == list(range(50))
