"""GPU parity at the full workload sizes, in the configuration bench.py times.

512 x 512 object, 64 x 64 probe, 3 levels, minibatch 256 (1600 positions) and
1024 x 1024 object, 128 x 128 probe, 4 levels, minibatch 256 (6400 positions).
The plan and tile height are the autotuner's, as in the benchmark.
Intensities come from the oracle's forward model of the true object, with
Poisson noise, rounded to FP32.

Per step (1e-5 relative in the masked norm, and element-wise over every covered
pixel, 1e-5 of the largest value): minibatch t of the epoch's order is run on the
GPU (magpie_run_minibatch, in the context holding all 1600 or 6400 positions, so the
accumulation screens every position overlapping each tile as in production) from
the oracle's own object after t minibatches (rounded to complex64), and compared
with the oracle's step from the same object.  From the flat object the exit waves
are the probe itself, whose far field no single-precision transform resolves
(an independent complex64 computation of that step is off by ~4e-5); the kernels
transform Q (z_k - 1) and add the probe's spectrum computed once in FP64, and the
flat-start step is held to 1e-5 like every other.  Whole epoch (512 x 512, 7
dependent minibatches, flat start): held to 1e-5 as well; the objective of the
oracle's object is compared at 1e-5.  Fifty
epochs from the flat start with identical permutations: the objective (eq. 2.1) of
the two trajectories agrees to 1e-4.
"""

import numpy as np
import pytest

import oracle
from synth import WORKLOADS, make_problem_inputs, poisson_counts

pytestmark = pytest.mark.gpu


def _problem(name):
    cfg = WORKLOADS[name]
    z, Q, offs, r_noise, _ = make_problem_inputs(cfg)
    Q32 = Q.astype(np.complex64)
    d = oracle.forward_model(z, Q32.astype(np.complex128), offs)
    sd32 = np.sqrt(poisson_counts(d, cfg.peak, r_noise)).astype(np.float32)
    ill = oracle.illumination((cfg.n, cfg.n), Q32.astype(np.complex128), offs)
    order = oracle.library_permutation(31 + cfg.seed_id, 0, cfg.n_pos)
    return cfg, Q32, offs, sd32, order, ill >= 0.1 * ill.max()


def _gpu(cfg, Q32, offs, sd32, z0):
    from paper_2504_10118_amd import Magpie
    g = Magpie(cfg.n, cfg.n, cfg.m, cfg.levels, cfg.alpha)
    g.set_probe(Q32)
    g.set_positions(offs)
    g.load_intensities(sd32, is_sqrt=True)
    g.set_object(z0.astype(np.complex64))
    g.autotune(min(cfg.batch, len(offs)))       # restores the object and the epoch counter
    return g


def _rel(a, b, mask):
    return float(np.linalg.norm((a - b)[mask]) / np.linalg.norm(b[mask]))


def _relx(a, b, cfg, offs):
    from gpu_cases import covered_pixels, elementwise_rel
    return elementwise_rel(a, b, covered_pixels((cfg.n, cfg.n), cfg.m, offs))


def _fp32_fft_step_errors(cfg, Q32, offs, sd32, chunk, z0, mask):
    """Relative errors (masked norm, element-wise over covered pixels) of a one-level
    step whose FFTs run in single precision (SciPy's complex64 transforms, an
    implementation independent of the HIP path) against the FP64 oracle's step from the
    same object z0: the FP32 floor of that step on these data."""
    import scipy.fft as sf
    m = cfg.m
    Q = Q32.astype(np.complex128)
    u = oracle.u_rpie(Q, cfg.alpha)
    zo = oracle.minibatch_step(z0, Q, offs, sd32.astype(np.float64), u, 1, chunk)
    w0 = u + np.abs(Q) ** 2
    num = np.zeros(z0.shape, dtype=np.complex128)
    den = np.zeros(z0.shape)
    for k in chunk:
        r, c = offs[k]
        psi = Q32 * z0[r:r + m, c:c + m].astype(np.complex64)
        P = sf.fft2(psi)
        a = np.abs(P)
        ph = np.where(a > 0, P / np.where(a > 0, a, 1), 1).astype(np.complex64)
        R = sf.ifft2((sd32[k] * ph).astype(np.complex64))
        num[r:r + m, c:c + m] -= (np.conj(Q32) * (psi - R)).astype(np.complex128)
        den[r:r + m, c:c + m] += w0
    zf = z0.copy()
    pos = den > 0
    zf[pos] += num[pos] / den[pos]
    return _rel(zf, zo, mask), _relx(zf, zo, cfg, offs)


@pytest.mark.parametrize("levels", [1, 4])
def test_full_size_flat_start_step(levels):
    """1024 x 1024, 128 x 128 probe, 1e5 photons, first step from the flat object: many
    far-field pixels carry a model amplitude ~1e-6 of the peak, whose phase a plain
    single-precision transform takes from rounding (an independent complex64
    computation of the one-grid step, printed for reference, is off by ~4e-5).  The
    GPU's step (one grid, and the workload's four) meets 1e-5."""
    cfg, Q32, offs, sd32, order, mask = _problem("1024x1024")
    chunk = order[:cfg.batch]
    Q = Q32.astype(np.complex128)
    u = oracle.u_rpie(Q, cfg.alpha)
    z0 = np.ones((cfg.n, cfg.n), dtype=np.complex128)
    floor, floor_x = _fp32_fft_step_errors(cfg, Q32, offs, sd32, chunk, z0, mask)
    zo = oracle.minibatch_step(z0, Q, offs, sd32.astype(np.float64), u, levels, chunk)
    from paper_2504_10118_amd import Magpie
    g = Magpie(cfg.n, cfg.n, cfg.m, levels, cfg.alpha)
    g.set_probe(Q32)
    g.set_positions(offs)
    g.load_intensities(sd32, is_sqrt=True)
    g.set_object(z0.astype(np.complex64))
    g.run_minibatch(chunk)
    zg = g.get_object().astype(np.complex128)
    g.close()
    rel = _rel(zg, zo, mask)
    relx = _relx(zg, zo, cfg, offs)
    print(f"flat-start step L={levels}: GPU rel {rel:.2e} (element-wise {relx:.2e}); plain complex64 transforms "
          f"{floor:.2e} (element-wise {floor_x:.2e})", flush=True)
    assert rel <= 1e-5
    assert relx <= 1e-5


@pytest.mark.parametrize("name,steps", [("512x512", 3), ("1024x1024", 3)])
def test_full_size_steps_match_oracle(name, steps):
    """Steps t = 0 .. steps-1 of the epoch (the first from the flat object), each from the
    oracle's object after t steps, one minibatch at a time in the context of all positions."""
    cfg, Q32, offs, sd32, order, mask = _problem(name)
    Q = Q32.astype(np.complex128)
    u = oracle.u_rpie(Q, cfg.alpha)
    sd = sd32.astype(np.float64)
    z = np.ones((cfg.n, cfg.n), dtype=np.complex128)
    g = _gpu(cfg, Q32, offs, sd32, z)
    tuning = g.get_tuning()
    for t in range(steps):
        chunk = order[t * cfg.batch:(t + 1) * cfg.batch]
        z_in = z.astype(np.complex64).astype(np.complex128)
        zo = oracle.minibatch_step(z_in, Q, offs, sd, u, cfg.levels, chunk)
        g.set_object(z_in.astype(np.complex64))
        g.run_minibatch(chunk)
        zg = g.get_object().astype(np.complex128)
        rel = _rel(zg, zo, mask)
        relx = _relx(zg, zo, cfg, offs)
        print(f"{cfg.n}x{cfg.n} minibatch {t}: plan {tuning}, rel {rel:.2e}, element-wise {relx:.2e}", flush=True)
        assert rel <= 1e-5
        assert relx <= 1e-5
        z = zo
    g.close()


def test_full_size_epoch_and_objective():
    cfg, Q32, offs, sd32, order, mask = _problem("512x512")
    g = _gpu(cfg, Q32, offs, sd32, np.ones((cfg.n, cfg.n)))
    g.run_epochs(1, cfg.batch, order=order[None, :])
    zg = g.get_object().astype(np.complex128)
    Q = Q32.astype(np.complex128)
    u = oracle.u_rpie(Q, cfg.alpha)
    zo = oracle.run_epochs(np.ones((cfg.n, cfg.n)), Q, offs, sd32.astype(np.float64), u, cfg.levels, [order],
                           cfg.batch)
    rel = _rel(zg, zo, mask)
    print(f"epoch rel {rel:.2e}", flush=True)
    assert rel <= 1e-5
    # the objective (eq. 2.1) over all 1600 positions at the oracle's object
    g.set_object(zo.astype(np.complex64))
    phi_g, _ = g.objective()
    phi_o = oracle.objective(zo.astype(np.complex64).astype(np.complex128), Q, offs, sd32.astype(np.float64))
    print(f"objective {phi_g:.6e} vs {phi_o:.6e}", flush=True)
    assert abs(phi_g - phi_o) <= 1e-5 * phi_o
    g.close()


def test_full_size_objective_after_50_epochs():
    """512 x 512, 64 x 64 probe, 3 levels, minibatch 256, 1e4 photons: 50 epochs from the
    flat start with the same explicit permutations on both sides; the objective (eq. 2.1,
    FP64 reduction) of the GPU's object and of the oracle's object agree to 1e-4.  The
    GPU path is deterministic (fixed-order sums), so the figure is a property of the
    build.  For context the test also prints the spread of the oracle's own objective
    when its flat start is perturbed at the FP32 rounding level (1e-7): the stochastic
    iteration amplifies any rounding-level difference (those runs end 2-3 % apart in the
    object and up to ~2e-4 apart in the objective)."""
    import multiprocessing as mp
    from oracle_runs import objective_after_epochs
    cfg, Q32, offs, sd32, _, mask = _problem("512x512")
    epochs = 50
    orders = np.stack([oracle.library_permutation(41, e, cfg.n_pos) for e in range(epochs)])
    g = _gpu(cfg, Q32, offs, sd32, np.ones((cfg.n, cfg.n)))
    g.run_epochs(epochs, cfg.batch, order=orders)
    phi_g, stat_g = g.objective()
    zg = g.get_object().astype(np.complex128)
    g.close()
    Q = Q32.astype(np.complex128)
    sd = sd32.astype(np.float64)
    base = (cfg.n, Q, offs, sd, cfg.alpha, cfg.levels, orders, cfg.batch)
    jobs = [base + (0.0, 0)] + [base + (1e-7, s) for s in (1, 2, 3)]
    with mp.get_context("spawn").Pool(4) as pool:
        res = pool.map(objective_after_epochs, jobs)
    phi_o, zo = res[0]
    band = max(abs(p - phi_o) for p, _ in res[1:])
    phi_0 = oracle.objective(np.ones((cfg.n, cfg.n)), Q, offs, sd)
    drift = _rel(zg, zo, mask)
    print(f"50 epochs: phi gpu {phi_g:.8e} oracle {phi_o:.8e} (start {phi_0:.4e}), rel {abs(phi_g - phi_o) / phi_o:.2e}, "
          f"object drift {drift:.2e}; oracle spread under 1e-7 start perturbations {band / phi_o:.2e}", flush=True)
    assert abs(phi_g - phi_o) <= 1e-4 * phi_o


def test_long_run_stays_finite():
    """2000 epochs of the 512 x 512 workload from the flat start (3.2 M steps of the kernel
    pipeline): the objective stays finite and does not rise above its level after 200
    epochs by more than the noise of the plateau (1 %), and the object stays finite."""
    cfg, Q32, offs, sd32, _, mask = _problem("512x512")
    g = _gpu(cfg, Q32, offs, sd32, np.ones((cfg.n, cfg.n)))
    g.run_epochs(200, cfg.batch, seed=17)
    phi_200, _ = g.objective()
    g.run_epochs(1800, cfg.batch, seed=17)
    phi_2000, stat = g.objective()
    z = g.get_object()
    g.close()
    print(f"long run: phi after 200 epochs {phi_200:.6e}, after 2000 {phi_2000:.6e}, statistic {stat:.3e}",
          flush=True)
    assert np.isfinite(phi_2000) and np.isfinite(stat) and np.all(np.isfinite(z))
    assert phi_2000 <= 1.01 * phi_200

