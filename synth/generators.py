"""Seeded generators for objects, probes, scans, noise and permutations.

Every stream comes from ``numpy.random.Generator(PCG64)`` spawned from
``SeedSequence(250410118 + seed_id)`` so that a workload is fully
reproducible from its seed id alone.  Nothing here evaluates the forward model:
callers compute noiseless intensities with their own implementation and pass
them to :func:`poisson_counts`.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_BASE = 250410118


@dataclasses.dataclass(frozen=True)
class ScanConfig:
    """One ptychography workload: object side n, probe side m, P x P raster; named by its
    object side, and seeded by seed_id (an offset of the seed sequence)."""

    name: str
    seed_id: int
    n: int                 # object side (pixels)
    m: int                 # probe / patch side (pixels)
    P: int                 # raster is P x P positions
    step: int              # raster step (pixels)
    levels: int            # number of grids (fine + coarse)
    peak: float | None     # peak photon count; None = noiseless
    batch: int             # minibatch size used for this workload
    rectangles: bool       # add 20 phase rectangles to the object
    epochs: int            # epochs of a standard run
    alpha: float = 0.5     # rPIE regularisation constant

    @property
    def n_pos(self) -> int:
        return self.P * self.P


# Workloads (sizes of the paper's Section 5 setup scaled around it).
WORKLOADS = {
    "128x128": ScanConfig("128x128", 1, n=128, m=32, P=8, step=12, levels=2, peak=None, batch=8,
                          rectangles=False, epochs=20),
    "512x512": ScanConfig("512x512", 2, n=512, m=64, P=40, step=10, levels=3, peak=1e4, batch=256,
                          rectangles=True, epochs=50),
    "1024x1024": ScanConfig("1024x1024", 3, n=1024, m=128, P=80, step=10, levels=4, peak=1e5, batch=256,
                            rectangles=True, epochs=20),
}


def workload_rngs(seed_id: int):
    """Independent generators: object, scan jitter, noise, permutations, learned-start set."""
    ss = np.random.SeedSequence(SEED_BASE + int(seed_id))
    return [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(5)]


def make_object(n: int, rng: np.random.Generator, rectangles: bool) -> np.ndarray:
    """Complex n x n object: amplitude U[0.8,1]; smooth phase bumps (+ rectangles).

    Phase = sum of 8 Gaussian bumps (centres uniform on the grid, widths
    U[4,16] px, weights U[-1,1]), min-max mapped to [-pi/2, pi/2]; with
    ``rectangles`` 20 axis-aligned rectangles (sides U{n/32..n/8}) each add
    0.5 rad, overlaps adding.  Returned as complex128.
    """
    amp = rng.uniform(0.8, 1.0, size=(n, n))
    yy, xx = np.mgrid[0:n, 0:n].astype(np.float64)
    phase = np.zeros((n, n))
    for _ in range(8):
        mu = rng.uniform(0.0, n, size=2)
        sig = rng.uniform(4.0, 16.0)
        c = rng.uniform(-1.0, 1.0)
        phase += c * np.exp(-((yy - mu[0]) ** 2 + (xx - mu[1]) ** 2) / (2.0 * sig * sig))
    lo, hi = phase.min(), phase.max()
    if hi > lo:
        phase = (phase - lo) / (hi - lo) * math.pi - math.pi / 2.0
    else:
        phase[:] = 0.0
    if rectangles:
        smin, smax = max(1, n // 32), max(1, n // 8)
        for _ in range(20):
            r0, c0 = rng.integers(0, n, size=2)
            h, w = rng.integers(smin, smax + 1, size=2)
            phase[r0:r0 + h, c0:c0 + w] += 0.5
    return amp * np.exp(1j * phase)


def make_probe(m: int) -> np.ndarray:
    """Gaussian-apodised disc probe with quadratic phase (complex128, max |Q| = 1).

    Radius R = 10 m / 32, apodisation width s = m / 16 outside the disc,
    phase pi r^2 / R^2 about the patch centre ((m-1)/2, (m-1)/2).
    """
    c = (m - 1) / 2.0
    yy, xx = np.mgrid[0:m, 0:m].astype(np.float64)
    r = np.hypot(yy - c, xx - c)
    R = 10.0 * m / 32.0
    s = m / 16.0
    amp = np.where(r <= R, 1.0, np.exp(-((r - R) ** 2) / (2.0 * s * s)))
    kappa = math.pi / (R * R)
    return amp * np.exp(1j * kappa * r * r)


def make_scan(n: int, m: int, P: int, step: int, rng: np.random.Generator,
              jitter: int = 1) -> np.ndarray:
    """P x P raster of top-left patch offsets (row, col), int32 [P*P, 2].

    Origin centres the raster; each axis gets an integer jitter in
    [-jitter, jitter], clamped to [0, n - m].  Position k = i * P + j.
    """
    o = (n - m - (P - 1) * step) // 2
    i, j = np.meshgrid(np.arange(P), np.arange(P), indexing="ij")
    rows = o + i.ravel() * step
    cols = o + j.ravel() * step
    if jitter:
        rows = rows + rng.integers(-jitter, jitter + 1, size=rows.shape)
        cols = cols + rng.integers(-jitter, jitter + 1, size=cols.shape)
    rows = np.clip(rows, 0, n - m)
    cols = np.clip(cols, 0, n - m)
    return np.stack([rows, cols], axis=1).astype(np.int32)


def poisson_counts(dtilde: np.ndarray, peak: float | None,
                   rng: np.random.Generator) -> np.ndarray:
    """Poisson-noisy intensities for given noiseless ones.

    Scale sigma = peak / max(dtilde); returns Poisson(sigma * dtilde) / sigma,
    i.e. the paper's eta * Poisson(dtilde / eta) with eta = 1 / sigma.
    ``peak=None`` returns the input unchanged.
    """
    if peak is None:
        return np.array(dtilde, copy=True)
    sigma = float(peak) / float(np.max(dtilde))
    return rng.poisson(sigma * np.asarray(dtilde, dtype=np.float64)) / sigma


def epoch_orders(n_epochs: int, n_pos: int, rng: np.random.Generator) -> np.ndarray:
    """Uniformly random permutations of 0..n_pos-1, one per epoch (int32 [E, N])."""
    return np.stack([rng.permutation(n_pos) for _ in range(n_epochs)]).astype(np.int32)


def make_problem_inputs(cfg: ScanConfig):
    """Object z*, probe Q, scan offsets and the rng for noise/permutations.

    Returns (z_true complex128 [n,n], probe complex128 [m,m], offsets int32 [N,2],
    noise_rng, perm_rng).  Intensities are not formed here.
    """
    r_obj, r_scan, r_noise, r_perm, _ = workload_rngs(cfg.seed_id)
    z = make_object(cfg.n, r_obj, cfg.rectangles)
    q = make_probe(cfg.m)
    offs = make_scan(cfg.n, cfg.m, cfg.P, cfg.step, r_scan)
    return z, q, offs, r_noise, r_perm


@dataclasses.dataclass(frozen=True)
class BatchedRecon:
    """One reconstruction of the batched workload (64 independent reconstructions)."""

    index: int
    n: int
    m: int
    P: int
    step: int
    peak: float
    levels: int
    batch: int
    seed: int

    @property
    def n_pos(self) -> int:
        return self.P * self.P


def batched_workload(count: int = 64, seed_id: int = 4):
    """The batched workload: `count` independent reconstructions of uneven size.

    Per reconstruction: n ~ U{256, 384, 512, 768, 1024}, m ~ U{64, 128},
    P ~ U{20..80} (capped so the raster fits), step = min(10, (n-m-2)//(P-1)),
    peak photons log-uniform in [1e4, 1e5], L = 3 (m = 64) or 4 (m = 128),
    minibatch min(256, P*P).
    """
    rng = workload_rngs(seed_id)[0]
    out = []
    for i in range(count):
        n = int(rng.choice([256, 384, 512, 768, 1024]))
        m = int(rng.choice([64, 128]))
        P = int(rng.integers(20, 81))
        P = min(P, (n - m - 2) // 2 + 1)
        step = min(10, (n - m - 2) // (P - 1))
        peak = float(10 ** rng.uniform(4.0, 5.0))
        levels = 3 if m == 64 else 4
        out.append(BatchedRecon(i, n, m, P, step, peak, levels, min(256, P * P),
                                int(rng.integers(0, 2**31 - 1))))
    return out


def make_batched_inputs(spec: BatchedRecon):
    """Object, probe and scan of one reconstruction of the batched workload."""
    ss = np.random.SeedSequence(spec.seed)
    r_obj, r_scan, r_noise = [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(3)]
    z = make_object(spec.n, r_obj, rectangles=True)
    q = make_probe(spec.m)
    offs = make_scan(spec.n, spec.m, spec.P, spec.step, r_scan)
    return z, q, offs, r_noise


def poisson_counts_device(dtilde, peak: float, seed: int):
    """Device-side Poisson counts for a torch tensor of noiseless intensities
    (same model as :func:`poisson_counts`; used where the data are too large to
    draw on the host)."""
    import torch
    gen = torch.Generator(device=dtilde.device)
    gen.manual_seed(int(seed))
    sigma = float(peak) / float(dtilde.max())
    return torch.poisson(dtilde * sigma, generator=gen) / sigma


def make_objects_device(count: int, n: int, rng: np.random.Generator, device="cuda", rectangles: bool = True):
    """`count` objects of the make_object model as a complex64 torch tensor [count, n, n] on `device`.

    Same distribution as :func:`make_object` (amplitude U[0.8, 1]; 8 Gaussian
    phase bumps min-max mapped to [-pi/2, pi/2]; 20 rectangles of +0.5 rad),
    with the per-object parameters drawn from `rng` and the pixel fields
    evaluated on the device; the amplitude noise comes from a torch generator
    seeded from `rng`.  Used where many objects are needed (training sets).
    """
    import torch
    mu = rng.uniform(0.0, n, size=(count, 8, 2))
    sig = rng.uniform(4.0, 16.0, size=(count, 8))
    c = rng.uniform(-1.0, 1.0, size=(count, 8))
    smin, smax = max(1, n // 32), max(1, n // 8)
    r0 = rng.integers(0, n, size=(count, 20, 2))
    hw = rng.integers(smin, smax + 1, size=(count, 20, 2))
    gen = torch.Generator(device=device)
    gen.manual_seed(int(rng.integers(0, 2**62)))
    t = lambda a: torch.as_tensor(a, dtype=torch.float64, device=device)  # noqa: E731
    ax = torch.arange(n, dtype=torch.float64, device=device)
    s2 = 2.0 * t(sig) ** 2
    gy = torch.exp(-(ax[None, None, :] - t(mu[..., 0])[..., None]) ** 2 / s2[..., None])   # [count, 8, n]
    gx = torch.exp(-(ax[None, None, :] - t(mu[..., 1])[..., None]) ** 2 / s2[..., None])
    phase = torch.einsum("bk,bky,bkx->byx", t(c), gy, gx)
    lo = phase.amin(dim=(1, 2), keepdim=True)
    hi = phase.amax(dim=(1, 2), keepdim=True)
    span = torch.where(hi > lo, hi - lo, torch.ones_like(hi))
    phase = torch.where(hi > lo, (phase - lo) / span * math.pi - math.pi / 2.0, torch.zeros_like(phase))
    if rectangles:
        ry = ((ax[None, None, :] >= t(r0[..., 0])[..., None]) &
              (ax[None, None, :] < t(r0[..., 0] + hw[..., 0])[..., None])).to(torch.float64)
        rx = ((ax[None, None, :] >= t(r0[..., 1])[..., None]) &
              (ax[None, None, :] < t(r0[..., 1] + hw[..., 1])[..., None])).to(torch.float64)
        phase = phase + 0.5 * torch.einsum("bky,bkx->byx", ry, rx)
    amp = 0.8 + 0.2 * torch.rand((count, n, n), generator=gen, device=device, dtype=torch.float64)
    return torch.polar(amp, phase).to(torch.complex64)
