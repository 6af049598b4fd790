#!/usr/bin/env python3
"""Throughput of the fused MAGPIE step on one MI355X: diffraction patterns/s.

A step is one epoch of minibatch MAGPIE over the workload's synthetic scan
(every position once, cut into minibatches): per position gather, exit wave,
2-D FFT, modulus replacement, inverse FFT, MAGPS V-cycle and staging, and per
minibatch the fixed-order accumulation and object update.  Inputs are
resident in HBM before the timed region starts.

Prints one JSON line.  ``roofline`` covers the per-position step kernel (the
dominant kernel) from HIP events recorded around each of its launches inside
the timed region; ``cpu_baseline`` times the FP64 oracle on a bounded sample
of the same workload on the host cores.
"""

from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0


def workload_inputs(cfg_id: int):
    from synth import CONFIGS, make_problem_inputs
    cfg = CONFIGS[cfg_id]
    z_true, Q, offs, r_noise, _ = make_problem_inputs(cfg)
    return cfg, z_true.astype(np.complex64), Q.astype(np.complex64), offs, r_noise


def describe(cfg, batch, levels, alpha):
    noise = "noiseless" if cfg.peak is None else f"Poisson {cfg.peak:.0e} peak photons"
    return (f"cfg{cfg.cfg_id}: object {cfg.n}x{cfg.n} complex64, probe {cfg.m}x{cfg.m}, "
            f"{cfg.P}x{cfg.P} jittered raster step {cfg.step} ({cfg.n_pos} positions), {noise}, "
            f"{levels} levels, minibatch {batch}, alpha {alpha}")


def cpu_baseline(cfg, Q32, offs, sqrt_d32, levels, batch, alpha, seed, seconds):
    """The oracle (literal Alg 3, minibatch combination) on whole minibatches of epoch 0 until `seconds` pass."""
    import oracle
    Q = Q32.astype(np.complex128)
    u = oracle.u_rpie(Q, alpha)
    z = np.ones((cfg.n, cfg.n), dtype=np.complex128)
    order = oracle.library_permutation(seed, 0, cfg.n_pos)
    done = 0
    nb = 0
    t0 = time.perf_counter()
    while True:
        for chunk in oracle.batches(order, batch):
            z = oracle.minibatch_step(z, Q, offs, sqrt_d32, u, levels, chunk)
            done += len(chunk)
            nb += 1
            if time.perf_counter() - t0 >= seconds:
                break
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    cpu = platform.processor() or platform.machine()
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": done / dt, "unit": "patterns/s", "cores": 1, "kind": "oracle",
            "sample": f"{nb} minibatches ({done} patterns; repeated passes over the minibatches of epoch 0), FP64 NumPy single thread, "
                      f"{dt:.1f} s on {cpu} ({os.cpu_count()} host cores visible)"}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500, help="timed epochs")
    ap.add_argument("--warmup", type=int, default=20, help="untimed epochs")
    ap.add_argument("--config", type=int, default=2, choices=[1, 2, 3])
    ap.add_argument("--batch", type=int, default=None)
    ap.add_argument("--levels", type=int, default=None)
    ap.add_argument("--alpha", type=float, default=None)
    ap.add_argument("--seed", type=int, default=2504)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2504_10118_amd import Magpie
    from synth import poisson_counts

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(3)

    cfg, z_true, Q32, offs, r_noise = workload_inputs(args.config)
    batch = args.batch or cfg.batch
    levels = args.levels or cfg.levels
    alpha = cfg.alpha if args.alpha is None else args.alpha
    m, N = cfg.m, cfg.n_pos

    ctx = Magpie(cfg.n, cfg.n, m, levels, alpha, device=0)
    ctx.set_probe(Q32)
    ctx.set_positions(offs)
    dtilde = ctx.forward_model(z_true)                       # GPU forward model
    d = poisson_counts(dtilde, cfg.peak, r_noise).astype(np.float32)
    ctx.load_intensities(d, is_sqrt=False)
    ctx.set_object(np.ones((cfg.n, cfg.n), dtype=np.complex64))
    if args.warmup:
        ctx.run_epochs(args.warmup, batch, seed=args.seed + 1)
    ctx.sync()
    ctx.set_object(np.ones((cfg.n, cfg.n), dtype=np.complex64))
    ctx.epoch_index = 0
    ctx.set_timing(True)
    ctx.get_timing()                                         # reset

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.run_epochs(args.steps, batch, seed=args.seed)
    ctx.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tm = ctx.get_timing()
    phi, stat = ctx.objective()
    ctx.close()

    wall = t1 - t0
    patterns = args.steps * N
    value = patterns / wall
    bytes_per_pattern = 20 * m * m          # sqrt(d) 4 m^2 + patch read 8 m^2 + staged update 8 m^2
    step_s = tm["step_ms"] * 1e-3
    achieved = tm["positions"] * bytes_per_pattern / step_s / 1e9 if step_s > 0 else None
    n_tiles = ((cfg.n + 63) // 64) * ((cfg.n + 15) // 16)
    out = {
        "metric": "diffraction patterns/s (fused step)",
        "value": value,
        "unit": "patterns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": describe(cfg, batch, levels, alpha),
            "object": cfg.n, "probe": m, "positions": N, "levels": levels, "batch": batch,
            "step": f"one epoch = {N} patterns in {(N + batch - 1) // batch} minibatches",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": f"step_kernel<{m}, MODE_STEP>",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
            "traffic": None,
            "bytes_per_pattern": bytes_per_pattern,
            "avg_launch_us": tm["step_ms"] * 1e3 / max(1, tm["step_launches"]),
            "launches": tm["step_launches"],
        },
        "accumulate_kernel": {
            "avg_launch_us": tm["accum_ms"] * 1e3 / max(1, tm["accum_launches"]),
            "launches": tm["accum_launches"], "tiles_per_launch": n_tiles,
        },
        "kernel_share": {
            "step": step_s / wall,
            "accumulate": tm["accum_ms"] * 1e-3 / wall,
        },
        "objective_after": phi,
        "stopping_statistic_after": stat,
    }
    if not args.no_cpu_baseline:
        sqrt_d = np.sqrt(d.astype(np.float64))
        out["cpu_baseline"] = cpu_baseline(cfg, Q32, offs, sqrt_d, levels, batch, alpha, args.seed,
                                           args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
