#!/usr/bin/env python3
"""Throughput of the fused MAGPIE step on one MI355X: diffraction patterns/s.

A step is one epoch of minibatch MAGPIE over the workload's synthetic scan
(every position once, cut into minibatches): per position gather, exit wave,
2-D FFT, modulus replacement, inverse FFT, MAGPS V-cycle and staging, and per
minibatch the fixed-order accumulation and object update.  Inputs are
resident in HBM before the timed region starts.

Prints one JSON line.  ``value`` is from the timed region, which runs the
production path.  ``roofline`` covers the per-position step kernel (the
dominant kernel): the same epochs are run a second time with HIP events
recorded by each launch's own dispatch on the context's stream, and the
algorithmic bytes per launch are divided by the mean event duration.
``cpu_baseline`` times the FP64 oracle on a bounded sample of the same
workload on the host cores.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0
ROOT = os.path.dirname(os.path.abspath(__file__))


def kernel_source_hash() -> str:
    """sha256 (16 hex digits) over the sources the step and accumulation kernels are
    built from (kernels.hip, kernels.h, cmath.h): a committed profile's traffic figures
    apply while this hash is unchanged."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2504_10118_amd", "csrc")
    for name in ("cmath.h", "kernels.h", "kernels.hip"):
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(name.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(cfg_id: int, m: int, rb: int):
    """Counter-measured HBM bytes per full launch of the step kernel, from the
    committed rocprofv3 summary, if it was taken on the current sources with the
    same FFT plan (threads per transform rb)."""
    path = os.path.join(ROOT, "profiles", f"step_kernel_m{m}_cfg{cfg_id}.md")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line and line.strip().startswith(("source_sha256", "traffic_bytes_per_launch",
                                                         "traffic_fetch_bytes", "traffic_write_bytes",
                                                         "patterns_per_launch", "plan_threads_per_transform")):
                k, v = line.strip().split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("source_sha256") != kernel_source_hash() or vals.get("plan_threads_per_transform") != str(rb):
        return None
    try:
        return {"bytes_per_full_launch": float(vals["traffic_bytes_per_launch"]),
                "fetch": float(vals["traffic_fetch_bytes"]), "write": float(vals["traffic_write_bytes"]),
                "patterns_per_launch": int(vals["patterns_per_launch"]), "summary": os.path.basename(path)}
    except (KeyError, ValueError):
        return None


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


def host_cpu_name() -> str:
    cpu = platform.processor() or platform.machine()
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return cpu


def oracle_intensities(z_true, Q, offs, peak, rng):
    """sqrt of Poisson counts of the oracle's own forward model (inputs of the CPU baseline)."""
    import oracle
    from synth import poisson_counts
    dt = oracle.forward_model(np.asarray(z_true, dtype=np.complex128), np.asarray(Q, dtype=np.complex128), offs)
    return np.sqrt(poisson_counts(dt, peak, rng))


def cpu_baseline(n, Q, offs, sqrt_d, levels, batch, alpha, seed, seconds):
    """The oracle (literal Alg 3, minibatch combination) on whole minibatches of epoch 0 until `seconds` pass.

    Returns (patterns, seconds, minibatches)."""
    import oracle
    Q = np.asarray(Q, dtype=np.complex128)
    u = oracle.u_rpie(Q, alpha)
    z = np.ones((n, n), dtype=np.complex128)
    order = oracle.library_permutation(seed, 0, len(offs))
    done = 0
    nb = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        for chunk in oracle.batches(order, batch):
            z = oracle.minibatch_step(z, Q, offs, sqrt_d, u, levels, chunk)
            done += len(chunk)
            nb += 1
            if time.perf_counter() - t0 >= seconds:
                break
    return done, time.perf_counter() - t0, nb


def learned_race(n_objects: int):
    """Wall time to 1e-3 relative object error, flat vs learned start (noiseless data)."""
    import torch
    from paper_2504_10118_amd import learned as L
    params, meta = L.load_weights()
    with torch.cuda.stream(torch.cuda.Stream()):
        net = L.load_network(stream=L._current_stream())
        res = L.race(net, L.held_out_objects(n_objects), target=1e-3, log=lambda s: None)
        net.close()
    plain = [r["plain"] for r in res]
    learned = [r["learned"] for r in res]
    ok = all(p["reached"] for p in plain) and all(q["reached"] for q in learned)
    sp = [p["seconds"] / q["seconds"] for p, q in zip(plain, learned)]
    return {
        "metric": "wall time to 1e-3 relative object error, learned vs plain start",
        "unit": "ms",
        "higher_is_better": False,
        "data": (f"noiseless intensities of {n_objects} held-out objects (the 512x512 workload's own object, "
                 f"then objects of the same model from a seed outside the training set), same scan geometry, "
                 f"3 levels, minibatch 256, error checked every 10 epochs off the clock"),
        "plain_ms": [p["seconds"] * 1e3 for p in plain],
        "learned_ms": [q["seconds"] * 1e3 for q in learned],
        "plain_epochs": [p["epochs"] for p in plain],
        "learned_epochs": [q["epochs"] for q in learned],
        "learned_start_ms": [q["start_seconds"] * 1e3 for q in learned],
        "start_error_plain": [p["error_start"] for p in plain],
        "start_error_learned": [q["error_start"] for q in learned],
        "learned_kept": [q["learned_used"] for q in learned],
        "all_reached": ok,
        "speedup_median": float(np.median(sp)),
        "speedup_min": float(np.min(sp)),
        "value_plain_median_ms": float(np.median([p["seconds"] * 1e3 for p in plain])),
        "value_learned_median_ms": float(np.median([q["seconds"] * 1e3 for q in learned])),
        "learned_includes": "input map + network inference + prolongation + the two objective evaluations of the fallback",
        "training": {"samples": meta["train"], "epochs": meta["epochs"], "gpu_seconds": meta["train_seconds"],
                     "data_seconds": meta["data_seconds"], "val_loss": meta["history"][-1]["val_loss"],
                     "weights": "paper_2504_10118_amd/weights/" + os.path.basename(L.DEFAULT_WEIGHTS)},
    }


def bench_batched(args):
    """64 independent reconstructions of uneven size advanced together by the
    multi-context entry point (one launch per FFT plan / tile group per round)."""
    import torch
    from paper_2504_10118_amd import Magpie, run_epochs_multi
    from synth import batched_workload, make_batched_inputs, poisson_counts_device

    alpha = 0.5 if args.alpha is None else args.alpha
    specs = batched_workload()
    ctxs, batches, first = [], [], None
    # torch (noise) and the contexts (forward model, loads) share one stream
    st = torch.cuda.Stream()
    torch.cuda.set_stream(st)
    for sp in specs:
        z_true, Q, offs, _ = make_batched_inputs(sp)
        ctx = Magpie(sp.n, sp.n, sp.m, sp.levels, alpha, device=0, stream=st.cuda_stream)
        ctx.set_probe(Q.astype(np.complex64))
        ctx.set_positions(offs)
        if args.tuning:
            ctx.set_tuning(*(int(x) for x in args.tuning.split(",")))
        dt = torch.empty((sp.n_pos, sp.m, sp.m), dtype=torch.float32, device="cuda")
        ctx.forward_model(z_true.astype(np.complex64), out=dt)                  # GPU forward model
        ctx.load_intensities(poisson_counts_device(dt, sp.peak, sp.seed), is_sqrt=False)
        ctx.sync()
        ctx._keep_d = None
        del dt
        ctx.set_object(np.ones((sp.n, sp.n), dtype=np.complex64))
        ctxs.append(ctx)
        batches.append(args.batch or sp.batch)
        if first is None:
            first = (sp, z_true, Q, offs)
    torch.cuda.synchronize()
    total_pos = sum(sp.n_pos for sp in specs)
    bytes_per_epoch = sum(20 * sp.m * sp.m * sp.n_pos for sp in specs)

    def reset():
        for sp, c in zip(specs, ctxs):
            c.set_object(np.ones((sp.n, sp.n), dtype=np.complex64))
            c.epoch_index = 0
        torch.cuda.synchronize()

    if args.warmup:
        run_epochs_multi(ctxs, args.warmup, batches, seed=args.seed + 1)
    reset()
    t0 = time.perf_counter()
    run_epochs_multi(ctxs, args.steps, batches, seed=args.seed)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # kernel timing pass: dispatch-recorded events on every multi launch
    reset()
    ctxs[0].set_timing(True)
    ctxs[0].get_timing()
    t2 = time.perf_counter()
    run_epochs_multi(ctxs, args.steps, batches, seed=args.seed)
    tm = ctxs[0].get_timing()
    t3 = time.perf_counter()
    ctxs[0].set_timing(False)
    phis = [c.objective()[0] for c in ctxs]
    for c in ctxs:
        c.close()

    wall = t1 - t0
    step_s = tm["step_ms"] * 1e-3
    achieved = args.steps * bytes_per_epoch / step_s / 1e9 if step_s > 0 else None
    ms = [sp.m for sp in specs]
    out = {
        "metric": "diffraction patterns/s (fused step)",
        "value": args.steps * total_pos / wall,
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
            "workload": (f"cfg4: {len(specs)} independent reconstructions, objects "
                         f"{min(sp.n for sp in specs)}..{max(sp.n for sp in specs)} px, probes 64 ({ms.count(64)}) "
                         f"and 128 ({ms.count(128)}), {min(sp.n_pos for sp in specs)}..{max(sp.n_pos for sp in specs)} "
                         f"positions each ({total_pos} total), Poisson 1e4..1e5 peak photons, L = 3 (m 64) / 4 (m 128), "
                         f"minibatch min(256, N), alpha {alpha}"),
            "reconstructions": len(specs), "positions": total_pos,
            "step": f"one epoch of every reconstruction = {total_pos} patterns",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "step_multi_kernel<64|128, MODE_STEP>",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
            "traffic": None,
            "bytes_per_pattern": "20 m^2",
            "avg_launch_us": tm["step_ms"] * 1e3 / max(1, tm["step_launches"]),
            "launches": tm["step_launches"],
        },
        "accumulate_kernel": {
            "avg_launch_us": tm["accum_ms"] * 1e3 / max(1, tm["accum_launches"]),
            "launches": tm["accum_launches"],
        },
        "event_pass": {"ms_per_step": (t3 - t2) * 1e3 / args.steps,
                       "step_share": step_s / (t3 - t2), "accumulate_share": tm["accum_ms"] * 1e-3 / (t3 - t2)},
        "objective_after_median": float(np.median(phis)),
    }
    if not args.no_cpu_baseline:
        sp, z_true, Q, offs = first
        sqrt_d = oracle_intensities(z_true, Q, offs, sp.peak, np.random.default_rng(sp.seed))
        done, dt, nb = cpu_baseline(sp.n, Q, offs, sqrt_d, sp.levels, args.batch or sp.batch, alpha, args.seed,
                                    args.cpu_seconds)
        out["cpu_baseline"] = {
            "value": done / dt, "unit": "patterns/s", "cores": 1, "kind": "oracle",
            "sample": f"reconstruction 0 (object {sp.n}, probe {sp.m}, {sp.n_pos} positions): {nb} minibatches "
                      f"({done} patterns) of epoch 0, FP64 NumPy single thread, {dt:.1f} s on {host_cpu_name()} "
                      f"({os.cpu_count()} host cores visible)"}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500, help="timed epochs")
    ap.add_argument("--warmup", type=int, default=20, help="untimed epochs")
    ap.add_argument("--config", type=int, default=2, choices=[1, 2, 3, 4],
                    help="1-3: one reconstruction; 4: 64 independent reconstructions of uneven size")
    ap.add_argument("--batch", type=int, default=None)
    ap.add_argument("--levels", type=int, default=None)
    ap.add_argument("--alpha", type=float, default=None)
    ap.add_argument("--seed", type=int, default=2504)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default FFT plan and tile height")
    ap.add_argument("--tuning", type=str, default="",
                    help="RB,TH: use this FFT plan (threads per transform) and tile height instead of the autotuner")
    ap.add_argument("--race-objects", type=int, default=4,
                    help="held-out objects of the learned-vs-plain time-to-1e-3 race (0: skip)")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="run one plain device-to-device copy of this many MiB first (HBM counter calibration)")
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

    if args.copy_calibration_mb:
        nbytes = args.copy_calibration_mb << 20
        src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if args.config == 4:
        return bench_batched(args)

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
    torch.cuda.synchronize()
    tl0 = time.perf_counter()
    ctx.load_intensities(d, is_sqrt=False)                   # host -> device, checked (synchronises)
    load_s = time.perf_counter() - tl0
    ctx.set_object(np.ones((cfg.n, cfg.n), dtype=np.complex64))
    tuning = None
    if args.tuning:
        rb, th = (int(x) for x in args.tuning.split(","))
        ctx.set_tuning(rb, th)
        tuning = {"threads_per_transform": rb, "tile_rows": th, "source": "--tuning"}
    elif not args.no_autotune:
        rb, th, su, au = ctx.autotune(batch)             # the library's own autotuner, on this data
        tuning = {"threads_per_transform": rb, "tile_rows": th, "trial_step_us": su, "trial_accumulate_us": au}
    if args.warmup:
        ctx.run_epochs(args.warmup, batch, seed=args.seed + 1)
    ctx.sync()
    # timed region: the production path (no per-kernel events)
    ctx.set_object(np.ones((cfg.n, cfg.n), dtype=np.complex64))
    ctx.epoch_index = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.run_epochs(args.steps, batch, seed=args.seed)
    ctx.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    phi, stat = ctx.objective()
    tr0 = time.perf_counter()
    ctx.get_object()                                         # device -> host read-back of the object
    readback_s = time.perf_counter() - tr0

    # kernel timing: the same epochs again, every launch bracketed by HIP events
    # that its own dispatch records on the context's stream
    ctx.set_object(np.ones((cfg.n, cfg.n), dtype=np.complex64))
    ctx.epoch_index = 0
    ctx.set_timing(True)
    ctx.get_timing()                                         # reset
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    ctx.run_epochs(args.steps, batch, seed=args.seed)
    tm = ctx.get_timing()                                    # synchronises
    t3 = time.perf_counter()
    ctx_rb, ctx_tile_rows = ctx.get_tuning()
    ctx.close()

    wall = t1 - t0
    patterns = args.steps * N
    value = patterns / wall
    bytes_per_pattern = 20 * m * m          # sqrt(d) 4 m^2 + patch read 8 m^2 + staged update 8 m^2
    step_s = tm["step_ms"] * 1e-3
    achieved = tm["positions"] * bytes_per_pattern / step_s / 1e9 if step_s > 0 else None
    th_used = ctx_tile_rows
    n_tiles = ((cfg.n + 63) // 64) * ((cfg.n + th_used - 1) // th_used)
    traffic = stored_traffic(args.config, m, ctx_rb) if batch == cfg.batch and levels == cfg.levels else None
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
            "tuning": tuning,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": f"step_kernel<{m}, {ctx_rb}, MODE_STEP>",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
            "traffic": None if traffic is None else traffic["bytes_per_full_launch"],
            "traffic_detail": traffic,
            "algorithmic_bytes_per_full_launch": bytes_per_pattern * min(batch, N),
            "bytes_per_pattern": bytes_per_pattern,
            "avg_launch_us": tm["step_ms"] * 1e3 / max(1, tm["step_launches"]),
            "launches": tm["step_launches"],
        },
        "accumulate_kernel": {
            "avg_launch_us": tm["accum_ms"] * 1e3 / max(1, tm["accum_launches"]),
            "launches": tm["accum_launches"], "tiles_per_launch": n_tiles,
        },
        "event_pass": {
            "note": "second pass over the same epochs with per-launch HIP events (slower: events serialise dispatch)",
            "ms_per_step": (t3 - t2) * 1e3 / args.steps,
            "step_share": step_s / (t3 - t2),
            "accumulate_share": tm["accum_ms"] * 1e-3 / (t3 - t2),
        },
        "pcie_inclusive": {
            "note": "the same job with the host-buffer boundary crossings added: the measured intensities "
                    "uploaded (and square-rooted, re-laid out, checked) by magpie_load_intensities, and the "
                    "object read back; not the value",
            "value": patterns / (wall + load_s + readback_s),
            "load_ms": load_s * 1e3, "readback_ms": readback_s * 1e3},
        "objective_after": phi,
        "stopping_statistic_after": stat,
    }
    if args.race_objects > 0 and args.config == 2:
        out["learned_race"] = learned_race(args.race_objects)
    if not args.no_cpu_baseline:
        sqrt_d = oracle_intensities(z_true, Q32, offs, cfg.peak, np.random.default_rng(args.seed))
        done, dt, nb = cpu_baseline(cfg.n, Q32, offs, sqrt_d, levels, batch, alpha, args.seed, args.cpu_seconds)
        out["cpu_baseline"] = {
            "value": done / dt, "unit": "patterns/s", "cores": 1, "kind": "oracle",
            "sample": f"{nb} minibatches of {batch} ({done} patterns; passes over the minibatches of epoch 0) of "
                      f"the same workload, FP64 NumPy single thread, {dt:.1f} s on {host_cpu_name()} "
                      f"({os.cpu_count()} host cores visible)"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
