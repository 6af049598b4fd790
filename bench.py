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
algorithmic bytes of a full launch (one whole minibatch) are divided by the
mean duration of the full launches; ``roofline.pipeline`` divides the whole
epoch's algorithmic bytes (patterns, staging and object updates) by the timed
wall time.  The default run (the 512 x 512 workload) also reports the
1024 x 1024 workload and the 64-reconstruction workload as extra keys, and
``cpu_baseline`` times the FP64 oracle on bounded samples of the same workloads
on the host cores (all usable cores, and one).
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
BATCHED = "64-reconstructions"   # 64 independent reconstructions of uneven size
ROOT = os.path.dirname(os.path.abspath(__file__))
ACC_TILE_W = 32           # accumulation tile width of the library (columns)


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


def stored_traffic(workload: str, m: int, rb: int, kind: str = "step"):
    """Counter-measured HBM bytes per launch of the step kernel (full launches) or of the
    accumulation kernel (kind "accumulate", mean over its launches), from the committed
    rocprofv3 summary, if it was taken on the current kernel sources (and, for the step
    kernel, with the same FFT plan: threads per transform rb)."""
    from synth import WORKLOADS
    n = WORKLOADS[workload].n
    name = f"step_kernel_m{m}_n{n}.md" if kind == "step" else f"accumulate_kernel_n{n}.md"
    path = os.path.join(ROOT, "profiles", name)
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
    if vals.get("source_sha256") != kernel_source_hash():
        return None
    if kind == "step" and vals.get("plan_threads_per_transform") != str(rb):
        return None
    try:
        out = {"bytes_per_launch": float(vals["traffic_bytes_per_launch"]),
               "fetch": float(vals["traffic_fetch_bytes"]), "write": float(vals["traffic_write_bytes"]),
               "summary": os.path.basename(path)}
        if kind == "step":
            out["patterns_per_launch"] = int(vals["patterns_per_launch"])
        return out
    except (KeyError, ValueError):
        return None


def workload_inputs(workload: str):
    from synth import WORKLOADS, make_problem_inputs
    cfg = WORKLOADS[workload]
    z_true, Q, offs, r_noise, _ = make_problem_inputs(cfg)
    return cfg, z_true.astype(np.complex64), Q.astype(np.complex64), offs, r_noise


def describe(cfg, batch, levels, alpha):
    noise = "noiseless" if cfg.peak is None else f"Poisson {cfg.peak:.0e} peak photons"
    return (f"object {cfg.n}x{cfg.n} complex64, probe {cfg.m}x{cfg.m}, "
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


def usable_cores() -> int:
    """Host cores this process may use, capped at 16 (the host share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def coverage_per_batch(offs, n: int, m: int, batch: int, seed: int, epochs: int):
    """(mean, list) of the number of distinct object pixels a minibatch covers (cov(B)),
    over the minibatches of the first `epochs` epochs of the library's permutations."""
    import oracle
    covs = []
    for e in range(epochs):
        order = oracle.library_permutation(seed, e, len(offs))
        for b in oracle.batches(order, batch):
            mask = np.zeros((n, n), dtype=bool)
            for k in b:
                r, c = offs[k]
                mask[r:r + m, c:c + m] = True
            covs.append(int(mask.sum()))
    return float(np.mean(covs)), covs


# ---------------------------------------------------------------------------
# CPU baseline: the FP64 oracle, unchanged, on whole minibatches of epoch 0
# ---------------------------------------------------------------------------
_CPU = {}


def _cpu_minibatch(args):
    import oracle
    i, = args
    d = _CPU
    chunk = d["chunks"][i % len(d["chunks"])]
    oracle.minibatch_step(d["z"], d["Q"], d["offs"], d["sqrt_d"], d["u"], d["levels"], chunk)
    return len(chunk)


def cpu_baseline(n, Q, offs, sqrt_d, levels, batch, alpha, seed, seconds, workers=1):
    """The oracle (literal Alg 3, minibatch combination) on whole minibatches of epoch 0
    from the flat object, for about `seconds` of wall time, on `workers` processes each
    running the unchanged oracle on its own minibatches.

    Returns (patterns, seconds, minibatches)."""
    import oracle
    Qd = np.asarray(Q, dtype=np.complex128)
    order = oracle.library_permutation(seed, 0, len(offs))
    _CPU.update(z=np.ones((n, n), dtype=np.complex128), Q=Qd, offs=offs, sqrt_d=sqrt_d,
                u=oracle.u_rpie(Qd, alpha), levels=levels, chunks=oracle.batches(order, batch))
    if workers <= 1:
        done = nb = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < seconds:
            done += _cpu_minibatch((nb,))
            nb += 1
        return done, time.perf_counter() - t0, nb
    import multiprocessing as mp
    ctx = mp.get_context("fork")
    with ctx.Pool(workers) as pool:
        pool.map(_cpu_minibatch, [(i,) for i in range(workers)])       # warm the workers
        # size the sample from a timed round: one minibatch per worker
        t0 = time.perf_counter()
        done = sum(pool.map(_cpu_minibatch, [(i,) for i in range(workers)]))
        t_round = time.perf_counter() - t0
        rounds = max(1, int(seconds / max(t_round, 1e-3)) - 1)
        nb = workers * (rounds + 1)
        done += sum(pool.map(_cpu_minibatch, [(i,) for i in range(workers, workers * (rounds + 1))]))
        dt = time.perf_counter() - t0
    return done, dt, nb


def cpu_baselines(workload, seconds_multi, seconds_single, seed):
    """Oracle patterns/s on a workload: all usable cores and one core."""
    import oracle
    from synth import WORKLOADS, make_problem_inputs, poisson_counts
    cfg = WORKLOADS[workload]
    z, Q, offs, r_noise, _ = make_problem_inputs(cfg)
    Q32 = Q.astype(np.complex64)
    d = oracle.forward_model(z.astype(np.complex64).astype(np.complex128), Q32.astype(np.complex128), offs)
    sd = np.sqrt(poisson_counts(d, cfg.peak, r_noise) if cfg.peak else d).astype(np.float32).astype(np.float64)
    out = {}
    for key, workers, secs in (("all_cores", usable_cores(), seconds_multi), ("one_core", 1, seconds_single)):
        done, dt, nb = cpu_baseline(cfg.n, Q32, offs, sd, cfg.levels, cfg.batch, cfg.alpha, seed, secs, workers)
        out[key] = {"value": done / dt, "cores": workers, "patterns": done, "minibatches": nb, "seconds": dt}
    return cfg, out


# ---------------------------------------------------------------------------
# GPU runs
# ---------------------------------------------------------------------------
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


def run_single(workload, steps, warmup, seed, batch=None, levels=None, alpha=None, tuning="", autotune=True,
               device_noise=False):
    """One reconstruction of the named workload: timed epochs (production path), then the
    same epochs with per-launch events.  Returns a dict of figures."""
    import torch
    from paper_2504_10118_amd import Magpie
    from synth import poisson_counts, poisson_counts_device

    cfg, z_true, Q32, offs, r_noise = workload_inputs(workload)
    batch = batch or cfg.batch
    levels = levels or cfg.levels
    alpha = cfg.alpha if alpha is None else alpha
    m, N, n = cfg.m, cfg.n_pos, cfg.n
    B = min(batch, N)

    ctx = Magpie(n, n, m, levels, alpha, device=0)
    ctx.set_probe(Q32)
    ctx.set_positions(offs)
    if device_noise:
        dt = torch.empty((N, m, m), dtype=torch.float32, device="cuda")
        ctx.forward_model(z_true, out=dt)                    # GPU forward model
        torch.cuda.synchronize()
        d = poisson_counts_device(dt, cfg.peak, 1000 + cfg.seed_id) if cfg.peak else dt
        torch.cuda.synchronize()
        tl0 = time.perf_counter()
        ctx.load_intensities(d, is_sqrt=False)
        ctx.sync()
        load_s = time.perf_counter() - tl0
        ctx._keep_d = None
        del dt, d
    else:
        dtilde = ctx.forward_model(z_true)                   # GPU forward model
        d = (poisson_counts(dtilde, cfg.peak, r_noise) if cfg.peak else dtilde).astype(np.float32)
        torch.cuda.synchronize()
        tl0 = time.perf_counter()
        ctx.load_intensities(d, is_sqrt=False)               # host -> device, checked (synchronises)
        load_s = time.perf_counter() - tl0
    ctx.set_object(np.ones((n, n), dtype=np.complex64))
    tune = None
    if tuning:
        rb, th = (int(x) for x in tuning.split(","))
        ctx.set_tuning(rb, th)
        tune = {"threads_per_transform": rb, "tile_rows": th, "source": "--tuning"}
    elif autotune:
        rb, th, su, au = ctx.autotune(batch)             # the library's own autotuner, on this data
        tune = {"threads_per_transform": rb, "tile_rows": th, "trial_step_us": su, "trial_accumulate_us": au}
    if warmup:
        ctx.run_epochs(warmup, batch, seed=seed + 1)
    ctx.sync()
    # timed region: the production path (no per-kernel events)
    ctx.set_object(np.ones((n, n), dtype=np.complex64))
    ctx.epoch_index = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.run_epochs(steps, batch, seed=seed)
    ctx.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    phi, stat = ctx.objective()
    tr0 = time.perf_counter()
    ctx.get_object()                                         # device -> host read-back of the object
    readback_s = time.perf_counter() - tr0

    # kernel timing: the same epochs again, every launch bracketed by HIP events
    # that its own dispatch records on the context's stream
    ctx.set_object(np.ones((n, n), dtype=np.complex64))
    ctx.epoch_index = 0
    ctx.set_timing(True)
    ctx.get_timing()                                         # reset
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    ctx.run_epochs(steps, batch, seed=seed)
    step_us, step_pos = ctx.launch_times(0)                  # synchronises
    acc_us, _ = ctx.launch_times(1)
    tm = ctx.get_timing()                                    # sums; resets
    t3 = time.perf_counter()
    rb_used, th_used = ctx.get_tuning()
    ctx.close()

    wall = t1 - t0
    patterns = steps * N
    nb = (N + B - 1) // B
    full = step_pos == B
    step_full_us = float(step_us[full].mean())
    bytes_per_pattern = 20 * m * m          # sqrt(d) 4 m^2 + patch read 8 m^2 + staged update 8 m^2
    achieved = bytes_per_pattern * B / (step_full_us * 1e-6) / 1e9
    cov_mean, covs = coverage_per_batch(offs, n, m, B, seed, min(steps, 4))
    # accumulation: full launches are every minibatch of B positions (all but a short last one)
    acc_full = np.array([(i % nb) < N // B for i in range(len(acc_us))])
    cov_full = float(np.mean([c for i, c in enumerate(covs) if (i % nb) < N // B]))
    acc_full_us = float(acc_us[acc_full].mean())
    acc_bytes = B * 8 * m * m + 16 * cov_full
    epoch_bytes = N * bytes_per_pattern + 16 * cov_mean * nb
    # the accumulation runs over the box of tiles some window reaches
    bx = (offs[:, 1].max() + m - 1) // ACC_TILE_W - offs[:, 1].min() // ACC_TILE_W + 1
    by = (offs[:, 0].max() + m - 1) // th_used - offs[:, 0].min() // th_used + 1
    n_tiles = int(bx * by)
    return {
        "cfg": cfg, "batch": batch, "levels": levels, "alpha": alpha, "N": N, "m": m, "n": n, "B": B,
        "tuning": tune, "rb": rb_used, "th": th_used,
        "value": patterns / wall, "wall": wall, "ms_per_step": wall * 1e3 / steps,
        "step_full_us": step_full_us, "step_mean_us": float(step_us.mean()), "step_launches": len(step_us),
        "achieved": achieved, "bytes_per_pattern": bytes_per_pattern,
        "acc_full_us": acc_full_us, "acc_launches": len(acc_us), "acc_bytes": acc_bytes, "n_tiles": n_tiles,
        "cov_mean": cov_mean, "epoch_bytes": epoch_bytes,
        "event_wall": t3 - t2, "step_ms_sum": tm["step_ms"], "acc_ms_sum": tm["accum_ms"],
        "load_s": load_s, "readback_s": readback_s, "phi": phi, "stat": stat,
    }


def single_summary(r, steps):
    """The compact figures of a single-reconstruction run (extra keys)."""
    pipe = r["epoch_bytes"] * steps / r["wall"] / 1e9
    return {
        "workload": describe(r["cfg"], r["batch"], r["levels"], r["alpha"]),
        "value": r["value"], "unit": "patterns/s", "ms_per_step": r["ms_per_step"], "steps": steps,
        "step_kernel_full_launch_us": r["step_full_us"], "step_kernel_frac": r["achieved"] / HBM_PEAK_GBS,
        "accumulate_full_launch_us": r["acc_full_us"],
        "accumulate_frac": r["acc_bytes"] / (r["acc_full_us"] * 1e-6) / 1e9 / HBM_PEAK_GBS,
        "pipeline_frac": pipe / HBM_PEAK_GBS, "tuning": [r["rb"], r["th"]],
    }


def bench_batched(steps, warmup, seed, batch=None, alpha=None, tuning=""):
    """64 independent reconstructions of uneven size advanced together by the
    multi-context entry point (one launch per FFT plan / tile group per round)."""
    import torch
    from paper_2504_10118_amd import Magpie, run_epochs_multi
    from synth import batched_workload, make_batched_inputs, poisson_counts_device

    alpha = 0.5 if alpha is None else alpha
    specs = batched_workload()
    ctxs, batches = [], []
    # torch (noise) and the contexts (forward model, loads) share one stream
    st = torch.cuda.Stream()
    torch.cuda.set_stream(st)
    for sp in specs:
        z_true, Q, offs, _ = make_batched_inputs(sp)
        ctx = Magpie(sp.n, sp.n, sp.m, sp.levels, alpha, device=0, stream=st.cuda_stream)
        ctx.set_probe(Q.astype(np.complex64))
        ctx.set_positions(offs)
        if tuning:
            ctx.set_tuning(*(int(x) for x in tuning.split(",")))
        dt = torch.empty((sp.n_pos, sp.m, sp.m), dtype=torch.float32, device="cuda")
        ctx.forward_model(z_true.astype(np.complex64), out=dt)                  # GPU forward model
        ctx.load_intensities(poisson_counts_device(dt, sp.peak, sp.seed), is_sqrt=False)
        ctx.sync()
        ctx._keep_d = None
        del dt
        ctx.set_object(np.ones((sp.n, sp.n), dtype=np.complex64))
        ctxs.append(ctx)
        batches.append(batch or sp.batch)
    torch.cuda.synchronize()
    total_pos = sum(sp.n_pos for sp in specs)
    bytes_per_epoch = sum(20 * sp.m * sp.m * sp.n_pos for sp in specs)

    def reset():
        for sp, c in zip(specs, ctxs):
            c.set_object(np.ones((sp.n, sp.n), dtype=np.complex64))
            c.epoch_index = 0
        torch.cuda.synchronize()

    if warmup:
        run_epochs_multi(ctxs, warmup, batches, seed=seed + 1)
    reset()
    t0 = time.perf_counter()
    run_epochs_multi(ctxs, steps, batches, seed=seed)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # kernel timing pass: dispatch-recorded events on every multi launch
    reset()
    ctxs[0].set_timing(True)
    ctxs[0].get_timing()
    t2 = time.perf_counter()
    run_epochs_multi(ctxs, steps, batches, seed=seed)
    tm = ctxs[0].get_timing()
    t3 = time.perf_counter()
    ctxs[0].set_timing(False)
    phis = [c.objective()[0] for c in ctxs]
    # the same epochs through the work-queue launch (flag PERSISTENT: one launch per FFT
    # plan and chunk of epochs), after one untimed epoch
    from paper_2504_10118_amd import PERSISTENT
    for c in ctxs:
        c.set_flags(PERSISTENT)
    run_epochs_multi(ctxs, 1, batches, seed=seed + 2)
    reset()
    t4 = time.perf_counter()
    run_epochs_multi(ctxs, steps, batches, seed=seed)
    torch.cuda.synchronize()
    t5 = time.perf_counter()
    phis_q = [c.objective()[0] for c in ctxs]
    for c in ctxs:
        c.set_flags(0)
    for c in ctxs:
        c.close()
    torch.cuda.set_stream(torch.cuda.default_stream())
    wall = t1 - t0
    step_s = tm["step_ms"] * 1e-3
    achieved = steps * bytes_per_epoch / step_s / 1e9 if step_s > 0 else None
    ms = [sp.m for sp in specs]
    return {
        "specs": specs, "total_pos": total_pos, "value": steps * total_pos / wall, "wall": wall,
        "ms_per_step": wall * 1e3 / steps, "achieved": achieved,
        "step_launch_us": tm["step_ms"] * 1e3 / max(1, tm["step_launches"]), "step_launches": tm["step_launches"],
        "acc_launch_us": tm["accum_ms"] * 1e3 / max(1, tm["accum_launches"]), "acc_launches": tm["accum_launches"],
        "event_wall": t3 - t2, "step_ms_sum": tm["step_ms"], "acc_ms_sum": tm["accum_ms"],
        "phi_median": float(np.median(phis)), "alpha": alpha,
        "queue": {"value": steps * total_pos / (t5 - t4), "ms_per_step": (t5 - t4) * 1e3 / steps,
                  "objectives_equal": bool(phis_q == phis)},
        "workload": (f"{len(specs)} independent reconstructions, objects "
                     f"{min(sp.n for sp in specs)}..{max(sp.n for sp in specs)} px, probes 64 ({ms.count(64)}) "
                     f"and 128 ({ms.count(128)}), {min(sp.n_pos for sp in specs)}..{max(sp.n_pos for sp in specs)} "
                     f"positions each ({total_pos} total), Poisson 1e4..1e5 peak photons, L = 3 (m 64) / 4 "
                     f"(m 128), minibatch min(256, N), alpha {alpha}"),
    }


def batched_summary(r, steps):
    return {"workload": r["workload"], "value": r["value"], "unit": "patterns/s", "ms_per_step": r["ms_per_step"],
            "steps": steps, "step_kernel_frac": (r["achieved"] / HBM_PEAK_GBS) if r["achieved"] else None,
            "step_launch_us": r["step_launch_us"], "accumulate_launch_us": r["acc_launch_us"],
            "step_kernel_frac_note": "algorithmic bytes over the summed durations of the step launches, "
                                     "which overlap across the concurrent plan partitions (understates)",
            "work_queue": r["queue"]}


def base_line(metric_value, steps, warmup, ms_per_step):
    return {
        "metric": "diffraction patterns/s (fused step)",
        "value": metric_value,
        "unit": "patterns/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
    }


def cpu_line(args, workload):
    cfg, res = cpu_baselines(workload, args.cpu_seconds, args.cpu_seconds_single, args.seed)
    a, o = res["all_cores"], res["one_core"]
    return cfg, {
        "value": a["value"], "unit": "patterns/s", "cores": a["cores"], "kind": "oracle",
        "sample": (f"{a['minibatches']} minibatches of {cfg.batch} ({a['patterns']} patterns) of epoch 0 of the "
                   f"{cfg.n}x{cfg.n} workload from the flat object, the unchanged FP64 NumPy oracle (literal Alg 3) "
                   f"in {a['cores']} processes (one minibatch each at a time), {a['seconds']:.1f} s on "
                   f"{host_cpu_name()} ({os.cpu_count()} host cores visible)"),
        "one_core": {"value": o["value"], "cores": 1, "patterns": o["patterns"], "seconds": o["seconds"]},
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500, help="timed epochs")
    ap.add_argument("--warmup", type=int, default=20, help="untimed epochs")
    ap.add_argument("--workload", default="512x512", choices=["128x128", "512x512", "1024x1024", BATCHED],
                    help="one reconstruction of the named object size, or 64 independent reconstructions "
                         "of uneven size")
    ap.add_argument("--batch", type=int, default=None)
    ap.add_argument("--levels", type=int, default=None)
    ap.add_argument("--alpha", type=float, default=None)
    ap.add_argument("--seed", type=int, default=2504)
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="all-core oracle sample (per workload)")
    ap.add_argument("--cpu-seconds-single", type=float, default=6.0, help="one-core oracle sample (per workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra-workloads", action="store_true",
                    help="default run: skip the 1024x1024 and 64-reconstruction extra keys")
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
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    # The oracle's CPU baselines run first, before anything initialises the GPU or
    # loads the HIP library: their worker processes are forked and must not inherit
    # GPU state.
    default_run = args.workload == "512x512" and not args.batch and not args.levels and args.alpha is None
    cpu = {}
    if not args.no_cpu_baseline and args.workload != BATCHED:
        _, cpu["main"] = cpu_line(args, args.workload)
        if default_run and not args.no_extra_workloads:
            for wl in ("128x128", "1024x1024"):
                c, line = cpu_line(args, wl)
                cpu[wl] = {"value": line["value"], "cores": line["cores"], "one_core": line["one_core"]["value"],
                            "workload": describe(c, c.batch, c.levels, c.alpha), "n": c.n}

    import torch
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

    if args.workload == BATCHED:
        r = bench_batched(args.steps, args.warmup, args.seed, args.batch, args.alpha, args.tuning)
        out = base_line(r["value"], args.steps, args.warmup, r["ms_per_step"])
        out["config"] = {"workload": r["workload"], "reconstructions": len(r["specs"]), "positions": r["total_pos"],
                         "step": f"one epoch of every reconstruction = {r['total_pos']} patterns"}
        out["roofline"] = {
            "bound": "hbm", "kernel": "step_multi_kernel<64|128, MODE_STEP>", "achieved": r["achieved"],
            "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": (r["achieved"] / HBM_PEAK_GBS) if r["achieved"] else None, "traffic": None,
            "bytes_per_pattern": "20 m^2", "avg_launch_us": r["step_launch_us"], "launches": r["step_launches"]}
        out["accumulate_kernel"] = {"avg_launch_us": r["acc_launch_us"], "launches": r["acc_launches"]}
        out["event_pass"] = {"ms_per_step": r["event_wall"] * 1e3 / args.steps,
                             "step_share": r["step_ms_sum"] * 1e-3 / r["event_wall"],
                             "accumulate_share": r["acc_ms_sum"] * 1e-3 / r["event_wall"]}
        out["objective_after_median"] = r["phi_median"]
        out["work_queue"] = dict(r["queue"], note="the same epochs with the flag PERSISTENT: one work-queue "
                                 "launch per FFT plan and chunk of epochs instead of launches per round")
        print(json.dumps(out), flush=True)
        return

    r = run_single(args.workload, args.steps, args.warmup, args.seed, args.batch, args.levels, args.alpha,
                   args.tuning, not args.no_autotune)
    cfg, m, B = r["cfg"], r["m"], r["B"]
    traffic = stored_traffic(args.workload, m, r["rb"]) if r["batch"] == cfg.batch and r["levels"] == cfg.levels \
        else None
    pipe_achieved = r["epoch_bytes"] * args.steps / r["wall"] / 1e9
    out = base_line(r["value"], args.steps, args.warmup, r["ms_per_step"])
    out["config"] = {
        "workload": describe(cfg, r["batch"], r["levels"], r["alpha"]),
        "object": cfg.n, "probe": m, "positions": r["N"], "levels": r["levels"], "batch": r["batch"],
        "step": f"one epoch = {r['N']} patterns in {(r['N'] + B - 1) // B} minibatches",
        "tuning": r["tuning"],
    }
    out["roofline"] = {
        "bound": "hbm",
        "kernel": f"step_kernel<{m}, {r['rb']}, MODE_STEP>",
        "achieved": r["achieved"],
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": r["achieved"] / HBM_PEAK_GBS,
        "traffic": None if traffic is None else traffic["bytes_per_launch"],
        "traffic_detail": traffic,
        "algorithmic_bytes_per_full_launch": r["bytes_per_pattern"] * B,
        "bytes_per_pattern": r["bytes_per_pattern"],
        "avg_launch_us": r["step_full_us"],
        "avg_launch_us_note": f"mean over the full launches ({B} patterns); all launches incl. the short last "
                              f"minibatch: {r['step_mean_us']:.3f} us",
        "launches": r["step_launches"],
        "pipeline": {
            "note": "whole epoch: N * 20 m^2 (sqrt(d), patch, staged update) + 16 B per covered pixel per "
                    "minibatch (object read + write), measured coverage, over the timed wall time",
            "bytes_per_epoch": r["epoch_bytes"], "achieved": pipe_achieved, "frac": pipe_achieved / HBM_PEAK_GBS,
            "bytes_per_pattern": r["epoch_bytes"] / r["N"], "covered_pixels_per_minibatch": r["cov_mean"]},
    }
    acc_traffic = stored_traffic(args.workload, m, r["rb"], "accumulate") \
        if r["batch"] == cfg.batch and r["th"] == 8 else None
    out["accumulate_kernel"] = {
        "avg_launch_us": r["acc_full_us"], "launches": r["acc_launches"], "tiles_per_launch": r["n_tiles"],
        "traffic_per_launch_all": None if acc_traffic is None else acc_traffic["bytes_per_launch"],
        "traffic_detail": acc_traffic,
        "tile": f"{ACC_TILE_W}x{r['th']}",
        "algorithmic_bytes_per_full_launch": r["acc_bytes"],
        "frac": r["acc_bytes"] / (r["acc_full_us"] * 1e-6) / 1e9 / HBM_PEAK_GBS,
        "bytes_note": "B * 8 m^2 staged reads + 16 B per covered pixel (object read + write)"}
    out["event_pass"] = {
        "note": "second pass over the same epochs with per-launch HIP events (slower: events serialise dispatch)",
        "ms_per_step": r["event_wall"] * 1e3 / args.steps,
        "step_share": r["step_ms_sum"] * 1e-3 / r["event_wall"],
        "accumulate_share": r["acc_ms_sum"] * 1e-3 / r["event_wall"],
    }
    out["pcie_inclusive"] = {
        "note": "the same job with the host-buffer boundary crossings added: the measured intensities "
                "uploaded (and square-rooted, re-laid out, checked) by magpie_load_intensities, and the "
                "object read back; not the value",
        "value": args.steps * r["N"] / (r["wall"] + r["load_s"] + r["readback_s"]),
        "load_ms": r["load_s"] * 1e3, "readback_ms": r["readback_s"] * 1e3}
    out["objective_after"] = r["phi"]
    out["stopping_statistic_after"] = r["stat"]
    if default_run and not args.no_extra_workloads:
        r3 = run_single("1024x1024", 20, 5, args.seed, device_noise=True)
        out["workload_1024x1024"] = single_summary(r3, 20)
        out["workload_1024x1024"]["noise"] = "Poisson counts drawn on the device (same model)"
        r4 = bench_batched(8, 2, args.seed)
        out["workload_64_reconstructions"] = batched_summary(r4, 8)
        torch.cuda.synchronize()
    if args.race_objects > 0 and args.workload == "512x512":
        out["learned_race"] = learned_race(args.race_objects)
    if "main" in cpu:
        out["cpu_baseline"] = cpu["main"]
        others = {f"workload_{wl}": v for wl, v in cpu.items() if wl != "main"}
        if others:
            out["cpu_baseline"]["other_workloads"] = others
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
