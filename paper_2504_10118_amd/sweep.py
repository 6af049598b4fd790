"""Parameter sweeps with the library's kernels on a synthetic workload: the number
of grids L = 1 (the rPIE update) .. log2(m) + 1 (the study of Sec. 5.1), the
noise level (Sec. 5.2: d = eta * Poisson(d~ / eta)) and the overlap ratio of
adjacent scans (Sec. 5.3), with minibatches and the synthetic probe.

For every overlap ratio, noise level, regularisation weight alpha and number of
grids L the sweep runs `epochs` epochs from the flat start and records, after each epoch,
the objective Phi (eq. 2.1) and the stopping statistic (the mean gradient norm
of Sec. 5), and at log-spaced epochs the relative object error (minimum over a
global phase, masked to the illuminated area) and the paper's magnitude error
||(|z| - |z*|)|| / ||z*||.  It notes the first epoch at which the statistic
falls below `tol` and the GPU wall time of the epochs (error checks and
objective passes off the clock).

Run ``python -m paper_2504_10118_amd.sweep --help``.
"""

from __future__ import annotations

import argparse
import dataclasses
import json
import os
import time

import numpy as np

from .magpie import Magpie


def checkpoints(epochs: int) -> list[int]:
    """1, 2, 3, 5, 10, 20, 30, 50, ... up to and including `epochs`."""
    out = []
    dec = 1
    while dec <= epochs:
        for f in (1, 2, 3, 5):
            if f * dec <= epochs:
                out.append(f * dec)
        dec *= 10
    if not out or out[-1] != epochs:
        out.append(epochs)
    return sorted(set(out))


def object_errors(z, z_true, mask) -> tuple[float, float]:
    """(relative error after removing the global phase, relative magnitude error), both on the mask."""
    a = np.asarray(z, dtype=np.complex128)[mask]
    b = np.asarray(z_true, dtype=np.complex128)[mask]
    ip = np.vdot(a, b)
    ph = ip / abs(ip) if ip != 0 else 1.0
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(ph * a - b) / nb), float(np.linalg.norm(np.abs(a) - np.abs(b)) / nb)


def scaled_error(a, b, mask=None) -> float:
    """min over complex c of ||c a - b|| / ||b|| (on the mask): the error of a blind
    reconstruction, where (c z, Q / c) explain the same data."""
    x = np.asarray(a, dtype=np.complex128)
    y = np.asarray(b, dtype=np.complex128)
    if mask is not None:
        x, y = x[mask], y[mask]
    x, y = x.ravel(), y.ravel()
    den = np.vdot(x, x)
    c = np.vdot(x, y) / den if den != 0 else 0.0
    return float(np.linalg.norm(c * x - y) / np.linalg.norm(y))


def illumination_mask(Q, offs, n: int) -> np.ndarray:
    m = Q.shape[0]
    A = np.abs(np.asarray(Q, dtype=np.complex128)) ** 2
    ill = np.zeros((n, n))
    for r, c in offs:
        ill[r:r + m, c:c + m] += A
    return ill >= 0.1 * ill.max()


def run_one(ctx: Magpie, z_true, mask, epochs: int, batch: int, seed: int, tol: float) -> dict:
    """Flat start, `epochs` epochs; per-epoch Phi and statistic, errors at the checkpoints."""
    n_rows, n_cols = ctx.n_rows, ctx.n_cols
    ctx.set_object(np.ones((n_rows, n_cols), dtype=np.complex64))
    ctx.epoch_index = 0
    phi0, stat0 = ctx.objective()
    cps = set(checkpoints(epochs))
    phi, stat, errs = [phi0], [stat0], []
    e_rel, e_mag = object_errors(ctx.get_object(), z_true, mask)
    errs.append((0, e_rel, e_mag))
    hit = 0 if stat0 <= tol else None
    gpu_s = 0.0
    for e in range(1, epochs + 1):
        t0 = time.perf_counter()
        ctx.run_epochs(1, batch, seed=seed)
        ctx.sync()
        gpu_s += time.perf_counter() - t0
        p, s = ctx.objective()
        phi.append(p)
        stat.append(s)
        if hit is None and s <= tol:
            hit = e
        if e in cps or e == hit:
            e_rel, e_mag = object_errors(ctx.get_object(), z_true, mask)
            errs.append((e, e_rel, e_mag))
    return {"phi": phi, "stat": stat, "errors": errs, "tol_epoch": hit, "seconds": gpu_s,
            "finite": bool(np.all(np.isfinite(phi)))}


def overlap_geometry(cfg, ratio: float):
    """Scan of `cfg` with the step that gives adjacent positions the overlap `ratio` of the
    probe's footprint (the disc of diameter 2R = 20 m / 32 of the synthetic probe), over the
    same scanned span; None keeps the workload's own step."""
    if ratio is None:
        return cfg
    step = max(1, int(round((1.0 - ratio) * 20.0 * cfg.m / 32.0)))
    span = (cfg.P - 1) * cfg.step
    return dataclasses.replace(cfg, step=step, P=span // step + 1)


def noise_label(noise) -> str:
    kind, val = noise
    return "none" if kind == "none" else f"{kind} {val:g}"


def run(workload: str = "512x512", levels=None, alphas=(0.2, 0.5, 1.0), peaks=(None, 1e4), epochs: int = 200,
        batch: int | None = None, tol: float = 1e-4, seed: int = 7, log=print, etas=(), overlaps=(None,)) -> dict:
    """The whole sweep on the named workload of the synthetic suite (object, probe and scan of
    synth.WORKLOADS); intensities from the library's forward model with Poisson noise, given as
    peak photon counts (None = noiseless) and as the paper's eta (d = eta Poisson(d~ / eta))."""
    from synth import WORKLOADS, make_problem_inputs, poisson_counts
    base = WORKLOADS[workload]
    noises = [("none", 0.0) if p is None else ("peak", float(p)) for p in peaks] + [("eta", float(e)) for e in etas]
    max_l = int(np.log2(base.m)) + 1
    levels = list(levels) if levels else list(range(1, max_l + 1))
    out = {"workload": workload, "n": base.n, "m": base.m, "epochs": epochs, "tol": tol,
           "checkpoints": checkpoints(epochs), "runs": []}
    for ov in overlaps:
        cfg = overlap_geometry(base, ov)
        z_true, Q, offs, _, _ = make_problem_inputs(cfg)
        Q32 = Q.astype(np.complex64)
        z32 = z_true.astype(np.complex64)
        n, m = cfg.n, cfg.m
        B = min(batch or cfg.batch, len(offs))
        mask = illumination_mask(Q32, offs, n)
        with Magpie(n, n, m, 1, 0.5) as fm:
            fm.set_probe(Q32)
            fm.set_positions(offs)
            dtilde = fm.forward_model(z32)
        for noise in noises:
            kind, val = noise
            if kind == "none":
                d = dtilde.astype(np.float32)
            else:
                peak = val if kind == "peak" else float(dtilde.max()) / val
                d = poisson_counts(dtilde, peak, np.random.default_rng(seed + 1000)).astype(np.float32)
            for alpha in alphas:
                for L in levels:
                    with Magpie(n, n, m, L, alpha) as ctx:
                        ctx.set_probe(Q32)
                        ctx.set_positions(offs)
                        ctx.load_intensities(d, is_sqrt=False)
                        r = run_one(ctx, z32, mask, epochs, B, seed, tol)
                    r.update({"noise": noise_label(noise), "peak": val if kind == "peak" else None,
                              "eta": val if kind == "eta" else None, "alpha": alpha, "levels": L,
                              "overlap": ov, "step": cfg.step, "positions": int(len(offs)), "batch": B})
                    out["runs"].append(r)
                    last = r["errors"][-1]
                    log(f"overlap {ov if ov is not None else 'as scanned'} (step {cfg.step}, {len(offs)} pos) "
                        f"noise {noise_label(noise):>10} alpha {alpha:<5g} L {L}: Phi {r['phi'][0]:.3e} -> "
                        f"{r['phi'][-1]:.3e}, err {last[1]:.3e} (magnitude {last[2]:.3e}) after {last[0]} epochs, "
                        f"stat <= {tol:g} at epoch {r['tol_epoch']}, {r['seconds'] * 1e3:.1f} ms")
    return out


def run_blind(workload: str = "512x512", levels=(1, 3), modes=("fixed", "simultaneous", "alternating"), epochs: int = 300,
              beta: float = 0.5, alpha: float = 0.5, batch: int | None = None, seed: int = 7, log=print) -> dict:
    """Blind reconstruction from noiseless data with the probe's defocus phase unknown: the
    start probe is |Q| (the aperture without its quadratic phase).  Modes: the probe kept
    at that start ("fixed"), probe steps simultaneous with the object steps, or alternating
    (each minibatch's probe step at its updated object).  Errors after removing the complex
    scale that blind data cannot fix, at log-spaced epochs; GPU wall time of the epochs."""
    from synth import WORKLOADS, make_problem_inputs
    from .magpie import PROBE_ALTERNATE, UPDATE_PROBE
    cfg = WORKLOADS[workload]
    z_true, Q, offs, _, _ = make_problem_inputs(cfg)
    Q32 = Q.astype(np.complex64)
    Q0 = np.abs(Q).astype(np.complex64)
    z32 = z_true.astype(np.complex64)
    n, m = cfg.n, cfg.m
    B = min(batch or cfg.batch, len(offs))
    mask = illumination_mask(Q32, offs, n)
    with Magpie(n, n, m, 1, alpha) as fm:
        fm.set_probe(Q32)
        fm.set_positions(offs)
        d = fm.forward_model(z32)
    flags = {"fixed": 0, "simultaneous": UPDATE_PROBE, "alternating": UPDATE_PROBE | PROBE_ALTERNATE}
    cps = set(checkpoints(epochs))
    out = {"workload": workload, "epochs": epochs, "beta": beta, "alpha": alpha, "batch": B,
           "probe_start": "|Q| (quadratic phase unknown)", "runs": []}
    for L in levels:
        for mode in modes:
            with Magpie(n, n, m, L, alpha) as ctx:
                ctx.set_probe(Q0)
                ctx.set_positions(offs)
                ctx.load_intensities(d, is_sqrt=False)
                ctx.set_object(np.ones((n, n), dtype=np.complex64))
                ctx.set_flags(flags[mode], beta)
                rows, gpu_s = [], 0.0
                for e in range(1, epochs + 1):
                    t0 = time.perf_counter()
                    ctx.run_epochs(1, B, seed=seed)
                    ctx.sync()
                    gpu_s += time.perf_counter() - t0
                    if e in cps:
                        phi, _ = ctx.objective()
                        rows.append((e, scaled_error(ctx.get_object(), z32, mask),
                                     scaled_error(ctx.get_probe(), Q32), phi))
            out["runs"].append({"levels": L, "mode": mode, "trace": rows, "seconds": gpu_s})
            last = rows[-1]
            log(f"L {L} {mode:>12}: after {last[0]} epochs object err {last[1]:.3e}, probe err {last[2]:.3e}, "
                f"Phi {last[3]:.3e} ({gpu_s * 1e3:.0f} ms)")
    return out


def run_batches(workload: str = "512x512", batches=(256, 400, 800, 1600), levels: int | None = None, alpha: float = 0.5,
                target: float = 1e-3, max_epochs: int = 20000, noisy_epochs: int = 400, check: int = 10,
                seed: int = 7, log=print) -> dict:
    """Wall time to error against the minibatch size B (flat start, the workload's levels):
    noiseless data until the relative object error reaches `target` (checked every `check`
    epochs off the clock, at most `max_epochs`), and data with the workload's Poisson noise
    for `noisy_epochs` epochs, where the error passes through a minimum (the noise floor)
    before the iteration fits the noise: the epoch and time at which the error first comes
    within 5 % of that minimum, and at which Phi first comes within 1e-3 of its last value."""
    from synth import WORKLOADS, make_problem_inputs, poisson_counts
    cfg = WORKLOADS[workload]
    L = levels or cfg.levels
    z_true, Q, offs, _, _ = make_problem_inputs(cfg)
    Q32 = Q.astype(np.complex64)
    z32 = z_true.astype(np.complex64)
    n, m = cfg.n, cfg.m
    mask = illumination_mask(Q32, offs, n)
    with Magpie(n, n, m, 1, alpha) as fm:
        fm.set_probe(Q32)
        fm.set_positions(offs)
        dtilde = fm.forward_model(z32)
    data = {"noiseless": dtilde.astype(np.float32),
            f"{cfg.peak:g} photons": poisson_counts(dtilde, cfg.peak, np.random.default_rng(seed + 1000))
            .astype(np.float32)}
    out = {"workload": workload, "levels": L, "alpha": alpha, "target": target, "check": check, "runs": []}
    for label, d in data.items():
        noiseless = label == "noiseless"
        for B in batches:
            with Magpie(n, n, m, L, alpha) as ctx:
                ctx.set_probe(Q32)
                ctx.set_positions(offs)
                ctx.load_intensities(d, is_sqrt=False)
                ctx.set_object(np.ones((n, n), dtype=np.complex64))
                ctx.epoch_index = 0
                ctx.run_epochs(check, B, seed=seed + 99)      # warm the kernels (discarded)
                ctx.set_object(np.ones((n, n), dtype=np.complex64))
                ctx.epoch_index = 0
                ctx.sync()
                trace, gpu_s, e = [], 0.0, 0
                limit = max_epochs if noiseless else noisy_epochs
                while e < limit:
                    t0 = time.perf_counter()
                    ctx.run_epochs(check, B, seed=seed)
                    ctx.sync()
                    gpu_s += time.perf_counter() - t0
                    e += check
                    err, _ = object_errors(ctx.get_object(), z32, mask)
                    phi, _ = ctx.objective()
                    trace.append((e, gpu_s, err, phi))
                    if noiseless and err <= target:
                        break
            r = {"data": label, "batch": B, "ms_per_epoch": gpu_s * 1e3 / e, "trace": trace}
            if noiseless:
                hit = trace[-1] if trace[-1][2] <= target else None
                r.update(reached=hit is not None, epochs=hit[0] if hit else None, seconds=hit[1] if hit else None,
                         final_error=trace[-1][2])
                log(f"{label} B {B}: {r['ms_per_epoch']:.3f} ms/epoch, error {target:g} "
                    + (f"at epoch {hit[0]} after {hit[1] * 1e3:.1f} ms" if hit else
                       f"not reached in {e} epochs (error {trace[-1][2]:.3e})"))
            else:
                errs = np.array([t[2] for t in trace])
                best = int(np.argmin(errs))
                near = int(np.argmax(errs <= 1.05 * errs[best]))
                phis = np.array([t[3] for t in trace])
                plate = int(np.argmax(np.abs(phis - phis[-1]) <= 1e-3 * phis[-1]))
                r.update(best_error=float(errs[best]), best_epoch=trace[best][0],
                         near_best_epoch=trace[near][0], near_best_seconds=trace[near][1],
                         phi_plateau_epoch=trace[plate][0], phi_plateau_seconds=trace[plate][1],
                         final_phi=float(phis[-1]))
                log(f"{label} B {B}: {r['ms_per_epoch']:.3f} ms/epoch, best error {errs[best]:.3e} at epoch "
                    f"{trace[best][0]}, within 5 % of it at epoch {trace[near][0]} ({trace[near][1] * 1e3:.1f} ms), "
                    f"Phi within 1e-3 of its end at epoch {trace[plate][0]} ({trace[plate][1] * 1e3:.1f} ms)")
            out["runs"].append(r)
    return out


def table(res: dict, at=None) -> str:
    """Markdown table: relative error at a few checkpoints per (peak, alpha, L)."""
    cps = at or [c for c in res["checkpoints"] if c in (1, 10, 50, 100, 200, 500, 1000)] or res["checkpoints"][-3:]
    head = "| overlap | noise | alpha | L | " + " | ".join(f"err @{c}" for c in cps) + " | Phi end | stat<=tol epoch |"
    rows = [head, "|" + "---|" * (len(cps) + 6)]
    for r in res["runs"]:
        e = {ep: er for ep, er, _ in r["errors"]}
        cells = " | ".join(f"{e[c]:.3e}" if c in e else "" for c in cps)
        ov = "as scanned" if r.get("overlap") is None else f"{r['overlap']:g}"
        rows.append(f"| {ov} | {r.get('noise', 'none')} | {r['alpha']:g} | {r['levels']} | {cells} | "
                    f"{r['phi'][-1]:.3e} | {r['tol_epoch']} |")
    return "\n".join(rows)


def main():
    ap = argparse.ArgumentParser(description="Sweep the number of multigrid levels on a synthetic workload.")
    ap.add_argument("--workload", default="512x512", choices=["128x128", "512x512", "1024x1024"])
    ap.add_argument("--levels", type=str, default="", help="comma list (default 1 .. log2(m) + 1)")
    ap.add_argument("--alphas", type=str, default="0.2,0.5,1.0")
    ap.add_argument("--peaks", type=str, default="none,1e4", help="comma list; 'none' = noiseless")
    ap.add_argument("--etas", type=str, default="", help="comma list of the paper's noise levels eta")
    ap.add_argument("--overlaps", type=str, default="",
                    help="comma list of overlap ratios of adjacent scans (default: the workload's own step)")
    ap.add_argument("--epochs", type=int, default=200)
    ap.add_argument("--batch", type=int, default=0)
    ap.add_argument("--tol", type=float, default=1e-4)
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--out", type=str, default="")
    ap.add_argument("--blind", action="store_true",
                    help="blind runs instead: the start probe lacks its phase; fixed / simultaneous / alternating "
                         "probe steps at each --levels (default 1,3), --alphas[0], --beta")
    ap.add_argument("--beta", type=float, default=0.5)
    ap.add_argument("--batches", type=str, default="",
                    help="comma list of minibatch sizes: wall time to error for each (noiseless: to --target; "
                         "with the workload's noise: to the error minimum) at the workload's levels and "
                         "--alphas[0]")
    ap.add_argument("--target", type=float, default=1e-3)
    ap.add_argument("--max-epochs", type=int, default=20000)
    a = ap.parse_args()
    if a.batches:
        bs = [int(x) for x in a.batches.split(",") if x]
        lv = [int(x) for x in a.levels.split(",") if x]
        res = run_batches(a.workload, bs, lv[0] if lv else None, float(a.alphas.split(",")[0]), a.target,
                          a.max_epochs, a.epochs, seed=a.seed)
        if a.out:
            os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
            with open(a.out, "w") as f:
                json.dump(res, f)
        return
    if a.blind:
        lv = [int(x) for x in a.levels.split(",") if x] or [1, 3]
        res = run_blind(a.workload, lv, epochs=a.epochs, beta=a.beta, alpha=float(a.alphas.split(",")[0]),
                        batch=a.batch or None, seed=a.seed)
        print("| L | mode | " + " | ".join(f"obj/probe err @{r[0]}" for r in res["runs"][0]["trace"]) + " |")
        for r in res["runs"]:
            print(f"| {r['levels']} | {r['mode']} | " + " | ".join(f"{o:.2e} / {q:.2e}" for _, o, q, _ in r["trace"])
                  + " |")
        if a.out:
            os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
            with open(a.out, "w") as f:
                json.dump(res, f)
        return
    levels = [int(x) for x in a.levels.split(",") if x]
    alphas = [float(x) for x in a.alphas.split(",") if x]
    peaks = [None if x.strip().lower() == "none" else float(x) for x in a.peaks.split(",") if x]
    etas = [float(x) for x in a.etas.split(",") if x]
    overlaps = [float(x) for x in a.overlaps.split(",") if x] or [None]
    res = run(a.workload, levels, alphas, peaks, a.epochs, a.batch or None, a.tol, a.seed, etas=etas,
              overlaps=overlaps)
    print(table(res), flush=True)
    if a.out:
        os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
        with open(a.out, "w") as f:
            json.dump(res, f)


if __name__ == "__main__":
    main()
