#!/usr/bin/env python3
"""Throughput of the seed-scan path on one MI355X.

Workload (one "step"): the signal-like three-turn event (227 hits on 172 wires,
10 % noise), and for each of its three turn partitions the whole path of the paper's
Sec. 2.1: a 16^4 seed grid (65 536 seeds) -> RK4 track recording, 1500 x 2 mm ->
DCA and Eq. 1 RSS (lambda = 0.8 mm) -> argmin, then two finer re-scans around the
best seed, then hit classification. Inputs are synthetic and already resident in
device memory when the timed region starts.

Prints one JSON line. `value` = seed x hit DCA evaluations per second (sum over
scans of seeds x hits, divided by wall time of the timed steps, which run without
any event timing; the three partitions are independent and run on a stream each). `roofline` covers the dominant kernel (the DCA scan), from a
separate pass that records HIP events around each launch on its stream: its two
ceilings are the FP64 flops of the distance evaluations it performs (15 per (seed,
wire, point) evaluated, counted by the kernel; the scan skips points that a distance
bound rules out, with the results of the full scan) against the FP64 vector peak, and
the HBM bytes the counters measured for its shape against the HBM peak; `bound` is
the one used more, and for "hbm" `achieved` is the launch's algorithmic bytes (one
read of the track and its window radii, d^2 written) per second.
`cpu_baseline` times the CPU reference (oracle/) on a bounded sample of the same
workload on the host cores. Further sections (each can be switched off): the same
step with tracks in a field map (RK4 and Runge-Kutta-Nystrom, and the batched scan in
the map), the batched persistent scan of the 1024-event mix, several references, half
tracks, the stage loop (plain, with the self-refining, with the seed's z axis), the
paper's per-stage chain and the first stage's efficiency and purity against lambda on
64 events of the mix, the gradient comparison on 256 events (coarse grid +
Levenberg-Marquardt vs a fine grid) and 64 events of the stress mix.

  python bench.py [--steps K] [--warmup W] [--gpus 1]
  python bench.py --sweep             # time every DCA kernel shape
  python bench.py --calibrate-copy    # a plain 1 GiB device copy, for counter scaling
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X FP64 vector peak: 256 CUs x 4 SIMDs x 16 FP64 FMA lanes x 2 flop x 2.4 GHz
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0     # MI355X HBM3E
FLOP_PER_POINT_WIRE = 15  # 6 FMA (in-plane coordinates) + 1 MUL + 1 FMA (squared distance)
METRIC = ("seed×hit DCA evals/s and events/s (FP64 % peak); "
          "grad-refine vs fine-grid time")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "dca_traffic.json")
KERNEL_SRCS = [os.path.join(ROOT, "paper_1911_09340_amd", "csrc", f)
               for f in ("comet.hip", "device_math.h", "dca_scan.h")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    """Hash of the sources of the forward-path kernels (traffic numbers go stale with them)."""
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def stored_traffic(shape: dict):
    """HBM bytes per DCA launch from the committed counter runs, if they were taken with
    the current kernel sources and the same kernel shape."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    from paper_1911_09340_amd import comet
    name = comet.dca_kernel_name(shape)
    if t.get("kernel_sha") != kernel_hash():
        return None
    return t.get("shapes", {}).get(name, {}).get("bytes_per_launch")


def calibrate_copy():
    import torch
    n = (1 << 30) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "launches": 3}))


def cpu_baseline(ev, sc, target_s: float):
    """The CPU reference on a bounded sample of partition 0's first grid."""
    import numpy as np
    import oracle
    from paper_1911_09340_amd import synth
    o = oracle.Oracle()
    grid = synth.grid_descriptor(ev.ref_states[0], sc)
    n = np.array(sc.n, dtype=np.int32)
    cfg = [ev.bz, ev.charge, sc.step_mm, sc.lambda_mm]
    all_seeds = o.seed_grid(grid, n)
    t0 = time.perf_counter()
    _, used = o.scan(all_seeds[:, :512], cfg, sc.n_steps, ev.wire_ends, ev.wire_offsets, ev.drift)
    per_seed = (time.perf_counter() - t0) / 512
    m = int(min(sc.n_seeds, max(64, target_s / max(per_seed, 1e-9))))
    idx = np.linspace(0, sc.n_seeds - 1, m).astype(np.int64)
    seeds = np.ascontiguousarray(all_seeds[:, idx])
    t0 = time.perf_counter()
    _, used = o.scan(seeds, cfg, sc.n_steps, ev.wire_ends, ev.wire_offsets, ev.drift)
    dt = time.perf_counter() - t0
    return {"value": m * ev.n_hits / dt, "unit": "seed×hit DCA evals/s", "cores": int(used),
            "kind": "oracle", "seconds": round(dt, 3),
            "sample": "%d of the 65536 seeds of turn partition 0's 16^4 grid (evenly spaced "
                      "indices), 1500 x 2 mm RK4, %d hits on %d wires, one scan" %
                      (m, ev.n_hits, ev.n_wires)}


def bench_batch(events, sc, reps: int = 2):
    """Every partition of `events` through the batched path, captured in a HIP graph."""
    import torch
    from paper_1911_09340_amd import comet, quality, refine, scan
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    packed = scan.PackedEvents.from_events(events)   # host CSR pack + copy to the device
    torch.cuda.synchronize()
    pack_s = time.perf_counter() - t0
    del packed
    runner = scan.BatchRunner(events, sc)
    tune = runner.autotune()
    log("  batched kernel shape %d %s; us per tile: %s"
        % (tune["variant"], tune["shape"], ", ".join("%.2f" % m for m in tune["us_per_tile"])))
    runner.capture()
    runner.replay()
    torch.cuda.synchronize()
    log("  captured one run in a HIP graph")
    comet.profile_begin()
    dts = []
    for r in range(reps):
        t0 = time.perf_counter()
        runner.replay()
        torch.cuda.synchronize()
        dts.append(time.perf_counter() - t0)
        log("  graph replay %d: %.3f s" % (r, dts[-1]))
    dt = float(np.median(dts))
    prof = comet.profile_end()  # graph replays record no events; eager run below
    comet.profile_begin()
    runner.run()
    torch.cuda.synchronize()
    prof = comet.profile_end()
    pw = 0
    hits = [ev.n_hits for ev in events]
    for e, ev in enumerate(events):
        pw += ev.n_turns * ev.n_wires
    scans = sc.n_refine + 1
    brute = FLOP_PER_POINT_WIRE * sc.n_seeds * (sc.n_steps + 1) * pw * scans
    flops = FLOP_PER_POINT_WIRE * prof["scan_points"]   # distance evaluations performed
    scan_ms = prof["dca"][0]
    return {"events": len(events), "partitions": runner.n_part, "seeds_per_partition": sc.n_seeds,
            "scans_per_partition": scans, "rk4_steps": sc.n_steps,
            "hits_min_mean_max": [min(hits), float(np.mean(hits)), max(hits)],
            "seconds_per_run": dt, "events_per_s": len(events) / dt,
            "host_pack_and_copy_s": pack_s,
            "evals_per_s": runner.evals_per_run / dt,
            "scan_kernel_ms_per_run": scan_ms,
            "scan_fp64_tflops": flops / (scan_ms * 1e-3) / 1e12,
            "scan_fp64_frac": flops / (scan_ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS,
            "scan_points_evaluated_frac": flops / brute,
            "kernel_shape": tune["shape"],
            "graph": "one HIP graph per run (frames, per scan: refine, counter reset, "
                     "persistent scan with in-kernel selection; classification)",
            "momentum_residual": refine.summary(
                refine.momentum_residuals(runner.best_seed.t().contiguous(), events)),
            "classification": quality.classification(runner.mask.cpu().numpy(), events)}


def bench_multiref(events, sc, n_ref: int = 10, n_iter: int = 2, n_fine=(4, 8, 8, 8),
                   n_final: int = 10, reps: int = 3):
    """The iterative re-scan around several sparse references (first scan on the full
    grid, n_iter re-scans of n_ref finer grids per partition, n_final final seeds and
    their classifications), captured in one HIP graph per run."""
    import torch
    from paper_1911_09340_amd import comet, multiref, quality, refine
    run = multiref.MultiRefRunner(events, sc, n_ref=n_ref, n_iter=n_iter, n_fine=n_fine,
                                  n_final=n_final)
    run.capture()
    run.replay()
    torch.cuda.synchronize()
    dts = []
    for r in range(reps):
        t0 = time.perf_counter()
        run.replay()
        torch.cuda.synchronize()
        dts.append(time.perf_counter() - t0)
        log("  graph replay %d: %.3f s" % (r, dts[-1]))
    dt = float(np.median(dts))
    comet.profile_begin()
    run.run()
    torch.cuda.synchronize()
    prof = comet.profile_end()
    S0, S1 = int(np.prod(sc.n)), int(np.prod(n_fine))
    masks = run.mask.cpu().numpy().reshape(run.n_part, n_final, -1)
    frss = run.final_rss.cpu().numpy()
    return {"events": len(events), "partitions": run.n_part,
            "first_grid": "x".join(map(str, sc.n)), "references": n_ref,
            "rescans": n_iter, "rescan_grid": "x".join(map(str, n_fine)),
            "final_seeds": n_final,
            "seeds_per_partition": S0 + n_iter * n_ref * S1,
            "seconds_per_run": dt, "events_per_s": len(events) / dt,
            "evals_per_s": run.evals_per_run / dt,
            "scan_kernel_ms_per_run": prof["dca"][0],
            "final_refs_taken_mean": float(np.mean(np.sum(~np.isnan(frss), axis=1))),
            "momentum_residual": refine.summary(refine.momentum_residuals(run.best_seeds(),
                                                                          events)),
            "classification": quality.classification(masks[:, 0, :], events)}


def bench_halves(events, sc, n_ref: int = 10, n_iter: int = 2, n_fine=(4, 8, 8, 8),
                 n_final: int = 10, reps: int = 3):
    """Both half tracks of every partition through the several-reference scan (half the
    RK4 steps each), the missing-layer veto and the ranked merge of half sets, captured
    in one HIP graph per run."""
    import torch
    from paper_1911_09340_amd import halves, quality, refine
    run = halves.HalfTrackRunner(events, sc, n_ref=n_ref, n_iter=n_iter, n_fine=n_fine,
                                 n_final=n_final)
    run.capture()
    run.replay()
    torch.cuda.synchronize()
    dts = []
    for r in range(reps):
        t0 = time.perf_counter()
        run.replay()
        torch.cuda.synchronize()
        dts.append(time.perf_counter() - t0)
        log("  graph replay %d: %.3f s" % (r, dts[-1]))
    dt = float(np.median(dts))
    nc = run.n_complete.cpu().numpy()
    seeds = run.best_complete_seeds()
    have = ~np.isnan(seeds[:, 0, 0])
    p_true = refine.true_momenta(events)
    res = np.linalg.norm(seeds[have, 0, 3:], axis=1) - p_true[have]
    vetoed = [float(np.mean(v.cpu().numpy() != 0)) for v in run.veto]
    return {"events": len(events), "partitions": run.n_part, "rk4_steps_per_half": run.sc_half.n_steps,
            "first_grid": "x".join(map(str, sc.n)), "references": n_ref, "rescans": n_iter,
            "rescan_grid": "x".join(map(str, n_fine)), "final_seeds_per_side": n_final,
            "seconds_per_run": dt, "events_per_s": len(events) / dt,
            "evals_per_s": run.evals_per_run / dt,
            "vetoed_fraction_entrance_exit": vetoed,
            "partitions_with_complete_set": float(np.mean(nc > 0)),
            "momentum_residual_entrance": refine.summary(res) if res.size else None,
            "classification": quality.classification(run.best_complete_masks(), events)}


def bench_stages(events, sc, max_stages: int = 5, min_wires: int = 30, reps: int = 3,
                 fit_iters: int = 0, eta: float = 0.3, n_z: int = 1, z_half: float = 0.0):
    """The stage loop: every event reconstructed turn by turn from its last turn, the
    hits of each stage left out of the next, each next stage's (z, p_z) from the
    backward extrapolation of the previous stage's seed (eager runs, device-synchronised
    wall time). With fit_iters > 0 each stage's seed is refined by Levenberg-Marquardt
    and its hits self-refined (lambda at the fitted track, eta re-admission). With
    n_z > 1 every stage also scans n_z values of the seed's z over z +- z_half."""
    import torch
    from paper_1911_09340_amd import stages
    run = stages.StageRunner(events, sc, max_stages=max_stages, min_wires=min_wires,
                             fit_iters=fit_iters, eta=eta, n_z=n_z, z_half=z_half)
    run.run()
    torch.cuda.synchronize()
    dts = []
    for r in range(reps):
        t0 = time.perf_counter()
        run.run()
        torch.cuda.synchronize()
        dts.append(time.perf_counter() - t0)
        log("  stage-loop run %d: %.3f s" % (r, dts[-1]))
    dt = float(np.median(dts))
    act = run.active_after.cpu().numpy()
    return {"events": len(events), "seeds_per_stage_scan": sc.n_seeds, "rescans": sc.n_refine,
            "max_stages": max_stages, "min_wires": min_wires, "fit_iters": fit_iters,
            "eta_mm": eta if fit_iters > 0 else None, "z_axis": None if n_z < 2 else {
                "points": n_z, "half_span_mm": z_half},
            "seconds_per_run": dt, "events_per_s": len(events) / dt,
            "events_active_after_stage": [int(a.sum()) for a in act],
            **_turn_quality(run, events)}


def _turn_quality(run, events) -> dict:
    """Hit-classification efficiency and purity (Sec. 3.2.1) of a stage loop's turn
    masks, over all turns and by the event's number of turns."""
    from paper_1911_09340_amd import quality
    tm = run.turn_masks()
    stride = max(ev.n_hits for ev in events)
    rows = []
    for ev, m in zip(events, tm):
        for t in range(ev.n_turns):
            row = np.zeros(stride, np.uint8)
            row[:ev.n_hits] = m[t]
            rows.append(row)
    masks = np.stack(rows)
    by_turns = {}
    p = 0
    for ev in events:
        q = quality.classification(masks[p:p + ev.n_turns], [ev])
        by_turns.setdefault(ev.n_turns, []).append((q["efficiency_mean"], q["purity_mean"]))
        p += ev.n_turns
    return {"classification_all_turns": quality.classification(masks, events),
            "efficiency_purity_by_turns": {
                str(k): [float(np.mean([x[0] for x in v])),
                         float(np.nanmean([x[1] for x in v])) if any(not np.isnan(x[1]) for x in v)
                         else None, len(v)] for k, v in sorted(by_turns.items())}}


def bench_chain(events, sc, reps: int = 3, fit_iters: int = 8, eta: float = 0.3):
    """The paper's per-stage chain (Sec. 3.1): per stage both half tracks with several
    references (first grid sc.n, 10 references, two re-scans of 4 x 8 x 8 x 8, 10 final
    seeds per side, half the steps of a turn), the missing-layer veto and the merge, the
    best complete set fitted by Levenberg-Marquardt and self-refined, then exclusion and
    backward extrapolation (eager launches, device-synchronised wall time)."""
    import torch
    from paper_1911_09340_amd import chain
    run = chain.StageChainRunner(events, sc, n_ref=10, n_iter=2, n_fine=(4, 8, 8, 8),
                                 n_final=10, fit_iters=fit_iters, eta=eta)
    run.run()
    torch.cuda.synchronize()
    dts = []
    for r in range(reps):
        t0 = time.perf_counter()
        run.run()
        torch.cuda.synchronize()
        dts.append(time.perf_counter() - t0)
        log("  chain run %d: %.3f s" % (r, dts[-1]))
    dt = float(np.median(dts))
    act = run.active_after.cpu().numpy()
    a0 = run.active0.cpu().numpy()
    nc = run.n_complete_at.cpu().numpy()
    stage_rows = [(s, e) for s in range(run.max_stages) for e in range(run.n_events)
                  if (a0[e] if s == 0 else act[s - 1, e])]
    return {"events": len(events), "first_grid": "x".join(map(str, sc.n)), "references": 10,
            "rescans": 2, "rescan_grid": "4x8x8x8", "final_seeds_per_side": 10,
            "rk4_steps_per_half": run.half_steps, "fit_iters": fit_iters, "eta_mm": eta,
            "seconds_per_run": dt, "events_per_s": len(events) / dt,
            "events_active_after_stage": [int(a.sum()) for a in act],
            "stages_with_complete_set": float(np.mean([nc[s, e] > 0 for s, e in stage_rows]))
            if stage_rows else None,
            **_turn_quality(run, events)}


def bench_lambda_sweep(events, sc, lambdas=(0.5, 0.6, 0.7, 0.8, 0.9, 1.0, 1.1, 1.2),
                       fit_iters: int = 8, eta: float = 0.3):
    """Hit-classification efficiency and purity of the first stage (each event's last
    turn) against the cutoff lambda, before and after the self-refining (Sec. 3.3's
    lambda scan at eta = 0.3 mm): the stage loop run for one stage per lambda."""
    import torch
    from dataclasses import replace
    from paper_1911_09340_amd import quality, stages
    rows = []
    for lam in lambdas:
        row = {"lambda_mm": lam}
        for key, fi in (("before", 0), ("after", fit_iters)):
            run = stages.StageRunner(events, replace(sc, lambda_mm=lam), max_stages=1,
                                     min_wires=30, fit_iters=fi, eta=eta)
            run.run()
            torch.cuda.synchronize()
            tm = run.turn_masks()
            eff, pur = [], []
            for ev, m in zip(events, tm):
                if ev.n_wires < 30:
                    continue
                e, u, _ = quality.turn_metrics(m[ev.n_turns - 1], ev.hit_turn)
                eff.append(e)
                pur.append(u)
            row[key] = {"efficiency_mean": float(np.mean(eff)),
                        "purity_mean": float(np.nanmean(pur)), "events": len(eff)}
        rows.append(row)
        log("  lambda %.1f mm: efficiency %.3f -> %.3f, purity %.3f -> %.3f (before -> after "
            "self-refining)" % (lam, row["before"]["efficiency_mean"],
                                row["after"]["efficiency_mean"], row["before"]["purity_mean"],
                                row["after"]["purity_mean"]))
    return {"eta_mm": eta, "stage": "first (each event's last turn)",
            "self_refining": "%d LM iterations, lambda re-test, eta re-admission" % fit_iters,
            "rows": rows}


def bench_field_batched(events, sc, reps: int = 2):
    """The batched persistent scan of the mix with every track in the solenoid map (RKN),
    eager runs, device-synchronised wall time."""
    import torch
    from paper_1911_09340_amd import comet, scan, synth
    fm = comet.FieldMap(*synth.solenoid_map(), stepper=1)
    run = scan.BatchRunner(events, sc, field=fm)
    run.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        run.run()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    return {"events": len(events), "partitions": run.n_part, "stepper": "rkn",
            "seconds_per_run": dt, "events_per_s": len(events) / dt,
            "evals_per_s": run.evals_per_run / dt}


def bench_field(ev, sc, steps: int = 3):
    """The signal workload's step with tracks recorded in the synthetic solenoid map,
    with classical RK4 and with Runge-Kutta-Nystrom (the event's hits come from the
    uniform-field helix, so only the timing means anything here)."""
    import torch
    from paper_1911_09340_amd import comet, scan, synth
    cfg = scan.config_for(ev, sc)
    dev = scan.DeviceEvent.from_event(ev)
    grids = [scan.grid_tensor(ev.ref_states[t], sc) for t in range(ev.n_turns)]
    P = sc.n_steps + 1
    out = {"map": "synthetic solenoid, 81 x 81 x 121 nodes, 25 mm, B_z = 1 T (1 + 0.1 (z / "
                  "1.5 m)^2) with the matching radial field"}
    for name, stepper in (("rk4", 0), ("rkn", 1)):
        fm = comet.FieldMap(*synth.solenoid_map(), stepper=stepper)
        runners = [scan.PartitionScanner(sc.n, cfg, ev.n_wires, ev.n_hits, field=fm)
                   for _ in range(ev.n_turns)]

        def step():
            for t in range(ev.n_turns):
                runners[t].run(dev, grids[t], sc.n_refine)
        step()
        torch.cuda.synchronize()
        comet.profile_begin()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        prof = comet.profile_end()
        ms_trk, n_trk = prof["track"]
        out[name] = {
            "ms_per_step": dt / steps * 1e3,
            "evals_per_s": ev.n_turns * (sc.n_refine + 1) * sc.n_seeds * ev.n_hits * steps / dt,
            "track_kernel_ms": ms_trk / n_trk,
            "track_write_gbs": 24.0 * P * sc.n_seeds / (ms_trk / n_trk * 1e-3) / 1e9,
            "dca_kernel_ms": prof["dca"][0] / prof["dca"][1]}
    return out


def bench_stress(events, sc, top_k: int = 64, n_iter: int = 8):
    """The stress mix: one batched scan of every partition, then Levenberg-Marquardt
    from the top_k lowest-RSS seeds of each partition (device time per phase)."""
    import torch
    from paper_1911_09340_amd import comet, refine
    refine.coarse_then_lm(events[:2], sc, top_k=top_k, n_iter=1)  # warm-up
    torch.cuda.synchronize()
    comet.profile_begin()
    t0 = time.perf_counter()
    out = refine.coarse_then_lm(events, sc, top_k=top_k, n_iter=n_iter)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = comet.profile_end()
    hits = [ev.n_hits for ev in events]
    pw = sum(ev.n_turns * ev.n_wires for ev in events)
    ph = sum(ev.n_turns * ev.n_hits for ev in events)
    brute = FLOP_PER_POINT_WIRE * sc.n_seeds * (sc.n_steps + 1) * pw
    flops = FLOP_PER_POINT_WIRE * prof["scan_points"]
    scan_ms = prof["dca"][0]
    res = refine.summary(refine.momentum_residuals(out["refined"], events))
    return {"events": len(events), "partitions": out["partitions"],
            "seeds_per_partition": sc.n_seeds, "rk4_steps": sc.n_steps, "step_mm": sc.step_mm,
            "hits_min_mean_max": [min(hits), float(np.mean(hits)), max(hits)],
            "lm_starts_per_partition": top_k, "lm_iterations": n_iter,
            "seconds": dt, "events_per_s": len(events) / dt,
            "evals_per_s": ph * sc.n_seeds / dt,
            "scan_kernel_ms": scan_ms, "scan_fp64_frac":
                flops / (scan_ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS,
            "scan_points_evaluated_frac": flops / brute,
            "momentum_residual": res,
            "timing": "wall time of the whole call: host pack, batched scan, top-k, LM"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--variant", type=int, default=None, help="DCA kernel shape id")
    ap.add_argument("--sweep", action="store_true", help="time every DCA kernel shape")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--one-stream", action="store_true",
                    help="time the signal step's partitions one after another on one stream")
    ap.add_argument("--batch-events", type=int, default=1024,
                    help="events of the batched mix timed through the persistent batched path "
                         "(0 = skip; 1024 = the full batching workload)")
    ap.add_argument("--mix-events", type=int, default=64,
                    help="events of the batched mix for the several-reference, half-track, "
                         "stage-loop and batched field-map sections (0 = skip them)")
    ap.add_argument("--grad-events", type=int, default=256,
                    help="events of the batched mix for the coarse+LM vs fine-grid comparison "
                         "(0 = skip; 256 = the full differentiation workload)")
    ap.add_argument("--grad-topk", type=int, default=128,
                    help="LM starts per partition (the lowest-RSS coarse seeds)")
    ap.add_argument("--grad-iters", type=int, default=32, help="LM iterations")
    ap.add_argument("--no-multiref", dest="multiref", action="store_false",
                    help="skip the several-reference re-scan on the batched mix")
    ap.add_argument("--no-halves", dest="halves", action="store_false",
                    help="skip the half-track scans and merge on the batched mix")
    ap.add_argument("--no-field", dest="field", action="store_false",
                    help="skip the field-map variant of the signal workload")
    ap.add_argument("--no-stages", dest="stages", action="store_false",
                    help="skip the stage loop on the batched mix")
    ap.add_argument("--stress-events", type=int, default=64,
                    help="events of the stress mix (1-6 turns, 200-1200 hits, 30%% noise, "
                         "131072 seeds, 2000 x 1.5 mm) through the batched scan and LM from "
                         "the 64 lowest-RSS seeds per partition (0 = skip; the full workload "
                         "is 8192 events)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only (--gpus 1): it measures the single-GPU path; "
              "sharding events across GPUs is not implemented.", file=sys.stderr)
        sys.exit(2)

    # events for the gradient comparison are drawn before the GPU is touched, so that
    # worker processes can be forked safely
    grad_events, batch_events, mix_events, stress_events = [], [], [], []
    n_mix = max(args.grad_events, args.batch_events, args.mix_events)
    if not args.calibrate_copy:
        from paper_1911_09340_amd import synth as _synth
        workers = min(16, os.cpu_count() or 1)
        if n_mix > 0:
            t0 = time.perf_counter()
            mix = _synth.event_mix_batch(range(n_mix), workers=workers)
            grad_events, batch_events = mix[:args.grad_events], mix[:args.batch_events]
            mix_events = mix[:args.mix_events]
            log("drew %d mix events in %.1f s" % (len(mix), time.perf_counter() - t0))
        if args.stress_events > 0:
            t0 = time.perf_counter()
            stress_events = _synth.event_mix_batch(range(args.stress_events), workers=workers,
                                                   kind="stress")
            log("drew %d stress events in %.1f s" % (len(stress_events), time.perf_counter() - t0))

    import torch
    from paper_1911_09340_amd import comet, scan, synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    comet.load()
    if args.calibrate_copy:
        calibrate_copy()
        return

    ev = synth.event_signal(0)
    sc = synth.C1
    cfg = scan.config_for(ev, sc)
    dev = scan.DeviceEvent.from_event(ev)
    grids = [scan.grid_tensor(ev.ref_states[t], sc) for t in range(ev.n_turns)]
    runners = [scan.PartitionScanner(sc.n, cfg, ev.n_wires, ev.n_hits) for _ in range(ev.n_turns)]
    scans_per_step = ev.n_turns * (sc.n_refine + 1)
    evals_per_step = scans_per_step * sc.n_seeds * ev.n_hits
    P = sc.n_steps + 1

    # the partitions are independent: each runs its chain of scans on a stream of its own
    # (default priority), so that one partition's small kernels and launch gaps overlap
    # another's scans
    streams = [torch.cuda.Stream() for _ in range(ev.n_turns)]

    def step(concurrent=True):
        if not concurrent or args.one_stream:
            for t in range(ev.n_turns):
                runners[t].run(dev, grids[t], sc.n_refine)
            return
        cur = torch.cuda.current_stream()
        for t in range(ev.n_turns):
            streams[t].wait_stream(cur)
            with torch.cuda.stream(streams[t]):
                runners[t].run(dev, grids[t], sc.n_refine)
        for t in range(ev.n_turns):
            cur.wait_stream(streams[t])

    def timed(steps, warmup, profile=False):
        """Wall time of `steps` steps; with profile, per-kind kernel times from HIP events
        and the DCA scans' evaluation count (a separate pass, with the partitions one
        after another on one stream so that each launch's time is its own: the headline
        runs without them, the partitions on streams of their own)."""
        for _ in range(warmup):
            step(not profile)
        torch.cuda.synchronize()
        if profile:
            comet.profile_begin()
        t0 = time.perf_counter()
        for _ in range(steps):
            step(not profile)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        return t1 - t0, (comet.profile_end() if profile else None)

    variants = comet.dca_variants()
    # autotune the DCA kernel shape on the live buffers of the first partition's first
    # scan (the costliest of the three: its seeds spread widest, so a wave's lanes need
    # the most chunks); the shape then serves every scan of this size
    step()
    r0 = runners[0]
    r0.run(dev, grids[0], 0)
    tuned, tune_ms = comet.dca_autotune(r0.track, dev.wire_ends, dev.wire_offsets, dev.drift, cfg,
                                        r0.rss, r0.workspace, reps=2)
    log("autotune: shape %d %s (%.3f ms); all: %s" % (tuned, variants[tuned], tune_ms[tuned],
                                                      ", ".join("%.3f" % m for m in tune_ms)))
    if args.sweep:
        for i, v in enumerate(variants):
            comet.set_dca_variant(i)
            dt, prof = timed(max(2, args.steps // 2), 1, profile=True)
            ms, n = prof["dca"]
            tfl = FLOP_PER_POINT_WIRE * prof["scan_points"] / n / (ms / n * 1e-3) / 1e12
            log("variant %d %s: %.3f ms/step, dca %.3f ms/launch, %.1f TFLOP/s (%.1f %% of FP64 peak)"
                % (i, v, dt / max(2, args.steps // 2) * 1e3, ms / n, tfl, 100 * tfl / PEAK_FP64_TFLOPS))
    comet.set_dca_variant(-1 if args.variant is None else args.variant)
    variant = comet.dca_variant_for(sc.n_seeds, P, ev.n_wires)

    log("warmup %d, timing %d steps (%d scans of %d seeds x %d hits each) ..."
        % (args.warmup, args.steps, scans_per_step, sc.n_seeds, ev.n_hits))
    dt, _ = timed(args.steps, args.warmup)
    log("timed region %.3f s (no event timing)" % dt)
    # per-kernel times and the evaluation count in a separate, event-timed pass
    prof_steps = max(3, args.steps // 2)
    _, prof = timed(prof_steps, 0, profile=True)
    ms_dca, n_dca = prof["dca"]
    dca_s = ms_dca / n_dca * 1e-3
    brute = FLOP_PER_POINT_WIRE * sc.n_seeds * ev.n_wires * P
    flops = FLOP_PER_POINT_WIRE * prof["scan_points"] / n_dca   # per launch, performed
    achieved = flops / dca_s / 1e12
    ms_trk, n_trk = prof["track"]
    # the track, the seeds read, and the radii of its 16-point windows written with it
    trk_bytes = 8 * 3 * P * sc.n_seeds + 8 * 6 * sc.n_seeds + 8 * ((P - 1) // 16 + 1) * sc.n_seeds
    traffic = stored_traffic(variants[variant])
    # the DCA launch's algorithmic bytes: one read of the track and of its window radii,
    # the per-(wire, seed) d^2 written
    n_win = (P - 1) // 16 + 1
    dca_alg_bytes = 8 * 3 * P * sc.n_seeds + 8 * n_win * sc.n_seeds + 8 * ev.n_wires * sc.n_seeds
    fp64_frac = achieved / PEAK_FP64_TFLOPS
    hbm_used_frac = None if traffic is None else traffic / dca_s / 1e9 / PEAK_HBM_GBS
    # the binding resource: the one the launch uses the larger share of
    if hbm_used_frac is not None and hbm_used_frac > fp64_frac:
        headline = {"bound": "hbm", "achieved": dca_alg_bytes / dca_s / 1e9,
                    "peak": PEAK_HBM_GBS, "unit": "GB/s",
                    "frac": dca_alg_bytes / dca_s / 1e9 / PEAK_HBM_GBS}
    else:
        headline = {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                    "unit": "TFLOP/s", "frac": fp64_frac}

    out = {
        "metric": METRIC,
        "value": evals_per_step * args.steps / dt,
        "unit": "seed×hit DCA evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "signal-like e- event, 104 MeV/c, 3 turn partitions; per partition a "
                        "16^4 seed grid (65536 seeds) + 2 finer re-scans + classification; "
                        "RK4 1500 x 2 mm, 1 T; %d hits on %d wires (10%% noise); lambda 0.8 mm"
                        % (ev.n_hits, ev.n_wires),
            "seeds_per_scan": sc.n_seeds,
            "scans_per_step": scans_per_step,
            "hits": ev.n_hits,
            "wires": ev.n_wires,
            "rk4_steps": sc.n_steps,
            "dca_kernel_shape": variants[variant],
        },
        "events_per_s": args.steps / dt,
        "roofline": dict(headline, **{
            "kernel": comet.dca_kernel_name(variants[variant]),
            "traffic": traffic,
            "avg_launch_ms": dca_s * 1e3,
            "launches": n_dca,
            "timing": "HIP events around each launch on its stream, in a separate pass of %d "
                      "steps after the timed region" % prof_steps,
            "ceilings": {
                "fp64_executed": {"achieved_tflops": achieved, "peak_tflops": PEAK_FP64_TFLOPS,
                                  "frac": fp64_frac},
                "hbm_measured": None if traffic is None else {
                    "bytes_per_launch": traffic, "achieved_gbs": traffic / dca_s / 1e9,
                    "peak_gbs": PEAK_HBM_GBS, "frac": hbm_used_frac},
                "hbm_algorithmic": {"bytes_per_launch": dca_alg_bytes,
                                    "achieved_gbs": dca_alg_bytes / dca_s / 1e9,
                                    "peak_gbs": PEAK_HBM_GBS,
                                    "frac": dca_alg_bytes / dca_s / 1e9 / PEAK_HBM_GBS},
            },
            "flop_per_launch": flops,
            "flop_unit": "%d FP64 flop per (seed, wire, track point) distance evaluated; the "
                         "scan skips points a distance bound rules out" % FLOP_PER_POINT_WIRE,
            "points_evaluated_frac": flops / brute,
            "full_scan_equivalent_tflops": brute / dca_s / 1e12,
        }),
        "track_recording": {
            "kernel": "rk4_record_kernel",
            "bound": "hbm",
            "achieved": trk_bytes / (ms_trk / n_trk * 1e-3) / 1e9,
            "peak": PEAK_HBM_GBS,
            "unit": "GB/s",
            "frac": trk_bytes / (ms_trk / n_trk * 1e-3) / 1e9 / PEAK_HBM_GBS,
            "avg_launch_ms": ms_trk / n_trk,
        },
        "kernel_ms_per_step": {k: v[0] / prof_steps for k, v in prof.items()
                               if k in comet.PROFILE_KINDS},
    }
    if args.field:
        log("signal workload with tracks in a field map ...")
        out["field_map"] = bench_field(ev, sc)
        fm = out["field_map"]
        if mix_events:
            fm["batched_rkn"] = bench_field_batched(mix_events, synth.C2)
            log("  batched mix in the map (RKN): %.1f events/s (uniform field: see batch)"
                % fm["batched_rkn"]["events_per_s"])
        for name in ("rk4", "rkn"):
            log("  %s: %.1f ms per step (uniform field: %.1f), map track recording %.2f ms per "
                "scan" % (name, fm[name]["ms_per_step"], dt / args.steps * 1e3,
                          fm[name]["track_kernel_ms"]))
    if batch_events:
        log("batched mix: %d events, persistent scans, HIP graph ..." % len(batch_events))
        out["batch"] = bench_batch(batch_events, synth.C2)
        log("  %.1f events/s, %.3g seed x hit evals/s, scan kernel %.1f %% of FP64 peak"
            % (out["batch"]["events_per_s"], out["batch"]["evals_per_s"],
               100 * out["batch"]["scan_fp64_frac"]))
    if mix_events and args.multiref:
        log("several references: %d events, 10 references, 2 re-scans of 4x8x8x8 ..."
            % len(mix_events))
        out["multiref"] = bench_multiref(mix_events, synth.C2)
        m = out["multiref"]
        log("  %.1f events/s; |p| residual core %.3f MeV/c; efficiency %.3f purity %.3f"
            % (m["events_per_s"], m["momentum_residual"]["core_sigma"],
               m["classification"]["efficiency_mean"], m["classification"]["purity_mean"]))
    if mix_events and args.halves:
        log("half tracks: %d events, both halves with several references, veto, merge ..."
            % len(mix_events))
        out["halves"] = bench_halves(mix_events, synth.C2)
        h = out["halves"]
        log("  %.1f events/s; complete sets in %.3f of partitions; efficiency %.3f purity %.3f"
            % (h["events_per_s"], h["partitions_with_complete_set"],
               h["classification"]["efficiency_mean"], h["classification"]["purity_mean"]))
    if mix_events and args.stages:
        log("stage loop: %d events, up to 5 stages from the last turn back ..." % len(mix_events))
        out["stages"] = bench_stages(mix_events, synth.C2)
        log("stage loop with self-refining (8 LM iterations, eta 0.3 mm) ...")
        out["stages_self_refined"] = bench_stages(mix_events, synth.C2, fit_iters=8)
        log("stage loop with self-refining and the seed's z as a fifth axis (5 x 4 mm) ...")
        out["stages_z"] = bench_stages(mix_events, synth.C2, fit_iters=8, n_z=5, z_half=8.0)
        log("per-stage chain: half tracks with several references, veto, merge, fit and "
            "self-refining per stage ...")
        out["stage_chain"] = bench_chain(mix_events, synth.C2)
        log("  stage chain: complete sets in %.3f of the scanned stages"
            % (out["stage_chain"]["stages_with_complete_set"] or 0.0))
        for key in ("stages", "stages_self_refined", "stages_z", "stage_chain"):
            st = out[key]
            log("  %s: %.1f events/s; efficiency %.3f purity %.3f over all turns; by turns: %s"
                % (key, st["events_per_s"], st["classification_all_turns"]["efficiency_mean"],
                   st["classification_all_turns"]["purity_mean"],
                   ", ".join("%s: %.2f/%s" % (k, v[0], "-" if v[1] is None else "%.2f" % v[1])
                             for k, v in st["efficiency_purity_by_turns"].items())))
    if mix_events and args.stages:
        log("lambda sweep of the first stage (eta 0.3 mm), %d events ..." % len(mix_events))
        out["lambda_sweep"] = bench_lambda_sweep(mix_events, synth.C2)
    if grad_events:
        from paper_1911_09340_amd import refine
        log("coarse 8^4 + LM vs fine 32^4 grid on %d events ..." % len(grad_events))
        out["grad_refine"] = refine.compare(grad_events, synth.C3_COARSE, synth.C3_FINE,
                                            local=(16, 16, 8, 8), local_topk=16, local_iters=32,
                                            top_k=args.grad_topk, n_iter=args.grad_iters)
        g = out["grad_refine"]
        log("  coarse+LM %.2f s, |p| residual rms %.3f core %.3f MeV/c; fine grid %.2f s, rms %.3f "
            "core %.3f; LM at or below the fine grid's RSS in %.3f of partitions" % (
                g["coarse_lm"]["seconds"], g["coarse_lm"]["rms"], g["coarse_lm"]["core_sigma"],
                g["fine_grid"]["seconds"], g["fine_grid"]["rms"], g["fine_grid"]["core_sigma"],
                g["rss_lm_below_fine"]))
        log("  by the event's turns (rms coarse+LM / fine, RSS below): " + ", ".join(
            "%s: %.3f / %.3f, %.3f" % (k, v["coarse_lm_rms"], v["fine_grid_rms"],
                                       v["rss_lm_below_fine"]) for k, v in g["by_turns"].items()))
    if stress_events:
        log("stress mix: %d events, batched scan + LM from the top 64 seeds ..." % len(stress_events))
        out["stress"] = bench_stress(stress_events, synth.C4)
        log("  %.2f events/s, %.3g seed x hit evals/s, scan kernel %.1f %% of FP64 peak"
            % (out["stress"]["events_per_s"], out["stress"]["evals_per_s"],
               100 * out["stress"]["scan_fp64_frac"]))
    if not args.no_cpu_baseline:
        log("CPU reference baseline (~%.0f s) ..." % args.cpu_seconds)
        out["cpu_baseline"] = cpu_baseline(ev, sc, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
