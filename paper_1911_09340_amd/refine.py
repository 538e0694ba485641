"""Gradient refinement from a coarse grid vs a fine grid (the differentiation form).

For every turn partition of a set of events:
  coarse + LM: one batched scan of a coarse seed grid for all partitions
               (comet_batch_scan), k starting seeds of each: the paper's several
               reference seeds (Sec. 2.1), i.e. the lowest-RSS seeds whose finer seed
               sets do not overlap (comet_sparse_select; or the k lowest, comet_topk),
               one batched Levenberg-Marquardt refinement of all of them driven by the
               hand-written adjoint (comet_lm_refine), and per partition the refined
               seed with the lowest RSS;
  fine grid:   one batched scan of a fine grid over the same ranges; its argmin.
Both report |p| of the final seed against the true |p| at the seed point, and their
device time. Every step runs in the library's kernels; this module orders launches.
"""
from __future__ import annotations

import time
from dataclasses import replace

import numpy as np
import torch

from . import comet, scan, synth


def coarse_then_lm(events, sc: synth.ScanConfig, top_k: int = 8, n_iter: int = 8,
                   mu0: float = 1e-3, device="cuda", starts: str = "topk", local=None,
                   local_topk: int = 4, local_iters: int = 16):
    """starts: "sparse" (several non-overlapping references) or "topk" (the k lowest).
    local (points per axis, or None): after the LM, a finer grid around each partition's
    refined seed (the grid descriptor of comet_stage_grids: the seed itself at offset 0,
    half-spans of one coarse spacing, Sec. 2.1's finer re-scan), LM again from its
    local_topk lowest seeds, and the lowest RSS of all refined seeds is kept."""
    runner = scan.BatchRunner(events, replace(sc, n_refine=0), device)
    runner.run()
    NP = runner.n_part
    k = min(top_k, sc.n_seeds, 64 if starts == "sparse" else sc.n_seeds)
    idx = torch.empty(NP, k, dtype=torch.int64, device=device)
    if starts == "sparse":
        new_grids = torch.empty(NP, k, 14, dtype=torch.float64, device=device)
        comet.sparse_select(runner.grids.view(NP, 1, 14), runner.rss.view(NP, 1, -1), sc.n, k,
                            idx, new_grids)
    else:
        comet.topk(runner.rss, k, idx)
    seeds = torch.empty(6, NP * k, dtype=torch.float64, device=device)
    comet.grid_seeds(runner.grids, sc.n, idx, seeds)
    coarse_best = seeds.view(6, NP, k)[:, :, 0].clone()
    rss = torch.empty(NP * k, dtype=torch.float64, device=device)
    acc = torch.empty(NP * k, dtype=torch.int32, device=device)
    seed_event = runner.part_event.repeat_interleave(k)
    comet.lm_refine(seeds, runner.cfg, runner.packed.wire_ends, runner.packed.wire_offsets,
                    runner.packed.drift, n_iter, mu0, rss,
                    comet.lm_workspace(NP * k, sc.n_steps, device),
                    n_accepted=acc, event_wires=runner.packed.event_wires, seed_event=seed_event)
    pick = torch.empty(NP, 1, dtype=torch.int64, device=device)
    comet.topk(rss.view(NP, k), 1, pick)
    cols = torch.arange(NP, device=device) * k + pick[:, 0].clamp(min=0)
    final = torch.index_select(seeds, 1, cols)
    final_rss = torch.index_select(rss, 0, cols)
    out = {"coarse": coarse_best, "refined": final, "rss": final_rss, "accepted": acc,
           "partitions": NP}
    if local is None:
        return out
    half = tuple(2.0 * h / (n - 1) if n > 1 else h for h, n in zip(sc.half, sc.n))
    lsc = replace(sc, n=tuple(int(v) for v in local), half=half, n_refine=0)
    lrun = scan.BatchRunner(events, lsc, device)
    ft = final.t().contiguous()
    comet.stage_grids(ft, ft, lsc.half, lrun.grids0)
    lrun.run()
    k2 = min(local_topk, lsc.n_seeds)
    idx2 = torch.empty(NP, k2, dtype=torch.int64, device=device)
    comet.topk(lrun.rss, k2, idx2)
    seeds2 = torch.empty(6, NP * k2, dtype=torch.float64, device=device)
    comet.grid_seeds(lrun.grids, lsc.n, idx2, seeds2)
    rss2 = torch.empty(NP * k2, dtype=torch.float64, device=device)
    comet.lm_refine(seeds2, runner.cfg, runner.packed.wire_ends, runner.packed.wire_offsets,
                    runner.packed.drift, local_iters, mu0, rss2,
                    comet.lm_workspace(NP * k2, sc.n_steps, device),
                    event_wires=runner.packed.event_wires,
                    seed_event=runner.part_event.repeat_interleave(k2))
    # the first LM result first, so that it wins ties
    cand = torch.cat([final.view(6, NP, 1), seeds2.view(6, NP, k2)], dim=2).reshape(6, -1)
    crss = torch.cat([final_rss.view(NP, 1), rss2.view(NP, k2)], dim=1).contiguous()
    comet.topk(crss, 1, pick)
    cols = torch.arange(NP, device=device) * (k2 + 1) + pick[:, 0].clamp(min=0)
    out["refined"] = torch.index_select(cand, 1, cols)
    out["rss"] = torch.index_select(crss.view(-1), 0, cols)
    out["local_improved"] = (pick[:, 0] > 0)
    return out


def fine_grid(events, sc: synth.ScanConfig, device="cuda"):
    runner = scan.BatchRunner(events, replace(sc, n_refine=0), device)
    runner.run()
    return {"best": runner.best_seed.t().contiguous(), "rss": runner.best_rss}


def true_momenta(events) -> np.ndarray:
    return np.concatenate([np.linalg.norm(ev.ref_states[:, 3:], axis=1) for ev in events])


def momentum_residuals(seeds: torch.Tensor, events) -> np.ndarray:
    p = np.linalg.norm(seeds[3:].cpu().numpy(), axis=0)
    return p - true_momenta(events)


def summary(res: np.ndarray) -> dict:
    """RMS and a robust core width (1.4826 x median absolute deviation), MeV/c."""
    med = float(np.median(res))
    return {"rms": float(np.sqrt(np.mean(res ** 2))),
            "core_sigma": float(1.4826 * np.median(np.abs(res - med))), "median": med,
            "n": int(res.size)}


def compare(events, coarse: synth.ScanConfig, fine: synth.ScanConfig, top_k: int = 8,
            n_iter: int = 8, mu0: float = 1e-3, device="cuda", starts: str = "topk",
            local=None, local_topk: int = 4, local_iters: int = 16) -> dict:
    """Both strategies on the same events (each timed with device synchronisation)."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lm = coarse_then_lm(events, coarse, top_k, n_iter, mu0, device, starts=starts, local=local,
                        local_topk=local_topk, local_iters=local_iters)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    fg = fine_grid(events, fine, device)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    lm_rss = lm["rss"].cpu().numpy()
    fg_rss = fg["rss"].cpu().numpy()
    lm_res = momentum_residuals(lm["refined"], events)
    fg_res = momentum_residuals(fg["best"], events)
    # per partition: its event's number of turns (the other turns' hits enter Eq. 1 too)
    turns = np.concatenate([np.full(ev.n_turns, ev.n_turns) for ev in events])
    by_turns = {}
    for lo, hi, name in ((1, 1, "1"), (2, 2, "2"), (3, 99, "3+")):
        sel = (turns >= lo) & (turns <= hi)
        if sel.any():
            by_turns[name] = {"partitions": int(sel.sum()),
                              "coarse_lm_rms": float(np.sqrt(np.mean(lm_res[sel] ** 2))),
                              "fine_grid_rms": float(np.sqrt(np.mean(fg_res[sel] ** 2))),
                              "rss_lm_below_fine": float(np.mean(lm_rss[sel] <= fg_rss[sel]))}
    return {
        "events": len(events),
        "partitions": lm["partitions"],
        "coarse_lm": {"seconds": t1 - t0, **summary(lm_res),
                      "mean_accepted_steps": float(lm["accepted"].float().mean().item()),
                      "starts_per_partition": top_k, "starts": starts,
                      "lm_iterations": n_iter,
                      "local_rescan": None if local is None else {
                          "grid": "x".join(map(str, local)), "lm_starts": local_topk,
                          "lm_iterations": local_iters,
                          "partitions_improved": float(lm["local_improved"].float().mean())}},
        "coarse_only": summary(momentum_residuals(lm["coarse"], events)),
        "fine_grid": {"seconds": t2 - t1, **summary(fg_res)},
        "rss_lm_below_fine": float(np.mean(lm_rss <= fg_rss)),
        "by_turns": by_turns,
        "coarse_grid": "%s = %d seeds" % ("x".join(map(str, coarse.n)), coarse.n_seeds),
        "fine_grid_shape": "%s = %d seeds" % ("x".join(map(str, fine.n)), fine.n_seeds),
    }
