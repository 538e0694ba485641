"""Device buffers and the launch sequence of one turn partition's seed scan.

One partition runs (Sec. 2.1): seed grid -> track recording (Alg. 1) -> DCA and
Eq. 1 RSS (Alg. 2) -> argmin, then `n_refine` finer re-scans around the best seed,
then classification of the hits at the final best seed. Every step is a call into
the HIP library through `comet`; this module only allocates buffers and orders
the launches on the current stream (no host synchronisation inside `run`).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import comet


@dataclass
class DeviceEvent:
    """An event's wires and hits in device memory (CSR by wire)."""
    wire_ends: torch.Tensor     # f64 [n_w, 6]
    wire_offsets: torch.Tensor  # i32 [n_w + 1]
    drift: torch.Tensor         # f64 [n_h]

    @classmethod
    def from_event(cls, ev, device="cuda"):
        return cls(torch.as_tensor(np.ascontiguousarray(ev.wire_ends), device=device),
                   torch.as_tensor(np.ascontiguousarray(ev.wire_offsets, dtype=np.int32),
                                   device=device),
                   torch.as_tensor(np.ascontiguousarray(ev.drift), device=device))

    @property
    def n_wires(self) -> int:
        return int(self.wire_ends.shape[0])

    @property
    def n_hits(self) -> int:
        return int(self.drift.shape[0])


class PartitionScanner:
    """Buffers sized for one grid shape, step count and event size."""

    def __init__(self, n, cfg: comet.Config, n_wires: int, n_hits: int, device="cuda",
                 field=None):
        """field: a comet.FieldMap to record tracks in (None: the uniform field of cfg)."""
        self.field = field
        self.n = tuple(int(v) for v in n)
        self.S = int(np.prod(self.n))
        self.cfg = cfg
        self.P = cfg.n_steps + 1
        f64 = dict(dtype=torch.float64, device=device)
        self.grid = torch.empty(14, **f64)
        self.seeds = torch.empty(6, self.S, **f64)
        self.track = torch.empty(3, self.P, self.S, **f64)
        self.rss = torch.empty(self.S, **f64)
        self.best = torch.empty(1, dtype=torch.int64, device=device)
        self.workspace = comet.dca_workspace(self.S, self.P, n_wires, device)
        self.mask = torch.empty(n_hits, dtype=torch.uint8, device=device)
        self.n_border = torch.empty(1, dtype=torch.int32, device=device)
        self.dca_best = torch.empty(n_wires, **f64)

    def run(self, ev: DeviceEvent, grid0: torch.Tensor, n_refine: int, on_scan=None) -> None:
        """The whole path for one partition; results stay in the buffers. on_scan (optional,
        for inspection) is called as on_scan(it, self) after scan it's selection, while
        self.grid, self.rss and self.best still hold that scan's grid, RSS and choice."""
        self.grid.copy_(grid0)
        for it in range(n_refine + 1):
            if it:
                comet.refine_grid(self.grid, self.n, self.best)
            comet.seed_grid(self.grid, self.n, self.seeds)
            comet.track_dca_rss(self.seeds, ev.wire_ends, ev.wire_offsets, ev.drift, self.cfg,
                                self.track, self.rss, self.workspace, field=self.field)
            last = it == n_refine
            comet.select_classify(self.rss, self.best, self.cfg, self.track, ev.wire_ends,
                                  ev.wire_offsets, ev.drift,
                                  hit_mask=self.mask if last else None,
                                  n_borderline=self.n_border if last else None,
                                  dca_best=self.dca_best if last else None)
            if on_scan is not None:
                on_scan(it, self)

    def result(self) -> dict:
        """Copy the partition's results to the host (synchronises)."""
        b = int(self.best.item())
        out = {"best": b, "grid": self.grid.cpu().numpy(), "mask": self.mask.cpu().numpy(),
               "n_borderline": int(self.n_border.item()), "dca_best": self.dca_best.cpu().numpy()}
        if b >= 0:
            out["best_seed"] = self.seeds[:, b].cpu().numpy()
            out["best_rss"] = float(self.rss[b].item())
        return out


@dataclass
class PackedEvents:
    """Several events in one CSR: event e owns wires [event_wires[e], event_wires[e+1])."""
    wire_ends: torch.Tensor     # f64 [W, 6]
    wire_offsets: torch.Tensor  # i32 [W + 1], global hit offsets
    drift: torch.Tensor         # f64 [H]
    event_wires: torch.Tensor   # i32 [E + 1]

    @classmethod
    def from_events(cls, events, device="cuda"):
        ends, offs, drift, ew = [], [0], [], [0]
        for ev in events:
            ends.append(ev.wire_ends)
            offs.extend((offs[-1] + ev.wire_offsets[1:]).tolist())
            drift.append(ev.drift)
            ew.append(ew[-1] + ev.n_wires)
        return cls(torch.as_tensor(np.ascontiguousarray(np.concatenate(ends)), device=device),
                   torch.as_tensor(np.asarray(offs, dtype=np.int32), device=device),
                   torch.as_tensor(np.ascontiguousarray(np.concatenate(drift)), device=device),
                   torch.as_tensor(np.asarray(ew, dtype=np.int32), device=device))


def grid_tensor(ref_state, scan_cfg, device="cuda") -> torch.Tensor:
    from .synth import grid_descriptor
    return torch.as_tensor(grid_descriptor(ref_state, scan_cfg), device=device)


def config_for(ev, scan_cfg) -> comet.Config:
    return comet.make_config(ev.bz, ev.charge, scan_cfg.step_mm, scan_cfg.n_steps,
                             scan_cfg.lambda_mm)


class BatchRunner:
    """All turn partitions of many events through comet_batch_scan (one call per run,
    capturable into a HIP graph)."""

    def __init__(self, events, scan_cfg, device="cuda", field=None):
        """field: a comet.FieldMap to record the tracks in (None: the uniform field)."""
        from .synth import grid_descriptor
        self.field = field
        self.events = list(events)
        self.sc = scan_cfg
        self.cfg = config_for(self.events[0], scan_cfg)
        self.packed = PackedEvents.from_events(self.events, device)
        part_event, grids = [], []
        for e, ev in enumerate(self.events):
            for t in range(ev.n_turns):
                part_event.append(e)
                grids.append(grid_descriptor(ev.ref_states[t], scan_cfg))
        self.n_part = len(part_event)
        self.part_event = torch.as_tensor(np.asarray(part_event, dtype=np.int32), device=device)
        self.grids0 = torch.as_tensor(np.stack(grids), device=device)
        self.grids = self.grids0.clone()
        S = scan_cfg.n_seeds
        f64 = dict(dtype=torch.float64, device=device)
        self.rss = torch.empty(self.n_part, S, **f64)
        self.best = torch.empty(self.n_part, dtype=torch.int64, device=device)
        self.best_seed = torch.empty(self.n_part, 6, **f64)
        self.best_rss = torch.empty(self.n_part, **f64)
        self.stride = max(ev.n_hits for ev in self.events)
        # entries past a partition's own hits are never written: start them at 0
        self.mask = torch.zeros(self.n_part, self.stride, dtype=torch.uint8, device=device)
        self.n_border = torch.empty(self.n_part, dtype=torch.int32, device=device)
        self.workspace = comet.batch_workspace(int(self.packed.wire_ends.shape[0]),
                                               scan_cfg.n_steps, self.n_part, device)
        self.graph = None

    @property
    def evals_per_run(self) -> int:
        """Seed x hit evaluations of one run (every scan of every partition)."""
        hits = np.asarray([self.events[e].n_hits for e in self.part_event.cpu().numpy()])
        return int(hits.sum()) * self.sc.n_seeds * (self.sc.n_refine + 1)

    def run(self, max_items: int = 0) -> None:
        comet.batch_scan(self.packed, self.part_event, self.grids, self.sc.n, self.cfg,
                         self.sc.n_refine, self.rss, self.best, self.workspace,
                         best_seed=self.best_seed, best_rss=self.best_rss, hit_mask=self.mask,
                         n_borderline=self.n_border, max_items=max_items, grids_init=self.grids0,
                         field=self.field)

    def autotune(self, items_per_block: int = 4, reps: int = 2) -> dict:
        """Time every shape of the batched scan kernel on a prefix of this run's work
        queue and keep the fastest per tile. A shape's prefix holds items_per_block work
        items for each of its persistent blocks (a work item is up to one 64-seed tile
        per wave), so that every block stays busy as in a full run. Every shape gives
        identical results."""
        variants = comet.batch_variants()
        total = self.n_part * ((self.sc.n_seeds + 63) // 64)
        us_per_tile, tiles = [], []
        for i, v in enumerate(variants):
            comet.set_batch_variant(i)
            n_tiles = min(total, items_per_block * v["blocks"] * v["nwv"])
            self.run(n_tiles)
            torch.cuda.synchronize()
            comet.profile_begin()
            for _ in range(reps):
                self.run(n_tiles)
            ms, n = comet.profile_end()["dca"]
            us_per_tile.append(1e3 * ms / max(n, 1) / n_tiles)
            tiles.append(n_tiles)
        best = int(np.argmin(us_per_tile))
        comet.set_batch_variant(best)
        return {"variant": best, "shape": variants[best], "us_per_tile": us_per_tile,
                "tiles": tiles}

    def capture(self) -> None:
        """Capture one run into a HIP graph (replay() then repeats it)."""
        self.run()  # warm-up outside capture
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.run()
        self.graph = g

    def replay(self) -> None:
        self.graph.replay()
