"""Iterative re-scan around several sparse reference seeds (Sec. 2.1).

For every turn partition of many events:
  scan 0      the partition's full seed grid (n = scan_cfg.n) in one batched launch;
  selection   the n_ref lowest-RSS seeds whose finer seed sets do not overlap
              (comet_sparse_select) become references; each gets a grid centred on it
              with half-spans of one previous spacing;
  scan k      every reference grid of every partition (n = n_fine, fewer seeds than
              scan 0) in one batched launch; selection again; n_iter times;
  final       the n_final sparse lowest-RSS seeds of the last scan and, for each, the
              classification of its event's hits (comet_batch_classify).
Reference 0 of the final set is the last scan's lowest-RSS seed. Every step runs in
the library's kernels; this module owns the buffers and orders the launches (all on
the current stream, no host synchronisation: capturable into one HIP graph).
"""
from __future__ import annotations

import numpy as np
import torch

from . import comet, scan, synth


class MultiRefScan:
    """Buffers and launches of the several-reference scan of NP partitions (part_event
    [NP] int32, device) over packed events given at run time. grids0 [NP, 14] holds the
    first grids (filled by the caller before run); n0 is their shape."""

    def __init__(self, part_event: torch.Tensor, n0, n_fine, n_ref: int, n_iter: int,
                 n_final: int, stride: int, n_wires: int, n_steps: int, device="cuda"):
        if n_iter < 0 or n_ref < 1 or n_final < 1:
            raise ValueError("need n_iter >= 0, n_ref >= 1 and n_final >= 1")
        self.n0 = tuple(int(v) for v in n0)
        self.n_fine = tuple(int(v) for v in n_fine)
        self.R, self.n_iter, self.F = int(n_ref), int(n_iter), int(n_final)
        NP = self.n_part = int(part_event.shape[0])
        self.part_event = part_event
        self.part_event_r = part_event.repeat_interleave(self.R)
        self.part_event_f = part_event.repeat_interleave(self.F)
        f64 = dict(dtype=torch.float64, device=device)
        i64 = dict(dtype=torch.int64, device=device)
        S0, S1 = int(np.prod(self.n0)), int(np.prod(self.n_fine))
        self.grids0 = torch.empty(NP, 14, **f64)
        self.rss0 = torch.empty(NP, S0, **f64)
        self.best0 = torch.empty(NP, **i64)
        # per re-scan k = 1..n_iter: its grids (the selection before it) and its RSS
        self.ref_idx = [torch.empty(NP, self.R, **i64) for _ in range(self.n_iter)]
        self.grids = [torch.empty(NP, self.R, 14, **f64) for _ in range(self.n_iter)]
        self.rss = [torch.empty(NP, self.R, S1, **f64) for _ in range(self.n_iter)]
        self.best = [torch.empty(NP * self.R, **i64) for _ in range(self.n_iter)]
        # final selection and classification
        self.final_idx = torch.empty(NP, self.F, **i64)
        self.final_rss = torch.empty(NP, self.F, **f64)
        self.final_grids = torch.empty(NP, self.F, 14, **f64)
        self.final_local = torch.empty(NP, self.F, **i64)
        self._final_new = torch.empty(NP, self.F, 14, **f64)
        self.final_seed = torch.empty(NP * self.F, 6, **f64)
        self.stride = int(stride)
        # entries past a partition's own hits are never written: start them at 0
        self.mask = torch.zeros(NP * self.F, self.stride, dtype=torch.uint8, device=device)
        self.n_border = torch.empty(NP * self.F, dtype=torch.int32, device=device)
        self.workspace = comet.batch_workspace(int(n_wires), int(n_steps),
                                               NP * max(self.R if self.n_iter else 1, 1), device)

    @property
    def seeds_per_partition(self) -> int:
        return int(np.prod(self.n0)) + self.n_iter * self.R * int(np.prod(self.n_fine))

    @property
    def last_n(self):
        return self.n_fine if self.n_iter else self.n0

    def last_scan(self):
        """(grids [NP, g, 14], rss [NP, g, S]) of the last scan."""
        NP = self.n_part
        if self.n_iter:
            return self.grids[-1], self.rss[-1]
        return self.grids0.view(NP, 1, 14), self.rss0.view(NP, 1, -1)

    def run(self, packed, cfg, event_active=None) -> None:
        """The scans of every partition whose event is active (all without
        event_active), the selections and the final classification."""
        NP, R = self.n_part, self.R
        comet.batch_scan(packed, self.part_event, self.grids0, self.n0, cfg, 0, self.rss0,
                         self.best0, self.workspace, event_active=event_active)
        src_g, src_r, src_n = self.grids0.view(NP, 1, 14), self.rss0.view(NP, 1, -1), self.n0
        for k in range(self.n_iter):
            comet.sparse_select(src_g, src_r, src_n, R, self.ref_idx[k], self.grids[k])
            comet.batch_scan(packed, self.part_event_r, self.grids[k].view(NP * R, 14),
                             self.n_fine, cfg, 0, self.rss[k].view(NP * R, -1), self.best[k],
                             self.workspace, event_active=event_active)
            src_g, src_r, src_n = self.grids[k], self.rss[k], self.n_fine
        comet.sparse_select(src_g, src_r, src_n, self.F, self.final_idx, self._final_new,
                            ref_rss=self.final_rss, ref_grids=self.final_grids,
                            ref_local=self.final_local)
        comet.batch_classify(packed, self.part_event_f, self.final_grids.view(-1, 14),
                             src_n, cfg, self.final_local.view(-1),
                             best_seed=self.final_seed, hit_mask=self.mask,
                             n_borderline=self.n_border)


class MultiRefRunner(MultiRefScan):
    """MultiRefScan over every turn partition of a list of events, with the first grids
    centred on each turn's true state at the seed radius."""

    def __init__(self, events, scan_cfg: synth.ScanConfig, n_ref: int = 10, n_iter: int = 2,
                 n_fine=(4, 8, 8, 8), n_final: int = 10, device="cuda"):
        from .synth import grid_descriptor
        self.events = list(events)
        self.sc = scan_cfg
        self.cfg = scan.config_for(self.events[0], scan_cfg)
        self.packed = scan.PackedEvents.from_events(self.events, device)
        part_event, grids = [], []
        for e, ev in enumerate(self.events):
            for t in range(ev.n_turns):
                part_event.append(e)
                grids.append(grid_descriptor(ev.ref_states[t], scan_cfg))
        pe = torch.as_tensor(np.asarray(part_event, dtype=np.int32), device=device)
        super().__init__(pe, scan_cfg.n, n_fine, n_ref, n_iter, n_final,
                         max(ev.n_hits for ev in self.events),
                         int(self.packed.wire_ends.shape[0]), scan_cfg.n_steps, device)
        self.grids0.copy_(torch.as_tensor(np.stack(grids), device=device))
        self.graph = None

    @property
    def evals_per_run(self) -> int:
        """Seed x hit evaluations of one run (every scan of every partition)."""
        hits = np.asarray([self.events[e].n_hits for e in self.part_event.cpu().numpy()])
        return int(hits.sum()) * self.seeds_per_partition

    def run(self) -> None:
        super().run(self.packed, self.cfg)

    def capture(self) -> None:
        """Capture one run into a HIP graph (replay() then repeats it)."""
        self.run()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.run()
        self.graph = g

    def replay(self) -> None:
        self.graph.replay()

    def best_seeds(self) -> torch.Tensor:
        """[6, NP]: reference 0 of every partition's final set (its lowest-RSS seed)."""
        return self.final_seed.view(self.n_part, self.F, 6)[:, 0, :].t().contiguous()
