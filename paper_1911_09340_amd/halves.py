"""Half-track scans and their merge (Sec. 3.1).

Every turn partition is split into an entrance and an exit half track (synth.half_events:
each half holds the event's wires on its side, the exit seed has momentum and charge
flipped). Each side goes through the several-reference scan (multiref.MultiRefRunner)
as its own batch, with half the RK4 steps of a full turn, and ends with n_final seeds
and their half sets of classified hits. Then, on the device:
  comet_layer_veto    excludes seeds whose half set leaves a layer without a hit;
  comet_merge_halves  ranks the complete sets (one kept seed of each side) by their
                      combined RSS.
This module builds the half events, owns the buffers and orders the launches.
"""
from __future__ import annotations

from dataclasses import replace

import numpy as np
import torch

from . import comet, multiref, synth


class HalfTrackRunner:
    def __init__(self, events, scan_cfg: synth.ScanConfig, n_ref: int = 10, n_iter: int = 2,
                 n_fine=(4, 8, 8, 8), n_final: int = 10, half_steps: int = None, device="cuda"):
        self.events = list(events)
        ent, ext = [], []
        for ev in self.events:
            for t in range(ev.n_turns):
                a, b = synth.half_events(ev, t)
                ent.append(a)
                ext.append(b)
        self.n_part = len(ent)
        self.F = int(n_final)
        steps = int(half_steps) if half_steps else scan_cfg.n_steps // 2
        self.sc_half = replace(scan_cfg, n_steps=steps)
        kw = dict(n_ref=n_ref, n_iter=n_iter, n_fine=n_fine, n_final=n_final, device=device)
        self.sides = (multiref.MultiRefRunner(ent, self.sc_half, **kw),
                      multiref.MultiRefRunner(ext, self.sc_half, **kw))
        self.half_events = (ent, ext)
        i32 = dict(dtype=torch.int32, device=device)
        self.wire_layer = [torch.as_tensor(np.concatenate([synth.wire_layers(e.wire_ids)
                                                           for e in evs]).astype(np.int32),
                                           device=device) for evs in (ent, ext)]
        self.veto = [torch.empty(self.n_part * self.F, **i32) for _ in range(2)]
        self.pair = torch.empty(self.n_part, self.F * self.F, **i32)
        self.pair_rss = torch.empty(self.n_part, self.F * self.F, dtype=torch.float64,
                                    device=device)
        self.n_complete = torch.empty(self.n_part, **i32)
        self.graph = None

    @property
    def evals_per_run(self) -> int:
        return sum(s.evals_per_run for s in self.sides)

    def run(self) -> None:
        for s, side in enumerate(self.sides):
            side.run()
            comet.layer_veto(side.mask, side.part_event_f, side.packed, self.wire_layer[s],
                             synth.N_LAYERS, self.veto[s])
        a, b = self.sides
        comet.merge_halves(a.final_rss, self.veto[0].view(self.n_part, self.F), b.final_rss,
                           self.veto[1].view(self.n_part, self.F), self.pair, self.pair_rss,
                           self.n_complete)

    def capture(self) -> None:
        self.run()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.run()
        self.graph = g

    def replay(self) -> None:
        self.graph.replay()

    # ---------------------------------------------------------- host-side reporting
    def best_complete_masks(self) -> np.ndarray:
        """[NP, max event hits] uint8: the union of the two half sets of each partition's
        top-ranked complete set, on the event's own hit indices (zeros where a partition
        has no complete set)."""
        pair = self.pair.cpu().numpy()
        masks = [s.mask.cpu().numpy().reshape(self.n_part, self.F, -1) for s in self.sides]
        stride = max(ev.n_hits for ev in self.events)
        out = np.zeros((self.n_part, stride), np.uint8)
        for p in range(self.n_part):
            k = int(pair[p, 0])
            if k < 0:
                continue
            for side, r in ((0, k // self.F), (1, k % self.F)):
                h = self.half_events[side][p].meta["hits"]
                out[p, h] |= masks[side][p, r, :h.size] & 1
        return out

    def best_complete_seeds(self) -> np.ndarray:
        """[NP, 2, 6]: entrance and exit seed (the exit one as scanned: momentum and
        charge flipped) of each partition's top-ranked complete set; NaN where none."""
        pair = self.pair.cpu().numpy()
        seeds = [s.final_seed.cpu().numpy().reshape(self.n_part, self.F, 6) for s in self.sides]
        out = np.full((self.n_part, 2, 6), np.nan)
        for p in range(self.n_part):
            k = int(pair[p, 0])
            if k >= 0:
                out[p, 0] = seeds[0][p, k // self.F]
                out[p, 1] = seeds[1][p, k % self.F]
        return out
