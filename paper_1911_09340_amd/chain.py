"""The paper's per-stage chain (Sec. 3.1), batched over events.

Stage s takes, for every event still active, its turn partition n_turns - 1 - s (the
reconstruction starts from the last turn) with the hits earlier stages left, and:
  1. entrance seed: the stage grid of the turn's transverse state at its outward
     crossing of the seed radius (the stand-in for the Hough-transform seed) with
     (z, p_z) true at stage 0 and from the backward extrapolation later
     (comet_stage_grids); exit seed: forwards from that seed to where the turn
     re-enters the seed region, momentum reversed (comet_exit_seeds), the transverse
     part again the turn's own (reversed) state;
  2. the hits split by side of the line through the chamber axis and the turn's circle
     centre (comet_half_split, comet_exclude_hits twice), each half's wire layers
     (comet_wire_layers);
  3. each half scanned with several references (multiref.MultiRefScan: a first grid,
     sparse references, finer re-scans, n_final final seeds and their half sets), the
     exit half with the charge reversed and both with half the steps of a turn;
  4. the missing-layer veto on each side (comet_layer_veto) and the combinatorial merge
     of the complete sets (comet_merge_halves);
  5. the best complete set (comet_union_halves): its entrance seed and the union of its
     two half sets on the stage's hits;
  6. with fit_iters > 0, Levenberg-Marquardt on Eq. 1 from that seed over the stage's
     hits (the fitted track); the self-refining of the union at the fitted track
     (comet_self_refine: lambda re-test, eta re-admission);
  7. the stage's hits recorded and excluded (comet_stage_record, comet_exclude_hits),
     the fitted seed extrapolated backwards (comet_backward_seeds), the stop rule
     (comet_stage_update).
This module owns the buffers and orders the launches; no host synchronisation.
"""
from __future__ import annotations

import numpy as np
import torch

from . import comet, multiref, scan, stages, synth


class StageChainRunner:
    def __init__(self, events, scan_cfg: synth.ScanConfig, max_stages: int = 5,
                 min_wires: int = 30, max_back_steps: int = 4000, n_ref: int = 10,
                 n_iter: int = 2, n_fine=(4, 8, 8, 8), n_final: int = 10, half_steps=None,
                 fit_iters: int = 8, eta: float = 0.3, mu0: float = 1e-3, device="cuda"):
        self.events = list(events)
        E = self.n_events = len(self.events)
        self.sc = scan_cfg
        self.max_stages, self.min_wires = int(max_stages), int(min_wires)
        self.max_back_steps = int(max_back_steps)
        self.fit_iters, self.eta, self.mu0 = int(fit_iters), float(eta), float(mu0)
        self.F = int(n_final)
        ev0 = self.events[0]
        steps_half = int(half_steps) if half_steps else scan_cfg.n_steps // 2
        self.half_steps = steps_half
        # the whole turn: fit, self-refining, exit seeds, backward extrapolation
        self.cfg = scan.config_for(ev0, scan_cfg)
        # entrance and exit halves (the exit half runs backwards: charge reversed)
        self.cfg_half = (comet.make_config(ev0.bz, ev0.charge, scan_cfg.step_mm, steps_half,
                                           scan_cfg.lambda_mm),
                         comet.make_config(ev0.bz, -ev0.charge, scan_cfg.step_mm, steps_half,
                                           scan_cfg.lambda_mm))
        self.packed0 = stages.StagePacked.from_events(self.events, device)
        self.bufs = [self.packed0.empty_like(), self.packed0.empty_like()]
        self.half_packed = [self.packed0.empty_like(), self.packed0.empty_like()]
        n_h = self.n_hits = int(self.packed0.drift.shape[0])
        n_w = int(self.packed0.wire_ends.shape[0])
        # per stage and event: the turn's transverse states, the side of every hit
        tr = np.empty((2, self.max_stages, E, 6))
        side = np.zeros((self.max_stages, max(n_h, 1)), np.uint8)
        layer = np.zeros(max(n_h, 1), np.int32)
        h0 = 0
        for e, ev in enumerate(self.events):
            counts = np.diff(ev.wire_offsets)
            layer[h0:h0 + ev.n_hits] = np.repeat(synth.wire_layers(ev.wire_ids), counts)
            for s in range(self.max_stages):
                t = max(ev.n_turns - 1 - s, 0)
                tr[0, s, e] = ev.ref_states[t]
                ex = ev.exit_states[t]
                tr[1, s, e] = np.concatenate([ex[:3], -ex[3:]])
                side[s, h0:h0 + ev.n_hits] = np.repeat(synth.entrance_sides(ev, t), counts)
            h0 += ev.n_hits
        self.transverse = torch.as_tensor(tr, device=device)
        self.side = torch.as_tensor(side, device=device)
        self.hit_layer = torch.as_tensor(layer, device=device)
        turns = np.array([ev.n_turns for ev in self.events], np.int32)
        self.n_turns = torch.as_tensor(turns, device=device)
        active0 = np.array([ev.n_wires >= self.min_wires for ev in self.events], np.int32)
        self.active0 = torch.as_tensor(active0, device=device)
        self.active = self.active0.clone()
        self.part_event = torch.arange(E, dtype=torch.int32, device=device)
        self.stride = max(max(ev.n_hits for ev in self.events), 1)
        f64 = dict(dtype=torch.float64, device=device)
        u8 = dict(dtype=torch.uint8, device=device)
        i32 = dict(dtype=torch.int32, device=device)
        self.exit_state = torch.empty(E, 6, **f64)
        self.excl = [torch.empty(max(n_h, 1), **u8) for _ in range(2)]
        self.wire_layer = [torch.empty(max(n_w, 1), **i32) for _ in range(2)]
        self.sides = [multiref.MultiRefScan(self.part_event, scan_cfg.n, n_fine, n_ref, n_iter,
                                            self.F, self.stride, n_w, steps_half, device)
                      for _ in range(2)]
        self.veto = [torch.empty(E * self.F, **i32) for _ in range(2)]
        self.pair = torch.empty(E, self.F * self.F, **i32)
        self.pair_rss = torch.empty(E, self.F * self.F, **f64)
        self.n_complete = torch.empty(E, **i32)
        self.mask = torch.zeros(E, self.stride, **u8)
        self.chosen = torch.empty(self.max_stages, E, 6, **f64)
        self.best = torch.empty(self.max_stages, E, dtype=torch.int64, device=device)
        self.fitted = torch.empty(self.max_stages, E, 6, **f64)
        self.ext = torch.empty(E, 6, **f64)
        self.stage_of_hit = torch.empty(max(n_h, 1), **i32)
        self.exclude = torch.empty(max(n_h, 1), **u8)
        self.ex_workspace = comet.exclude_workspace(E, device)
        self.active_after = torch.empty(self.max_stages, E, **i32)
        self.n_complete_at = torch.empty(self.max_stages, E, **i32)
        if self.fit_iters > 0:
            self.fit_soa = torch.empty(6, E, **f64)
            self.fit_rss = torch.empty(E, **f64)
            self.lm_ws = comet.lm_workspace(E, scan_cfg.n_steps, device)

    @property
    def evals_per_stage(self) -> int:
        """Seed x hit evaluations of one stage when every event is active (each half
        scans its own hits; at most all of the event's hits)."""
        hits = sum(ev.n_hits for ev in self.events)
        return hits * self.sides[0].seeds_per_partition

    def run(self) -> None:
        E, F = self.n_events, self.F
        self.stage_of_hit.fill_(-1)
        self.active.copy_(self.active0)
        for s in range(self.max_stages):
            src = self.packed0 if s == 0 else self.bufs[(s - 1) % 2]
            dst = self.bufs[s % 2]
            ent, ext = self.sides
            ext_in = self.transverse[0, 0] if s == 0 else self.ext
            # 1. seeds of both halves
            comet.stage_grids(self.transverse[0, s], ext_in, self.sc.half, ent.grids0)
            comet.exit_seeds(ent.grids0, 14, self.cfg, synth.SEED_RADIUS,
                             self.max_back_steps, self.exit_state)
            comet.stage_grids(self.transverse[1, s], self.exit_state, self.sc.half, ext.grids0)
            # 2. the halves' hits and wire layers
            comet.half_split(src, self.side[s], self.excl[0], self.excl[1])
            for k in range(2):
                comet.exclude_hits(src, self.excl[k], self.half_packed[k], self.ex_workspace)
                comet.wire_layers(self.half_packed[k], self.hit_layer, self.wire_layer[k])
            # 3.-4. several references on each half, veto, merge
            for k, side in enumerate(self.sides):
                side.run(self.half_packed[k], self.cfg_half[k], event_active=self.active)
                comet.layer_veto(side.mask, side.part_event_f, self.half_packed[k],
                                 self.wire_layer[k], synth.N_LAYERS, self.veto[k])
            comet.merge_halves(ent.final_rss, self.veto[0].view(E, F), ext.final_rss,
                               self.veto[1].view(E, F), self.pair, self.pair_rss, self.n_complete)
            self.n_complete_at[s].copy_(self.n_complete)
            # 5. the best complete set on the stage's hits
            comet.union_halves(self.pair, self.n_complete, F, src, self.side[s], ent.mask,
                               ext.mask, ent.final_seed, self.active, self.mask, self.chosen[s],
                               self.best[s])
            # 6. fit and self-refining
            if self.fit_iters > 0:
                self.fit_soa.copy_(self.chosen[s].t())
                comet.lm_refine(self.fit_soa, self.cfg, src.wire_ends, src.wire_offsets,
                                src.drift, self.fit_iters, self.mu0, self.fit_rss, self.lm_ws,
                                event_wires=src.event_wires, seed_event=self.part_event)
                self.fitted[s].copy_(self.fit_soa.t())
            else:
                self.fitted[s].copy_(self.chosen[s])
            comet.self_refine(self.fitted[s], self.part_event, self.cfg, src, self.eta,
                              self.mask, self.mask)
            # 7. record, exclude, extrapolate backwards, stop rule
            comet.stage_record(self.mask, src, self.active, s, self.stage_of_hit, self.exclude)
            comet.exclude_hits(src, self.exclude, dst, self.ex_workspace)
            comet.backward_seeds(self.fitted[s], self.cfg, synth.SEED_RADIUS,
                                 self.max_back_steps, self.ext)
            comet.stage_update(self.active, self.best[s], dst.event_wires, self.n_turns, s,
                               self.max_stages, self.min_wires)
            self.active_after[s].copy_(self.active)

    def turn_masks(self) -> list:
        """Per event, [n_turns, n_hits] masks of the hits each stage classified (the
        stage that scanned turn t is n_turns - 1 - t)."""
        soh = self.stage_of_hit.cpu().numpy()
        out, h0 = [], 0
        for ev in self.events:
            m = np.zeros((ev.n_turns, ev.n_hits), np.uint8)
            part = soh[h0:h0 + ev.n_hits]
            for s in range(min(ev.n_turns, self.max_stages)):
                m[ev.n_turns - 1 - s] = part == s
            out.append(m)
            h0 += ev.n_hits
        return out
