"""The stage loop of the event reconstruction (Sec. 3.1), batched over events.

Stage s scans, for every event still active, its turn partition n_turns - 1 - s (the
reconstruction starts from the last turn). The grid's transverse seed is the turn's
true state at the seed radius (the stand-in for the paper's Hough-transform seed); its
longitudinal seed (z, p_z) is the true one at stage 0 (the stand-in for the hodoscope
prior of the last turn) and, later, the previous stage's chosen seed extrapolated
backwards by one turn (comet_backward_seeds). Per stage, on the device:
  comet_stage_grids -> comet_batch_scan_active (scan, re-scans, classification of the
     events still active; the others are skipped)
  [with n_z > 1, the seed's z as a fifth axis (Sec. 3.1: five degrees of freedom):
     comet_stage_grids_z (n_z values of z over ext z +- z_half) -> one scan of all n_z
     grids -> comet_sparse_select (the lowest RSS of the n_z grids, the grid re-centred
     on it, z kept) -> comet_batch_scan_active from that grid with n_refine - 1 re-scans]
  [-> with fit_iters > 0: comet_lm_refine from the chosen seed (the fitted track) and
     comet_self_refine (classified hits re-tested with lambda at the fitted track, wires
     left without one re-admit their closest hit below eta)]
  -> comet_stage_record (the classified hits get the stage number and are marked)
  -> comet_exclude_hits (later stages scan only the hits left)
  -> comet_backward_seeds (from the fitted seed when there is a fit)
  -> comet_stage_update (stop when fewer than min_wires wires
     remain, when max_stages tracks were found or when the event has no turn left).
This module owns the buffers and orders the launches; no host synchronisation.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import comet, scan, synth


@dataclass
class StagePacked:
    """Packed events (CSR as scan.PackedEvents) plus each hit's original index."""
    wire_ends: torch.Tensor
    wire_offsets: torch.Tensor
    drift: torch.Tensor
    event_wires: torch.Tensor
    hit_ids: torch.Tensor

    @classmethod
    def from_events(cls, events, device="cuda"):
        p = scan.PackedEvents.from_events(events, device)
        n_h = int(p.drift.shape[0])
        return cls(p.wire_ends, p.wire_offsets, p.drift, p.event_wires,
                   torch.arange(n_h, dtype=torch.int32, device=device))

    def empty_like(self):
        return StagePacked(*(torch.empty_like(t) for t in (self.wire_ends, self.wire_offsets,
                                                           self.drift, self.event_wires,
                                                           self.hit_ids)))


class StageRunner:
    def __init__(self, events, scan_cfg: synth.ScanConfig, max_stages: int = 5,
                 min_wires: int = 30, max_back_steps: int = 4000, fit_iters: int = 0,
                 eta: float = 0.3, mu0: float = 1e-3, device="cuda", n_z: int = 1,
                 z_half: float = 0.0):
        self.events = list(events)
        self.sc = scan_cfg
        self.n_z, self.z_half = int(n_z), float(z_half)
        if self.n_z > 1 and scan_cfg.n_refine < 1:
            raise ValueError("a z axis needs at least one re-scan (n_refine >= 1)")
        self.max_stages, self.min_wires = int(max_stages), int(min_wires)
        self.max_back_steps = int(max_back_steps)
        self.fit_iters, self.eta, self.mu0 = int(fit_iters), float(eta), float(mu0)
        E = self.n_events = len(self.events)
        self.cfg = scan.config_for(self.events[0], scan_cfg)
        # stage 0 reads the events as given; later stages alternate between two buffers
        self.packed0 = StagePacked.from_events(self.events, device)
        self.bufs = [self.packed0.empty_like(), self.packed0.empty_like()]
        self.n_hits = int(self.packed0.drift.shape[0])
        turns = np.array([ev.n_turns for ev in self.events], np.int32)
        self.n_turns = torch.as_tensor(turns, device=device)
        tr = np.empty((self.max_stages, E, 6))
        for s in range(self.max_stages):
            for e, ev in enumerate(self.events):
                tr[s, e] = ev.ref_states[max(ev.n_turns - 1 - s, 0)]
        self.transverse = torch.as_tensor(tr, device=device)
        active0 = np.array([ev.n_wires >= self.min_wires for ev in self.events], np.int32)
        self.active0 = torch.as_tensor(active0, device=device)
        self.active = self.active0.clone()
        f64 = dict(dtype=torch.float64, device=device)
        S = scan_cfg.n_seeds
        self.part_event = torch.arange(E, dtype=torch.int32, device=device)
        self.grids = torch.empty(E, 14, **f64)
        self.rss = torch.empty(E, S, **f64)
        self.best = torch.empty(max(self.max_stages, 1), E, dtype=torch.int64, device=device)
        self.seeds = torch.empty(self.max_stages, E, 6, **f64)
        self.best_rss = torch.empty(self.max_stages, E, **f64)
        self.ext = torch.empty(E, 6, **f64)
        self.stride = max(max(ev.n_hits for ev in self.events), 1)
        self.mask = torch.zeros(E, self.stride, dtype=torch.uint8, device=device)
        self.n_border = torch.empty(E, dtype=torch.int32, device=device)
        self.stage_of_hit = torch.empty(self.n_hits, dtype=torch.int32, device=device)
        self.exclude = torch.empty(self.n_hits, dtype=torch.uint8, device=device)
        self.workspace = comet.batch_workspace(int(self.packed0.wire_ends.shape[0]),
                                               scan_cfg.n_steps, E, device)
        self.ex_workspace = comet.exclude_workspace(E, device)
        self.active_after = torch.empty(self.max_stages, E, dtype=torch.int32, device=device)
        # the fitted seed of every stage (the chosen seed itself without a fit)
        self.fitted = torch.empty(self.max_stages, E, 6, **f64)
        if self.fit_iters > 0:
            self.fit_soa = torch.empty(6, E, **f64)
            self.fit_rss = torch.empty(E, **f64)
            self.lm_ws = comet.lm_workspace(E, scan_cfg.n_steps, device)
        if self.n_z > 1:
            Z = self.n_z
            self.part_event_z = torch.arange(E, dtype=torch.int32,
                                             device=device).repeat_interleave(Z)
            self.grids_z = torch.empty(E, Z, 14, **f64)
            self.rss_z = torch.empty(E * Z, S, **f64)
            self.best_z = torch.empty(E * Z, dtype=torch.int64, device=device)
            self.ref_z = torch.empty(E, 1, dtype=torch.int64, device=device)
            self.grids_ref = torch.empty(E, 1, 14, **f64)
            self.workspace_z = comet.batch_workspace(int(self.packed0.wire_ends.shape[0]),
                                                     scan_cfg.n_steps, E * Z, device)

    def run(self) -> None:
        self.stage_of_hit.fill_(-1)
        self.active.copy_(self.active0)
        for s in range(self.max_stages):
            src = self.packed0 if s == 0 else self.bufs[(s - 1) % 2]
            dst = self.bufs[s % 2]
            ext = self.transverse[0] if s == 0 else self.ext
            if self.n_z > 1:
                # the z sub-grids: one scan of all, the lowest RSS over each event's grids
                # (lowest sub-grid and seed index on ties), its grid re-centred on it
                comet.stage_grids_z(self.transverse[s], ext, self.sc.half, self.n_z,
                                    self.z_half, self.grids_z)
                comet.batch_scan(src, self.part_event_z, self.grids_z.view(-1, 14), self.sc.n,
                                 self.cfg, 0, self.rss_z, self.best_z, self.workspace_z,
                                 event_active=self.active)
                comet.sparse_select(self.grids_z, self.rss_z.view(self.n_events, self.n_z, -1),
                                    self.sc.n, 1, self.ref_z, self.grids_ref)
                comet.batch_scan(src, self.part_event, self.grids, self.sc.n, self.cfg,
                                 self.sc.n_refine - 1, self.rss, self.best[s], self.workspace,
                                 best_seed=self.seeds[s], best_rss=self.best_rss[s],
                                 hit_mask=self.mask, n_borderline=self.n_border,
                                 grids_init=self.grids_ref.view(-1, 14),
                                 event_active=self.active)
            else:
                comet.stage_grids(self.transverse[s], ext, self.sc.half, self.grids)
                comet.batch_scan(src, self.part_event, self.grids, self.sc.n, self.cfg,
                                 self.sc.n_refine, self.rss, self.best[s], self.workspace,
                                 best_seed=self.seeds[s], best_rss=self.best_rss[s],
                                 hit_mask=self.mask, n_borderline=self.n_border,
                                 event_active=self.active)
            if self.fit_iters > 0:
                self.fit_soa.copy_(self.seeds[s].t())
                comet.lm_refine(self.fit_soa, self.cfg, src.wire_ends, src.wire_offsets,
                                src.drift, self.fit_iters, self.mu0, self.fit_rss, self.lm_ws,
                                event_wires=src.event_wires, seed_event=self.part_event)
                self.fitted[s].copy_(self.fit_soa.t())
                comet.self_refine(self.fitted[s], self.part_event, self.cfg, src, self.eta,
                                  self.mask, self.mask)
            else:
                self.fitted[s].copy_(self.seeds[s])
            comet.stage_record(self.mask, src, self.active, s, self.stage_of_hit, self.exclude)
            comet.exclude_hits(src, self.exclude, dst, self.ex_workspace)
            comet.backward_seeds(self.fitted[s], self.cfg, synth.SEED_RADIUS,
                                 self.max_back_steps, self.ext)
            comet.stage_update(self.active, self.best[s], dst.event_wires, self.n_turns, s,
                               self.max_stages, self.min_wires)
            self.active_after[s].copy_(self.active)

    # ---------------------------------------------------------- host-side reporting
    def turn_masks(self) -> list:
        """Per event, [n_turns, n_hits] bit-0 masks: the hits classified to each turn (the
        stage that scanned it), from stage_of_hit."""
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
