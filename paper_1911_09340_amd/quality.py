"""Hit-classification efficiency and purity (Sec. 3.2.1) from the synthetic truth labels.

The hits classified for a turn partition are split by their true turn index; the
turn of the largest subset is the one the set represents (noise hits, labelled -1,
never represent a turn but count in the set's size). Efficiency = size of that
subset / number of hits the represented turn induced; purity = size of that subset
/ number of classified hits. A partition that classified nothing has efficiency 0
and no purity. This is host-side reporting on copied-back masks, not part of the
scan.
"""
from __future__ import annotations

import numpy as np


def turn_metrics(mask_row: np.ndarray, hit_turn: np.ndarray):
    """(efficiency, purity, represented turn) of one partition's bit-0 mask."""
    sel = (np.asarray(mask_row) & 1).astype(bool)
    turns = hit_turn[sel]
    signal = turns[turns >= 0]
    if sel.sum() == 0 or signal.size == 0:
        return 0.0, (float("nan") if sel.sum() == 0 else 0.0), -1
    ids, counts = np.unique(signal, return_counts=True)
    k = int(np.argmax(counts))          # ties: the lower turn index
    t = int(ids[k])
    return float(counts[k] / np.sum(hit_turn == t)), float(counts[k] / sel.sum()), t


def classification(mask: np.ndarray, events) -> dict:
    """Per-partition metrics over all partitions (partition order: events in order,
    turns in order) and their means."""
    eff, pur, same = [], [], []
    p = 0
    for ev in events:
        for t in range(ev.n_turns):
            e, u, rep = turn_metrics(mask[p, :ev.n_hits], ev.hit_turn)
            eff.append(e)
            pur.append(u)
            same.append(rep == t)
            p += 1
    eff, pur = np.asarray(eff), np.asarray(pur)
    return {"efficiency_mean": float(np.mean(eff)),
            "purity_mean": float(np.nanmean(pur)) if np.any(~np.isnan(pur)) else float("nan"),
            "represents_own_turn": float(np.mean(same)),
            "eff_and_purity_above_0.9": float(np.mean((eff > 0.9) & (np.nan_to_num(pur) > 0.9))),
            "partitions": int(p)}
