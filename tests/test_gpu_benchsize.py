"""Parity at the benchmark's own sizes and on the classification's borderline.

- One turn partition of the signal workload exactly as the benchmark runs it: a 16^4
  grid (65 536 seeds), 1500 x 2 mm, two finer re-scans and the classification, in the
  DCA shape the autotuner picks on the live buffers. Every intermediate (each scan's
  grid, its whole RSS row and its choice) and the final seed, RSS and hit mask are
  compared with the CPU reference bit for bit (Sec. 2.1).
- The whole first-scan RSS row of the other two turn partitions.
- Hits placed on the cutoff: drift distances set from the CPU reference's D of a fixed
  seed so that |D - r| equals lambda exactly or misses it by 3e-10, 5e-10 or 2e-9 mm,
  on single- and multi-hit wires. The strict rule |e| < lambda and the borderline bit
  (| |e| - lambda | < 1e-9) must agree through comet_select_classify and
  comet_batch_classify.
"""
from types import SimpleNamespace

import numpy as np
import pytest
import torch

from paper_1911_09340_amd import comet, scan, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    torch.cuda.set_device(0)
    comet.load()
    yield
    comet.set_dca_variant(-1)


def _n(*n):
    return np.array(n, dtype=np.int32)


def _ocfg(ev, sc):
    return [ev.bz, ev.charge, sc.step_mm, sc.lambda_mm]


def test_signal_partition_end_to_end_in_bench_configuration(orc, ev_signal):
    ev, sc, turn = ev_signal, synth.C1, 0
    cfg = scan.config_for(ev, sc)
    dev = scan.DeviceEvent.from_event(ev)
    g0 = synth.grid_descriptor(ev.ref_states[turn], sc)
    n = _n(*sc.n)
    runner = scan.PartitionScanner(sc.n, cfg, ev.n_wires, ev.n_hits)
    grid0 = torch.as_tensor(g0, device="cuda")
    # as the benchmark: the autotuner picks the shape on the live buffers of the first scan
    runner.run(dev, grid0, sc.n_refine)
    runner.run(dev, grid0, 0)
    tuned, _ = comet.dca_autotune(runner.track, dev.wire_ends, dev.wire_offsets, dev.drift, cfg,
                                  runner.rss, runner.workspace, reps=1)
    assert comet.dca_variant_for(sc.n_seeds, sc.n_steps + 1, ev.n_wires) == tuned
    print("DCA shape", tuned, comet.dca_variants()[tuned], flush=True)
    snaps = []

    def keep(it, r):
        snaps.append((r.grid.clone(), r.rss.clone(), r.best.clone()))

    runner.run(dev, grid0, sc.n_refine, on_scan=keep)
    torch.cuda.synchronize()
    got = runner.result()
    ocfg = _ocfg(ev, sc)
    g = g0.copy()
    b = -1
    for it in range(sc.n_refine + 1):
        if it > 0:
            g = orc.refine_grid(g, n, b)
        rss, _ = orc.scan(orc.seed_grid(g, n), ocfg, sc.n_steps, ev.wire_ends, ev.wire_offsets,
                          ev.drift)
        b = orc.argmin(rss)
        grid_d, rss_d, best_d = (t.cpu().numpy() for t in snaps[it])
        assert np.array_equal(grid_d, g), ("grid", it)
        assert np.array_equal(rss_d, rss), ("rss row", it, int(np.sum(rss_d != rss)))
        assert int(best_d[0]) == b, ("best", it, int(best_d[0]), b)
    seed = orc.seed(g, n, b)
    mask, dca, nb = orc.classify(seed, ocfg, sc.n_steps, ev.wire_ends, ev.wire_offsets, ev.drift)
    assert got["best"] == b and np.array_equal(got["best_seed"], seed)
    assert got["best_rss"] == rss[b]
    assert np.array_equal(got["mask"], mask) and got["n_borderline"] == nb
    assert np.array_equal(got["dca_best"], dca)
    assert int((mask & 1).sum()) > 50


@pytest.mark.parametrize("turn", [1, 2])
def test_signal_first_scan_whole_row(orc, ev_signal, turn):
    ev, sc = ev_signal, synth.C1
    cfg = scan.config_for(ev, sc)
    g = synth.grid_descriptor(ev.ref_states[turn], sc)
    n = _n(*sc.n)
    seeds = torch.empty(6, sc.n_seeds, dtype=torch.float64, device="cuda")
    comet.seed_grid(torch.as_tensor(g, device="cuda"), n, seeds)
    dev = scan.DeviceEvent.from_event(ev)
    track = torch.empty(3, sc.n_steps + 1, sc.n_seeds, dtype=torch.float64, device="cuda")
    rss = torch.empty(sc.n_seeds, dtype=torch.float64, device="cuda")
    ws = comet.dca_workspace(sc.n_seeds, sc.n_steps + 1, ev.n_wires)
    comet.track_dca_rss(seeds, dev.wire_ends, dev.wire_offsets, dev.drift, cfg, track, rss, ws)
    best = torch.empty(1, dtype=torch.int64, device="cuda")
    comet.select_classify(rss, best, cfg)
    want, _ = orc.scan(orc.seed_grid(g, n), _ocfg(ev, sc), sc.n_steps, ev.wire_ends,
                       ev.wire_offsets, ev.drift)
    got = rss.cpu().numpy()
    assert np.array_equal(got, want), int(np.sum(got != want))
    assert int(best.item()) == orc.argmin(want)


def _borderline_event(orc, ev, seed, cfg, K):
    """The event's wires with drift distances placed around |D - r| = lambda."""
    lam = cfg[3]
    _, D, _ = orc.classify(seed, cfg, K, ev.wire_ends, ev.wire_offsets, ev.drift)
    patterns = [
        [0.0],                      # |e| = lambda (exactly where D - lambda is exact)
        [5e-10],                    # just inside: classified, borderline
        [-5e-10],                   # just outside: borderline
        [2e-9],                     # inside, not borderline
        [-2e-9],                    # outside, not borderline
        ["+"],                      # r = D + lambda: e = -lambda
        [-3e-10, 3e-10],            # the second hit is closer
        [3e-10, "+3e-10"],          # both |e| = lambda - 3e-10 (up to rounding): first on ties
        [0.0, "+"],                 # both |e| = lambda
        [],                         # a wire without hits
        [-1e-9, 1e-9, 0.0],
    ]
    offs, drift = [0], []
    for i in range(ev.n_wires):
        for v in patterns[i % len(patterns)]:
            if v == "+":
                r = D[i] + lam
            elif v == "+3e-10":
                r = (D[i] + lam) - 3e-10
            else:
                r = (D[i] - lam) + v
            drift.append(r)
        offs.append(len(drift))
    return SimpleNamespace(wire_ends=ev.wire_ends, wire_offsets=np.asarray(offs, np.int32),
                           drift=np.asarray(drift, np.float64), n_wires=ev.n_wires,
                           n_hits=len(drift), n_turns=1)


@pytest.mark.parametrize("lam", [1.0, 0.8])
def test_borderline_hits_select_and_batch_classify(orc, ev_plain, lam):
    ev = ev_plain
    sc = synth.ScanConfig("border", (1, 1, 1, 1), (0.0, 0.0, 0.0, 0.0), 1000, 2.0, lam, 0)
    g = synth.grid_descriptor(ev.ref_states[0], sc)
    n = _n(1, 1, 1, 1)
    seed = orc.seed(g, n, 0)
    ocfg = [ev.bz, ev.charge, sc.step_mm, lam]
    bev = _borderline_event(orc, ev, seed, ocfg, sc.n_steps)
    wmask, wdca, wnb = orc.classify(seed, ocfg, sc.n_steps, bev.wire_ends, bev.wire_offsets,
                                    bev.drift)
    e_exact = sum(1 for i in range(0, bev.n_wires, 11)
                  if abs(wdca[i] - bev.drift[bev.wire_offsets[i]]) == lam)
    print("lambda", lam, "borderline", wnb, "classified", int((wmask & 1).sum()),
          "wires with |e| == lambda exactly", e_exact, flush=True)
    assert wnb >= bev.n_wires // 3 and int((wmask & 1).sum()) > 0
    if lam == 1.0:
        assert e_exact > 0
    cfg = scan.config_for(ev, sc)
    dev = scan.DeviceEvent.from_event(bev)
    seeds = torch.empty(6, 1, dtype=torch.float64, device="cuda")
    comet.seed_grid(torch.as_tensor(g, device="cuda"), n, seeds)
    track = torch.empty(3, sc.n_steps + 1, 1, dtype=torch.float64, device="cuda")
    comet.extrapolate_seeds(seeds, cfg, track)
    rss = torch.zeros(1, dtype=torch.float64, device="cuda")
    best = torch.empty(1, dtype=torch.int64, device="cuda")
    mask = torch.full((bev.n_hits,), 9, dtype=torch.uint8, device="cuda")
    nb = torch.empty(1, dtype=torch.int32, device="cuda")
    dca = torch.empty(bev.n_wires, dtype=torch.float64, device="cuda")
    comet.select_classify(rss, best, cfg, track, dev.wire_ends, dev.wire_offsets, dev.drift,
                          hit_mask=mask, n_borderline=nb, dca_best=dca)
    assert int(best.item()) == 0
    assert np.array_equal(dca.cpu().numpy(), wdca)
    assert np.array_equal(mask.cpu().numpy(), wmask)
    assert int(nb.item()) == wnb
    # the batched classification of the same seed (grid of one point, best index 0)
    packed = scan.PackedEvents.from_events([bev])
    part_event = torch.zeros(1, dtype=torch.int32, device="cuda")
    grids = torch.as_tensor(g[None, :].copy(), device="cuda")
    bbest = torch.zeros(1, dtype=torch.int64, device="cuda")
    bmask = torch.full((1, bev.n_hits + 3), 9, dtype=torch.uint8, device="cuda")
    bnb = torch.empty(1, dtype=torch.int32, device="cuda")
    bseed = torch.empty(1, 6, dtype=torch.float64, device="cuda")
    comet.batch_classify(packed, part_event, grids, n, cfg, bbest, best_seed=bseed,
                         hit_mask=bmask, n_borderline=bnb)
    torch.cuda.synchronize()
    assert np.array_equal(bseed.cpu().numpy()[0], seed)
    assert np.array_equal(bmask.cpu().numpy()[0, :bev.n_hits], wmask)
    assert int(bnb.item()) == wnb
