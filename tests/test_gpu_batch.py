"""Batched persistent path (many uneven events) vs the single-event path and the CPU
reference; top-k selection; HIP-graph capture and replay."""
from dataclasses import replace

import numpy as np
import pytest
import torch

import oracle
from paper_1911_09340_amd import comet, refine, scan, synth

pytestmark = pytest.mark.gpu

SC = synth.ScanConfig("batch-test", (2, 4, 5, 7), (5.0, 5.0, 0.05, 0.05), 1000, 2.0, 0.8, 2)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    torch.cuda.set_device(0)
    comet.load()
    yield
    comet.set_batch_variant(0)


@pytest.fixture(scope="module")
def events():
    return [synth.event_mix(i) for i in range(6)]


def _single(ev, turn, sc):
    cfg = scan.config_for(ev, sc)
    r = scan.PartitionScanner(sc.n, cfg, ev.n_wires, ev.n_hits)
    r.run(scan.DeviceEvent.from_event(ev), scan.grid_tensor(ev.ref_states[turn], sc), sc.n_refine)
    torch.cuda.synchronize()
    out = r.result()
    out["rss"] = r.rss.cpu().numpy()
    return out


def _check_against_single(runner, events, sc):
    rss = runner.rss.cpu().numpy()
    best = runner.best.cpu().numpy()
    grids = runner.grids.cpu().numpy()
    seeds = runner.best_seed.cpu().numpy()
    brss = runner.best_rss.cpu().numpy()
    mask = runner.mask.cpu().numpy()
    nb = runner.n_border.cpu().numpy()
    p = 0
    for ev in events:
        for t in range(ev.n_turns):
            want = _single(ev, t, sc)
            assert best[p] == want["best"], p
            assert np.array_equal(grids[p], want["grid"]), p
            assert np.array_equal(rss[p], want["rss"]), p
            assert np.array_equal(seeds[p], want["best_seed"]), p
            assert brss[p] == want["best_rss"], p
            assert np.array_equal(mask[p, :ev.n_hits], want["mask"]), p
            assert nb[p] == want["n_borderline"], p
            p += 1


# 26 tiles per partition (the last one half full): several work items per partition
SC_WIDE = synth.ScanConfig("batch-wide", (3, 4, 8, 17), (5.0, 5.0, 0.05, 0.05), 700, 2.0, 0.8, 1)


def test_batch_equals_single_event_path(events):
    runner = scan.BatchRunner(events, SC)
    assert runner.n_part == sum(ev.n_turns for ev in events) and runner.n_part > 6
    runner.run()
    torch.cuda.synchronize()
    _check_against_single(runner, events, SC)


def test_batch_many_tiles_per_partition(events):
    for i in range(len(comet.batch_variants())):
        comet.set_batch_variant(i)
        runner = scan.BatchRunner(events[:3], SC_WIDE)
        runner.run()
        torch.cuda.synchronize()
        _check_against_single(runner, events[:3], SC_WIDE)
    comet.set_batch_variant(0)


def test_batch_azimuth_shapes_on_an_event_past_their_wire_limit(events):
    """The shapes that take each event's wires in azimuth order keep the d^2 of
    3 (K + 1) + (K / 16 + 2) wires per wave; an event with more (here ~1200 wires, most of
    them noise, at K = 300: a limit of 923) takes the wires in wire order. Every such shape
    gives the bits of shape 0 on it and on a normal event."""
    import numpy as np
    from dataclasses import replace
    sc = replace(SC, n_steps=300)
    big = synth.event_mix(3, noise_frac=0.85, hits=(1000, 2000))
    assert big.n_wires > 3 * 301 + 301 // 16 + 2 and events[0].n_wires < 900
    evs = [big, events[0]]
    az = [i for i, v in enumerate(comet.batch_variants()) if v["form"].startswith("wide_cap_az")]
    assert az
    ref = None
    for i in [0] + az:
        comet.set_batch_variant(i)
        runner = scan.BatchRunner(evs, sc)
        runner.run()
        got = (runner.rss.cpu().numpy(), runner.best.cpu().numpy(), runner.mask.cpu().numpy())
        if ref is None:
            ref = got
        else:
            for a, b in zip(got, ref):
                assert np.array_equal(a, b), i
    comet.set_batch_variant(0)


def test_batch_every_shape_identical(events):
    ref = None
    for i in range(len(comet.batch_variants())):
        comet.set_batch_variant(i)
        runner = scan.BatchRunner(events[:3], SC)
        runner.run()
        mask = runner.mask.cpu().numpy()
        parts = [t for ev in events[:3] for t in range(ev.n_turns)]
        hits = [ev.n_hits for ev in events[:3] for _ in range(ev.n_turns)]
        masks = [mask[p, :h] for p, h in enumerate(hits)]
        assert len(parts) == runner.n_part
        got = (runner.rss.cpu().numpy(), runner.best.cpu().numpy(), *masks)
        if ref is None:
            ref = got
        else:
            assert all(np.array_equal(a, b) for a, b in zip(got, ref)), i
    comet.set_batch_variant(0)


def test_batch_every_shape_identical_on_a_blocked_grid(events):
    """A grid whose axes hold 2 x 2 x 4 x 4 blocks (2 x 4 x 8 x 8 = 512 seeds, 8 tiles):
    the blocked shapes take each tile as such a block and write every RSS to its seed's
    place; every shape must give the bits of shape 0 (RSS in grid order, best seeds,
    masks), also after a re-scan."""
    sc = synth.ScanConfig("blocked", (2, 4, 8, 8), (5.0, 5.0, 0.05, 0.05), 400, 2.0, 0.8, 1)
    ref = None
    try:
        for i in range(len(comet.batch_variants())):
            comet.set_batch_variant(i)
            runner = scan.BatchRunner(events[:3], sc)
            runner.run()
            got = (runner.rss.cpu().numpy(), runner.best.cpu().numpy(), runner.mask.cpu().numpy())
            if ref is None:
                ref = got
            else:
                for a, b in zip(got, ref):
                    assert np.array_equal(a, b), i
    finally:
        comet.set_batch_variant(0)


def test_batch_matches_cpu_reference(orc, events):
    runner = scan.BatchRunner(events[:2], SC)
    runner.run()
    torch.cuda.synchronize()
    p = 0
    for ev in events[:2]:
        for t in range(ev.n_turns):
            want = orc.scan_partition(synth.grid_descriptor(ev.ref_states[t], SC),
                                      np.array(SC.n, np.int32),
                                      [ev.bz, ev.charge, SC.step_mm, SC.lambda_mm], SC.n_steps,
                                      SC.n_refine, ev.wire_ends, ev.wire_offsets, ev.drift)
            assert int(runner.best[p]) == want["best"]
            assert np.array_equal(runner.rss[p].cpu().numpy(), want["rss"])
            assert np.array_equal(runner.best_seed[p].cpu().numpy(), want["best_seed"])
            assert np.array_equal(runner.mask[p, :ev.n_hits].cpu().numpy(), want["mask"])
            p += 1


def test_graph_capture_replays_match_eager(events):
    """Captured once, replayed several times with eager work in between."""
    runner = scan.BatchRunner(events[:4], SC)
    runner.run()
    torch.cuda.synchronize()
    eager = [t.clone() for t in (runner.rss, runner.best, runner.best_seed, runner.mask,
                                 runner.grids)]
    runner.capture()
    hits = [ev.n_hits for ev in events[:4] for _ in range(ev.n_turns)]
    for rep in range(3):
        for t in (runner.rss, runner.best_seed, runner.grids):
            t.fill_(float("nan"))
        runner.best.fill_(-7)
        runner.mask.fill_(7)  # entries past a partition's own hits are not outputs
        runner.replay()
        torch.cuda.synchronize()
        got = (runner.rss, runner.best, runner.best_seed, runner.grids)
        assert all(torch.equal(a, b) for a, b in zip(got, eager[:3] + eager[4:])), rep
        for p, h in enumerate(hits):
            assert torch.equal(runner.mask[p, :h], eager[3][p, :h]), (rep, p)
        _ = torch.randn(1000, device="cuda").sum().item()  # eager work between replays


@pytest.mark.parametrize("sc,max_items", [(SC, 3), (SC_WIDE, 37)])
def test_max_items_scans_a_prefix(events, sc, max_items):
    runner = scan.BatchRunner(events[:2], replace(sc, n_refine=0))
    runner.rss.fill_(-1.0)
    runner.run(max_items=max_items)
    torch.cuda.synchronize()
    flat = runner.rss.cpu().numpy().ravel()
    S = sc.n_seeds
    tiles = (S + 63) // 64
    done = np.zeros_like(flat, dtype=bool)
    for item in range(max_items):
        p, t = divmod(item, tiles)
        done[p * S + t * 64:p * S + min(S, (t + 1) * 64)] = True
    assert np.all(flat[done] >= 0) and np.all(flat[~done] == -1.0)
    # partitions scanned in full select their best seed; the others keep -1
    best = runner.best.cpu().numpy()
    for p in range(runner.n_part):
        full = (p + 1) * tiles <= max_items
        assert (best[p] >= 0) == full, (p, best[p])


def test_topk_matches_cpu_reference(orc):
    rng = np.random.default_rng(4)
    v = np.round(rng.normal(size=(3, 5000)), 2)
    v[0, rng.integers(0, 5000, 300)] = np.nan
    v[2, :] = np.nan
    v[2, 17] = 1.0
    out = torch.empty(3, 64, dtype=torch.int64, device="cuda")
    comet.topk(torch.as_tensor(v, device="cuda"), 64, out)
    for r in range(3):
        assert np.array_equal(out[r].cpu().numpy(), orc.topk(v[r], 64)), r


def test_select_classify_top_k(orc, ev_plain):
    sc = synth.C0
    g = synth.grid_descriptor(ev_plain.ref_states[0], sc)
    cfg = scan.config_for(ev_plain, sc)
    seeds = torch.empty(6, sc.n_seeds, dtype=torch.float64, device="cuda")
    comet.seed_grid(torch.as_tensor(g, device="cuda"), sc.n, seeds)
    track = torch.empty(3, sc.n_steps + 1, sc.n_seeds, dtype=torch.float64, device="cuda")
    comet.extrapolate_seeds(seeds, cfg, track)
    dev = scan.DeviceEvent.from_event(ev_plain)
    rss = torch.empty(sc.n_seeds, dtype=torch.float64, device="cuda")
    comet.dca_rss(track, dev.wire_ends, dev.wire_offsets, dev.drift, cfg, rss,
                  comet.dca_workspace(sc.n_seeds, sc.n_steps + 1, dev.n_wires))
    best = torch.empty(64, dtype=torch.int64, device="cuda")
    mask = torch.empty(ev_plain.n_hits, dtype=torch.uint8, device="cuda")
    comet.select_classify(rss, best, cfg, track, dev.wire_ends, dev.wire_offsets, dev.drift,
                          hit_mask=mask, top_k=64)
    want = orc.topk(rss.cpu().numpy(), 64)
    assert np.array_equal(best.cpu().numpy(), want)
    wmask, _, _ = orc.classify(orc.seed(g, np.array(sc.n, np.int32), int(want[0])),
                               [ev_plain.bz, ev_plain.charge, sc.step_mm, sc.lambda_mm],
                               sc.n_steps, ev_plain.wire_ends, ev_plain.wire_offsets,
                               ev_plain.drift)
    assert np.array_equal(mask.cpu().numpy(), wmask)


def test_grid_seeds_match_cpu_reference(orc, events):
    runner = scan.BatchRunner(events[:2], SC)
    idx = torch.tensor([[0, 5, SC.n_seeds - 1, -1]] * runner.n_part, dtype=torch.int64,
                       device="cuda")
    out = torch.empty(6, runner.n_part * 4, dtype=torch.float64, device="cuda")
    comet.grid_seeds(runner.grids0, SC.n, idx, out)
    got = out.cpu().numpy()
    g0 = runner.grids0.cpu().numpy()
    for p in range(runner.n_part):
        for r, i in enumerate([0, 5, SC.n_seeds - 1]):
            assert np.array_equal(got[:, p * 4 + r], orc.seed(g0[p], np.array(SC.n, np.int32), i))
        assert np.all(np.isnan(got[:, p * 4 + 3]))


@pytest.mark.parametrize("starts", ["sparse", "topk"])
def test_multistart_refinement_matches_cpu_lm(orc, events, starts):
    """coarse_then_lm: every start's LM result equals the CPU LM from the same start
    (the sparse references of Sec. 2.1, or the k lowest-RSS seeds)."""
    sc = synth.ScanConfig("c", (4, 4, 4, 4), (5.0, 5.0, 0.05, 0.05), 1000, 2.0, 0.8, 0)
    evs = events[:2]
    out = refine.coarse_then_lm(evs, sc, top_k=3, n_iter=6, starts=starts)
    final = out["refined"].cpu().numpy()
    p = 0
    o = oracle.Oracle()
    for ev in evs:
        cfg = [ev.bz, ev.charge, sc.step_mm, sc.lambda_mm]
        for t in range(ev.n_turns):
            g = synth.grid_descriptor(ev.ref_states[t], sc)
            seeds = o.seed_grid(g, np.array(sc.n, np.int32))
            rss, _ = o.scan(seeds, cfg, sc.n_steps, ev.wire_ends, ev.wire_offsets, ev.drift)
            if starts == "topk":
                first = o.topk(rss, 3)
            else:
                first, _, _, taken = o.sparse_select(g, rss, np.array(sc.n, np.int32), 3)
                assert taken == 3
            res = [o.lm_refine(seeds[:, i], cfg, sc.n_steps, ev.wire_ends, ev.wire_offsets,
                               ev.drift, 6, 1e-3) for i in first]
            best = min(range(3), key=lambda r: (res[r][1], r))
            ws = res[best][0]
            assert np.max(np.abs(final[:, p] - ws) / np.maximum(np.abs(ws), 1.0)) < 1e-7, p
            p += 1


def test_local_rescan_after_lm_matches_cpu(orc, events):
    """coarse_then_lm with the local re-scan: a finer grid around each partition's LM seed
    (stage-grid descriptor, half-spans of one coarse spacing), LM from its lowest seeds, and
    the lowest RSS of all: the same chain on the CPU reference, to the LM bar (1e-7)."""
    sc = synth.ScanConfig("c", (4, 4, 4, 4), (5.0, 5.0, 0.05, 0.05), 1000, 2.0, 0.8, 0)
    evs = events[:2]
    out = refine.coarse_then_lm(evs, sc, top_k=2, n_iter=4, local=(3, 3, 3, 3), local_topk=2,
                                local_iters=3)
    final = out["refined"].cpu().numpy()
    frss = out["rss"].cpu().numpy()
    half = [2 * h / (n - 1) for h, n in zip(sc.half, sc.n)]
    p = 0
    o = oracle.Oracle()
    for ev in evs:
        cfg = [ev.bz, ev.charge, sc.step_mm, sc.lambda_mm]
        for t in range(ev.n_turns):
            g = synth.grid_descriptor(ev.ref_states[t], sc)
            seeds = o.seed_grid(g, np.array(sc.n, np.int32))
            rss, _ = o.scan(seeds, cfg, sc.n_steps, ev.wire_ends, ev.wire_offsets, ev.drift)
            res = [o.lm_refine(seeds[:, i], cfg, sc.n_steps, ev.wire_ends, ev.wire_offsets,
                               ev.drift, 4, 1e-3) for i in o.topk(rss, 2)]
            b1 = min(range(2), key=lambda r: (res[r][1], r))
            s1, r1 = res[b1][0], res[b1][1]
            g2 = o.stage_grid(s1, s1, half)
            n2 = np.array([3, 3, 3, 3], np.int32)
            seeds2 = o.seed_grid(g2, n2)
            rss2, _ = o.scan(seeds2, cfg, sc.n_steps, ev.wire_ends, ev.wire_offsets, ev.drift)
            res2 = [o.lm_refine(seeds2[:, i], cfg, sc.n_steps, ev.wire_ends, ev.wire_offsets,
                                ev.drift, 3, 1e-3) for i in o.topk(rss2, 2)]
            cands = [(r1, 0, s1)] + [(res2[r][1], r + 1, res2[r][0]) for r in range(2)]
            wr, _, ws = min(cands, key=lambda c: (c[0], c[1]))
            assert np.max(np.abs(final[:, p] - ws) / np.maximum(np.abs(ws), 1.0)) < 1e-7, p
            assert abs(frss[p] - wr) <= 1e-7 * max(wr, 1.0), p
            p += 1
