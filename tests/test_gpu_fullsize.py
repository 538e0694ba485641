"""Full-size workloads in the launch configuration the bench times, checked on sampled
seeds against the CPU reference (which computes each seed on its own):

- the batched mix: 32768 seeds per partition (8 x 16 x 16 x 16), 1000 x 2 mm, two
  finer re-scans, graph-free eager run of the persistent kernel; every seed of the last
  grid of each partition;
- the stress mix: 131072 seeds per partition (8 x 16 x 32 x 32), 2000 x 1.5 mm;
- the fine grid of the differentiation workload: 32^4 = 1048576 seeds;
- Levenberg-Marquardt on stress-size tracks (2000 steps) vs the CPU LM.
"""
import numpy as np
import pytest
import torch

from paper_1911_09340_amd import comet, refine, scan, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    torch.cuda.set_device(0)
    comet.load()
    comet.set_batch_variant(0)


def _cfg(ev, sc):
    return [ev.bz, ev.charge, sc.step_mm, sc.lambda_mm]


def _check_partitions(orc, runner, events, sc, n_sample, seed):
    """RSS of the last grid bit for bit (every seed when n_sample is None, else a sample
    and the chosen one), the choice against the GPU row's first minimum (and against the
    CPU row's when it is whole), and the classification of the chosen seed."""
    rss = runner.rss.cpu().numpy()
    best = runner.best.cpu().numpy()
    grids = runner.grids.cpu().numpy()
    mask = runner.mask.cpu().numpy()
    n = np.array(sc.n, np.int32)
    rng = np.random.default_rng(seed)
    p = 0
    for ev in events:
        for _ in range(ev.n_turns):
            row = rss[p]
            assert best[p] == int(np.argmin(row)), p      # first index of the minimum
            if n_sample is None:
                want, _ = orc.scan(orc.seed_grid(grids[p], n), _cfg(ev, sc), sc.n_steps,
                                   ev.wire_ends, ev.wire_offsets, ev.drift)
                assert np.array_equal(row, want), (p, int(np.sum(row != want)))
                assert best[p] == orc.argmin(want), p
            else:
                idx = np.unique(np.concatenate([rng.integers(0, sc.n_seeds, n_sample),
                                                [0, sc.n_seeds - 1, best[p]]]))
                seeds = np.stack([orc.seed(grids[p], n, int(i)) for i in idx], axis=1)
                want, _ = orc.scan(seeds, _cfg(ev, sc), sc.n_steps, ev.wire_ends,
                                   ev.wire_offsets, ev.drift)
                assert np.array_equal(row[idx], want), p
            wmask, _, _ = orc.classify(orc.seed(grids[p], n, int(best[p])), _cfg(ev, sc),
                                       sc.n_steps, ev.wire_ends, ev.wire_offsets, ev.drift)
            assert np.array_equal(mask[p, :ev.n_hits], wmask), p
            p += 1


def test_batched_mix_full_size_sampled(orc):
    events = [synth.event_mix(i) for i in (3, 11)]
    sc = synth.C2
    runner = scan.BatchRunner(events, sc)
    runner.run()
    torch.cuda.synchronize()
    _check_partitions(orc, runner, events, sc, None, 1)   # every partition's whole row


def test_stress_full_size_sampled(orc):
    events = [synth.event_stress(5)]
    sc = synth.C4
    runner = scan.BatchRunner(events, sc)
    runner.run()
    torch.cuda.synchronize()
    _check_partitions(orc, runner, events, sc, 12, 2)


def test_fine_grid_full_size_sampled(orc):
    events = [synth.event_mix(7)]
    sc = synth.C3_FINE
    runner = scan.BatchRunner(events, sc)
    runner.run()
    torch.cuda.synchronize()
    _check_partitions(orc, runner, events, sc, 12, 3)


def test_lm_stress_size_matches_cpu(orc):
    """Two starts on a stress event (2000 x 1.5 mm): device LM = CPU LM to 1e-7."""
    ev = synth.event_stress(9)
    sc = synth.C4
    cfg = scan.config_for(ev, sc)
    starts = []
    for t in range(min(2, ev.n_turns)):
        s = ev.ref_states[t] * np.array([1.0, 1.0, 1.0, 1.003, 0.997, 1.002])
        starts.append(s)
    seeds = torch.as_tensor(np.ascontiguousarray(np.stack(starts, axis=1)), device="cuda")
    dev = scan.DeviceEvent.from_event(ev)
    rss = torch.empty(seeds.shape[1], dtype=torch.float64, device="cuda")
    acc = torch.empty(seeds.shape[1], dtype=torch.int32, device="cuda")
    comet.lm_refine(seeds, cfg, dev.wire_ends, dev.wire_offsets, dev.drift, 6, 1e-3, rss,
                    comet.lm_workspace(seeds.shape[1], sc.n_steps, "cuda"), n_accepted=acc)
    got = seeds.cpu().numpy()
    for r, s0 in enumerate(starts):
        ws, wrss, wacc = orc.lm_refine(s0, _cfg(ev, sc), sc.n_steps, ev.wire_ends,
                                       ev.wire_offsets, ev.drift, 6, 1e-3)
        assert int(acc[r]) == wacc, r
        assert np.max(np.abs(got[:, r] - ws) / np.maximum(np.abs(ws), 1.0)) < 1e-7, r
        assert abs(float(rss[r]) - wrss) <= 1e-7 * max(wrss, 1.0), r


def test_dca_far_offsets_every_direct_shape(orc):
    """A single-event scan whose track spans more than 2^29 doubles per coordinate
    (524 288 seeds x 1025 points), where the wave-independent shapes address the track
    with 64-bit pointers instead of 32-bit buffer offsets: sampled RSS bit for bit with
    the CPU reference for every such shape, the last seed included."""
    ev = synth.event_plain(0)
    sc = synth.ScanConfig("far", (8, 16, 64, 64), (5.0, 5.0, 0.05, 0.05), 1024, 2.0, 1.0)
    S, P = sc.n_seeds, sc.n_steps + 1
    assert P * S >= (1 << 29) - 64
    cfg = scan.config_for(ev, sc)
    dev = scan.DeviceEvent.from_event(ev)
    seeds = torch.empty(6, S, dtype=torch.float64, device="cuda")
    g = synth.grid_descriptor(ev.ref_states[0], sc)
    comet.seed_grid(torch.as_tensor(g, device="cuda"), np.array(sc.n, np.int32), seeds)
    track = torch.empty(3, P, S, dtype=torch.float64, device="cuda")
    comet.extrapolate_seeds(seeds, cfg, track)
    rss = torch.empty(S, dtype=torch.float64, device="cuda")
    ws = comet.dca_workspace(S, P, dev.n_wires)
    rng = np.random.default_rng(12)
    idx = np.unique(np.concatenate([rng.integers(0, S, 48), [0, S - 1]]))
    n = np.array(sc.n, np.int32)
    want, _ = orc.scan(np.stack([orc.seed(g, n, int(i)) for i in idx], axis=1), _cfg(ev, sc),
                       sc.n_steps, ev.wire_ends, ev.wire_offsets, ev.drift)
    shapes = [i for i, v in enumerate(comet.dca_variants()) if v["direct"]]
    assert shapes
    try:
        for v in shapes:
            comet.set_dca_variant(v)
            rss.fill_(np.nan)
            comet.dca_rss(track, dev.wire_ends, dev.wire_offsets, dev.drift, cfg, rss, ws)
            torch.cuda.synchronize()
            got = rss.cpu().numpy()
            assert np.array_equal(got[idx], want), v
    finally:
        comet.set_dca_variant(-1)


@pytest.mark.parametrize("stepper", [0, 1])
def test_field_signal_full_size_sampled(orc, stepper):
    """The signal partition at full size (16^4 seeds, 1500 x 2 mm) with tracks in the
    solenoid map, in the launch configuration the bench times (one fused track-and-scan
    call per scan): sampled RSS bit for bit with the CPU reference's map tracks, and the
    argmin of the whole row."""
    ev = synth.event_signal(0)
    sc = synth.C1
    cfg = scan.config_for(ev, sc)
    fmap = synth.solenoid_map()
    f = comet.FieldMap(*fmap, stepper=stepper)
    r = scan.PartitionScanner(sc.n, cfg, ev.n_wires, ev.n_hits, field=f)
    dev = scan.DeviceEvent.from_event(ev)
    r.run(dev, scan.grid_tensor(ev.ref_states[0], sc), 0)
    torch.cuda.synchronize()
    row = r.rss.cpu().numpy()
    best = int(r.best.item())
    assert best == int(np.argmin(row))
    g = synth.grid_descriptor(ev.ref_states[0], sc)
    n = np.array(sc.n, np.int32)
    rng = np.random.default_rng(21)
    idx = np.unique(np.concatenate([rng.integers(0, sc.n_seeds, 24), [0, sc.n_seeds - 1, best]]))
    for i in idx:
        pts = orc.track_field(orc.seed(g, n, int(i)), fmap, ev.charge, sc.step_mm, sc.n_steps,
                              stepper=stepper)
        want = orc.rss_track(pts, ev.wire_ends, ev.wire_offsets, ev.drift, sc.lambda_mm)
        assert row[i] == want, (int(i), stepper)


def test_stage_loop_full_size_matches_cpu(orc):
    """The stage loop at the grid size the bench runs it (per stage the 8 x 16 x 16 x 16
    grid, 1000 x 2 mm, two finer re-scans), two stages of a five-turn event against the
    CPU chain (about a minute of CPU work): both stages' chosen indices and seeds and the
    stage of every hit, bit for bit."""
    from paper_1911_09340_amd import stages
    from test_gpu_stages import _oracle_stages
    ev = synth.event_mix(3)
    sc = synth.C2
    run = stages.StageRunner([ev], sc, max_stages=2, min_wires=30, max_back_steps=4000)
    run.run()
    torch.cuda.synchronize()
    soh = run.stage_of_hit.cpu().numpy()
    best, seeds = run.best.cpu().numpy(), run.seeds.cpu().numpy()
    want, per_stage = _oracle_stages(orc, ev, sc, 2, 30, 4000)
    assert len(per_stage) == 2
    assert np.array_equal(soh, want)
    for s, (b, seed, _) in enumerate(per_stage):
        assert best[s, 0] == b, s
        assert np.array_equal(seeds[s, 0], seed), s
