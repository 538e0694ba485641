"""GPU path vs the CPU reference, through the C ABI.

The bar: the evaluation-order contract makes both sides compute the same binary64
operations in the same order, so seeds, tracks, RSS, chosen indices and hit masks
are compared for exact equality (stronger than the paper's < 1e-12 relative RSS
agreement, Sec. 4.1). Sizes span several seed tiles, several wire groups and
ragged tails; the full-size signal partition is checked on sampled seeds.
"""
import numpy as np
import pytest
import torch

import oracle
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


def gpu_seeds(grid, n):
    S = int(np.prod(n))
    seeds = torch.empty(6, S, dtype=torch.float64, device="cuda")
    comet.seed_grid(torch.as_tensor(grid, device="cuda"), n, seeds)
    return seeds


def gpu_rss(ev, seeds, cfg):
    S = seeds.shape[1]
    track = torch.empty(3, cfg.n_steps + 1, S, dtype=torch.float64, device="cuda")
    comet.extrapolate_seeds(seeds, cfg, track)
    dev = scan.DeviceEvent.from_event(ev)
    rss = torch.empty(S, dtype=torch.float64, device="cuda")
    comet.dca_rss(track, dev.wire_ends, dev.wire_offsets, dev.drift, cfg, rss,
                  comet.dca_workspace(S, cfg.n_steps + 1, dev.n_wires))
    return rss, track, dev


def _ocfg(ev, sc):
    return [ev.bz, ev.charge, sc.step_mm, sc.lambda_mm]


# ------------------------------------------------------------------ A1 seed grid
def test_seed_grid_bitwise(orc):
    rng = np.random.default_rng(11)
    cases = [(synth.grid_descriptor(synth.event_plain(0).ref_states[0], synth.C0), _n(8, 8, 8, 8)),
             (synth.grid_descriptor(synth.event_plain(0).ref_states[0], synth.C0), _n(7, 9, 8, 9))]
    for _ in range(6):
        ref = np.concatenate([rng.uniform(-600, 600, 3), rng.uniform(-120, 120, 3)])
        g = np.concatenate([ref, rng.uniform(-3, 3, 1), [abs(rng.uniform(60, 110))],
                            rng.uniform(-0.1, 0.1, 2), rng.uniform(0.1, 20, 2),
                            rng.uniform(0.001, 0.2, 2)])
        cases.append((g, _n(*rng.integers(1, 12, 4))))
    for g, n in cases:
        got = gpu_seeds(g, n).cpu().numpy()
        assert np.array_equal(got, orc.seed_grid(g, n)), (g, n)


def test_refine_grid_bitwise(orc):
    g0 = synth.grid_descriptor(synth.event_plain(0).ref_states[0], synth.C0)
    for n, b in [(_n(8, 8, 8, 8), 1476), (_n(5, 3, 1, 7), 3 * 21 + 2 * 7 + 5), (_n(2, 2, 2, 2), 0),
                 (_n(3, 3, 3, 3), -1)]:
        grid = torch.as_tensor(g0, device="cuda").clone()
        comet.refine_grid(grid, n, torch.tensor([b], dtype=torch.int64, device="cuda"))
        want = orc.refine_grid(g0, n, b)
        assert np.array_equal(grid.cpu().numpy(), want), (n, b)


# ------------------------------------------------------------------ A2 RK4
@pytest.mark.parametrize("bz,charge,h,K", [(1.0, -1.0, 2.0, 1000), (1.3, 1.0, 1.5, 257),
                                           (0.0, -1.0, 3.0, 1)])
def test_track_bitwise(orc, bz, charge, h, K):
    ev = synth.event_plain(0)
    n = _n(3, 5, 4, 3)   # 180 seeds: three tiles, ragged
    g = synth.grid_descriptor(ev.ref_states[0], synth.C0)
    seeds = gpu_seeds(g, n)
    cfg = comet.make_config(bz, charge, h, K, 1.0)
    track = torch.empty(3, K + 1, seeds.shape[1], dtype=torch.float64, device="cuda")
    comet.extrapolate_seeds(seeds, cfg, track)
    got = track.cpu().numpy()
    oseeds = orc.seed_grid(g, n)
    for s in range(oseeds.shape[1]):
        want = orc.track(oseeds[:, s], bz, charge, h, K)
        assert np.array_equal(got[:, :, s].T, want), s


# ------------------------------------------------------------------ A3/A4 RSS
@pytest.mark.parametrize("variant", range(40))
def test_rss_bitwise_plain_every_variant(orc, ev_plain, variant):
    """Ragged 7x9x8x9 grid (4536 seeds, 71 tiles with a partial last tile)."""
    assert variant < len(comet.dca_variants())
    comet.set_dca_variant(variant)
    try:
        sc = synth.C0
        g = synth.grid_descriptor(ev_plain.ref_states[0], sc)
        n = _n(7, 9, 8, 9)
        cfg = scan.config_for(ev_plain, sc)
        rss, _, _ = gpu_rss(ev_plain, gpu_seeds(g, n), cfg)
        want, _ = orc.scan(orc.seed_grid(g, n), _ocfg(ev_plain, sc), sc.n_steps,
                           ev_plain.wire_ends, ev_plain.wire_offsets, ev_plain.drift)
        got = rss.cpu().numpy()
        assert np.array_equal(got, want), np.max(np.abs(got - want) / want)
    finally:
        comet.set_dca_variant(-1)


def test_rss_signal_full_grid_sampled(orc, ev_signal):
    """Full-size signal partition: 16^4 grid, 1500 steps, 172 wires with 10 % noise."""
    sc = synth.C1
    cfg = scan.config_for(ev_signal, sc)
    for turn in range(ev_signal.n_turns):
        g = synth.grid_descriptor(ev_signal.ref_states[turn], sc)
        n = _n(*sc.n)
        rss, _, _ = gpu_rss(ev_signal, gpu_seeds(g, n), cfg)
        got = rss.cpu().numpy()
        rng = np.random.default_rng(turn)
        idx = np.unique(np.concatenate([rng.integers(0, sc.n_seeds, 120), [0, sc.n_seeds - 1],
                                        [int(np.argmin(got))]]))
        oseeds = np.stack([orc.seed(g, n, int(i)) for i in idx], axis=1)
        want, _ = orc.scan(oseeds, _ocfg(ev_signal, sc), sc.n_steps, ev_signal.wire_ends,
                           ev_signal.wire_offsets, ev_signal.drift)
        assert np.array_equal(got[idx], want), turn
        # every term is at most lambda^2, so no RSS exceeds the all-capped sum (the same
        # sequential sum, since rounded addition is monotonic)
        cap = 0.0
        for _ in range(ev_signal.n_wires):
            cap = cap + sc.lambda_mm * sc.lambda_mm
        assert np.all(np.isfinite(got)) and np.all(got <= cap)


def test_rss_deterministic_repeat(ev_signal):
    sc = synth.C1
    g = synth.grid_descriptor(ev_signal.ref_states[0], sc)
    cfg = scan.config_for(ev_signal, sc)
    seeds = gpu_seeds(g, _n(8, 8, 8, 8))
    a, _, _ = gpu_rss(ev_signal, seeds, cfg)
    b, _, _ = gpu_rss(ev_signal, seeds, cfg)
    assert torch.equal(a, b)


# ------------------------------------------------------------------ A5 select/classify
def test_select_classify_bitwise(orc, ev_plain):
    sc = synth.C0
    g = synth.grid_descriptor(ev_plain.ref_states[0], sc)
    n = _n(*sc.n)
    cfg = scan.config_for(ev_plain, sc)
    rss, track, dev = gpu_rss(ev_plain, gpu_seeds(g, n), cfg)
    best = torch.empty(1, dtype=torch.int64, device="cuda")
    mask = torch.empty(ev_plain.n_hits, dtype=torch.uint8, device="cuda")
    nb = torch.empty(1, dtype=torch.int32, device="cuda")
    dca = torch.empty(ev_plain.n_wires, dtype=torch.float64, device="cuda")
    comet.select_classify(rss, best, cfg, track, dev.wire_ends, dev.wire_offsets, dev.drift,
                          hit_mask=mask, n_borderline=nb, dca_best=dca)
    want_rss, _ = orc.scan(orc.seed_grid(g, n), _ocfg(ev_plain, sc), sc.n_steps,
                           ev_plain.wire_ends, ev_plain.wire_offsets, ev_plain.drift)
    b = orc.argmin(want_rss)
    assert int(best.item()) == b
    wmask, wdca, wnb = orc.classify(orc.seed(g, n, b), _ocfg(ev_plain, sc), sc.n_steps,
                                    ev_plain.wire_ends, ev_plain.wire_offsets, ev_plain.drift)
    assert np.array_equal(mask.cpu().numpy(), wmask)
    assert np.array_equal(dca.cpu().numpy(), wdca)
    assert int(nb.item()) == wnb


def test_select_ties_and_nan():
    cfg = comet.make_config(1.0, -1.0, 2.0, 10, 1.0)
    best = torch.empty(1, dtype=torch.int64, device="cuda")
    for vals, want in [([3.0, 1.0, 1.0, 2.0], 1), ([np.nan, 2.0, 2.0], 1), ([np.nan, np.nan], -1),
                       ([np.inf, np.inf], 0)]:
        comet.select_classify(torch.tensor(vals, dtype=torch.float64, device="cuda"), best, cfg)
        assert int(best.item()) == want, vals
    # ties far apart in a long array: the first index wins
    v = torch.full((100003,), 5.0, dtype=torch.float64, device="cuda")
    v[77777] = 1.0
    v[99999] = 1.0
    v[1025] = 1.0
    comet.select_classify(v, best, cfg)
    assert int(best.item()) == 1025


def test_classify_without_selection_leaves_zero_mask(ev_plain):
    """best = -1 (every RSS NaN): no hit is classified."""
    sc = synth.C0
    cfg = scan.config_for(ev_plain, sc)
    dev = scan.DeviceEvent.from_event(ev_plain)
    track = torch.zeros(3, sc.n_steps + 1, 4, dtype=torch.float64, device="cuda")
    rss = torch.full((4,), float("nan"), dtype=torch.float64, device="cuda")
    best = torch.empty(1, dtype=torch.int64, device="cuda")
    mask = torch.full((ev_plain.n_hits,), 7, dtype=torch.uint8, device="cuda")
    nb = torch.full((1,), 9, dtype=torch.int32, device="cuda")
    comet.select_classify(rss, best, cfg, track, dev.wire_ends, dev.wire_offsets, dev.drift,
                          hit_mask=mask, n_borderline=nb)
    assert int(best.item()) == -1
    assert int(mask.sum().item()) == 0 and int(nb.item()) == 0


# ------------------------------------------------------------------ A1-A6 whole partition
def _partition_compare(orc, ev, sc, turn):
    cfg = scan.config_for(ev, sc)
    runner = scan.PartitionScanner(sc.n, cfg, ev.n_wires, ev.n_hits)
    runner.run(scan.DeviceEvent.from_event(ev), scan.grid_tensor(ev.ref_states[turn], sc),
               sc.n_refine)
    torch.cuda.synchronize()
    got = runner.result()
    want = orc.scan_partition(synth.grid_descriptor(ev.ref_states[turn], sc), _n(*sc.n),
                              _ocfg(ev, sc), sc.n_steps, sc.n_refine, ev.wire_ends,
                              ev.wire_offsets, ev.drift)
    assert got["best"] == want["best"]
    assert np.array_equal(got["grid"], want["grid"])
    assert np.array_equal(got["best_seed"], want["best_seed"])
    assert got["best_rss"] == want["best_rss"]
    assert np.array_equal(got["mask"], want["mask"])
    assert got["n_borderline"] == want["n_borderline"]
    return got


def test_partition_path_plain(orc, ev_plain):
    got = _partition_compare(orc, ev_plain, synth.C0, 0)
    assert (got["mask"] & 1).sum() >= 30


@pytest.mark.parametrize("turn", [0, 1, 2])
def test_partition_path_signal(orc, ev_signal, turn):
    sc = synth.ScanConfig("signal-5^4", (5, 5, 5, 5), synth.C1.half, synth.C1.n_steps,
                          synth.C1.step_mm, synth.C1.lambda_mm, 2)
    _partition_compare(orc, ev_signal, sc, turn)


# ------------------------------------------------------------------ edge cases
def test_no_wires_gives_zero_rss():
    cfg = comet.make_config(1.0, -1.0, 2.0, 5, 1.0)
    track = torch.zeros(3, 6, 70, dtype=torch.float64, device="cuda")
    rss = torch.full((70,), 3.0, dtype=torch.float64, device="cuda")
    empty6 = torch.zeros(0, 6, dtype=torch.float64, device="cuda")
    comet.dca_rss(track, empty6, torch.zeros(1, dtype=torch.int32, device="cuda"),
                  torch.zeros(0, dtype=torch.float64, device="cuda"), cfg, rss,
                  torch.zeros(1, dtype=torch.float64, device="cuda"))
    assert torch.equal(rss, torch.zeros_like(rss))


@pytest.mark.parametrize("S_shape,K", [((1, 1, 1, 1), 1000), ((1, 1, 5, 13), 1000), ((2, 2, 2, 2), 1),
                                       ((1, 1, 1, 129), 37)])
def test_small_and_ragged_shapes(orc, ev_plain, S_shape, K):
    sc = synth.ScanConfig("t", S_shape, (5.0, 5.0, 0.05, 0.05), K, 2.0, 1.0)
    g = synth.grid_descriptor(ev_plain.ref_states[0], sc)
    n = _n(*S_shape)
    cfg = scan.config_for(ev_plain, sc)
    rss, _, _ = gpu_rss(ev_plain, gpu_seeds(g, n), cfg)
    want, _ = orc.scan(orc.seed_grid(g, n), _ocfg(ev_plain, sc), K, ev_plain.wire_ends,
                       ev_plain.wire_offsets, ev_plain.drift)
    assert np.array_equal(rss.cpu().numpy(), want)


def test_empty_wire_and_multi_hit_wires(orc, ev_signal):
    """A wire without hits (contributes lambda^2) and wires with several hits."""
    ev = ev_signal
    ends = np.concatenate([ev.wire_ends[:5], [[700.0, 0.0, -750.0, 700.0, 40.0, 750.0]],
                           ev.wire_ends[5:]])
    offs = np.concatenate([ev.wire_offsets[:6], ev.wire_offsets[5:]]).astype(np.int32)
    assert np.any(np.diff(ev.wire_offsets) > 1)
    ev2 = synth.Event(wire_ids=np.arange(len(ends), dtype=np.int32), wire_ends=ends,
                      wire_offsets=offs, drift=ev.drift, hit_turn=ev.hit_turn, true_dca=ev.true_dca,
                      ref_states=ev.ref_states, charge=ev.charge, bz=ev.bz)
    sc = synth.ScanConfig("t", (2, 3, 4, 5), synth.C1.half, 1500, 2.0, 0.8)
    g = synth.grid_descriptor(ev.ref_states[0], sc)
    n = _n(*sc.n)
    cfg = scan.config_for(ev2, sc)
    rss, _, _ = gpu_rss(ev2, gpu_seeds(g, n), cfg)
    want, _ = orc.scan(orc.seed_grid(g, n), _ocfg(ev2, sc), 1500, ends, offs, ev.drift)
    assert np.array_equal(rss.cpu().numpy(), want)


def test_far_seed_gives_n_lambda2(ev_plain):
    cfg = comet.make_config(1.0, -1.0, 2.0, 400, 0.8)
    seeds = torch.tensor([[0.0], [0.0], [6000.0], [10.0], [0.0], [100.0]], dtype=torch.float64,
                         device="cuda")
    rss, _, _ = gpu_rss(ev_plain, seeds, cfg)
    want = 0.0
    for _ in range(ev_plain.n_wires):
        want = want + 0.8 * 0.8
    assert float(rss[0].item()) == want


def test_workspace_too_small_raises(ev_plain):
    cfg = comet.make_config(1.0, -1.0, 2.0, 10, 1.0)
    dev = scan.DeviceEvent.from_event(ev_plain)
    track = torch.zeros(3, 11, 64, dtype=torch.float64, device="cuda")
    rss = torch.empty(64, dtype=torch.float64, device="cuda")
    with pytest.raises(comet.CometError) as ei:
        comet.dca_rss(track, dev.wire_ends, dev.wire_offsets, dev.drift, cfg, rss,
                      torch.empty(4, dtype=torch.float64, device="cuda"))
    assert ei.value.status == comet.EWORKSPACE


def test_autotune_picks_a_shape_and_keeps_results(orc, ev_plain):
    sc = synth.C0
    g = synth.grid_descriptor(ev_plain.ref_states[0], sc)
    n = _n(5, 5, 6, 7)
    cfg = scan.config_for(ev_plain, sc)
    seeds = gpu_seeds(g, n)
    rss, track, dev = gpu_rss(ev_plain, seeds, cfg)
    ws = comet.dca_workspace(seeds.shape[1], cfg.n_steps + 1, dev.n_wires)
    rss2 = torch.empty_like(rss)
    best, ms = comet.dca_autotune(track, dev.wire_ends, dev.wire_offsets, dev.drift, cfg, rss2, ws,
                                  reps=1)
    assert 0 <= best < len(comet.dca_variants()) and len(ms) == len(comet.dca_variants())
    assert all(m > 0 for m in ms) and ms[best] == min(ms)
    assert comet.dca_variant_for(seeds.shape[1], sc.n_steps + 1, dev.n_wires) == best
    assert torch.equal(rss, rss2)
    rss3 = torch.empty_like(rss)
    comet.dca_rss(track, dev.wire_ends, dev.wire_offsets, dev.drift, cfg, rss3, ws)
    assert torch.equal(rss, rss3)


def _odd_tracks(ev, kind, S, P, seed):
    """Polylines that no integrator would make: random walks with long jumps, and
    small orbits around a wire that repeat every 16 points (exact ties between chunks,
    where the first index must win)."""
    rng = np.random.default_rng(seed)
    mid = 0.5 * (ev.wire_ends[:, :3] + ev.wire_ends[:, 3:])
    tr = np.empty((3, P, S))
    for s in range(S):
        c = mid[rng.integers(0, mid.shape[0])]
        if kind == "walk":
            steps = rng.normal(0.0, 3.0, (P, 3))
            jump = rng.random(P) < 0.02
            steps[jump] += rng.normal(0.0, 300.0, (int(jump.sum()), 3))
            steps[0] = c + rng.normal(0.0, 20.0, 3)
            tr[:, :, s] = np.cumsum(steps, axis=0).T
        else:
            r = rng.uniform(2.0, 15.0)
            ph = 2.0 * np.pi * (np.arange(P) % 16) / 16.0 + rng.uniform(0, 2 * np.pi)
            tr[0, :, s] = c[0] + r * np.cos(ph)
            tr[1, :, s] = c[1] + r * np.sin(ph)
            tr[2, :, s] = c[2] + 40.0 * ((np.arange(P) // 16) % 3)   # three z levels, revisited
    return tr


@pytest.mark.parametrize("kind", ["walk", "orbit"])
def test_rss_arbitrary_tracks_every_variant(orc, ev_signal, kind):
    """The distance bound that lets the scan skip chunks must never change a result,
    whatever the track: every DCA shape vs the CPU reference on odd polylines (2 full
    tiles and a ragged one, 401 points)."""
    ev = ev_signal
    S, P = 145, 401
    tr = _odd_tracks(ev, kind, S, P, 17 if kind == "walk" else 23)
    lam = 1.0e4   # no cap: every wire's D enters the RSS
    cfg = comet.make_config(ev.bz, ev.charge, 2.0, P - 1, lam)
    want = np.array([orc.rss_track(np.ascontiguousarray(tr[:, :, s].T), ev.wire_ends,
                                   ev.wire_offsets, ev.drift, lam) for s in range(S)])
    dev = scan.DeviceEvent.from_event(ev)
    track = torch.as_tensor(np.ascontiguousarray(tr), device="cuda")
    rss = torch.empty(S, dtype=torch.float64, device="cuda")
    ws = comet.dca_workspace(S, P, dev.n_wires)
    try:
        for v in range(len(comet.dca_variants())):
            comet.set_dca_variant(v)
            rss.fill_(-1.0)
            comet.dca_rss(track, dev.wire_ends, dev.wire_offsets, dev.drift, cfg, rss, ws)
            torch.cuda.synchronize()
            assert np.array_equal(rss.cpu().numpy(), want), (kind, v)
    finally:
        comet.set_dca_variant(-1)


def test_profile_counts_the_distance_evaluations(ev_signal):
    """While profiling, the scans count their (seed, wire, point) evaluations: at least
    one point per chunk and wire, at most the full scan plus its sample pass; a seed far
    from every wire lets the bound skip almost everything."""
    ev = ev_signal
    S, P = 200, 801
    cfg = comet.make_config(ev.bz, ev.charge, 2.0, P - 1, 0.8)
    dev = scan.DeviceEvent.from_event(ev)
    ws = comet.dca_workspace(S, P, dev.n_wires)
    rss = torch.empty(S, dtype=torch.float64, device="cuda")
    for far in (False, True):
        seeds = np.tile(ev.ref_states[0][:, None], (1, S))
        if far:
            seeds[0] += 5.0e4        # 50 m off in x: every wire line far from every point
        track = torch.empty(3, P, S, dtype=torch.float64, device="cuda")
        comet.extrapolate_seeds(torch.as_tensor(seeds, device="cuda"), cfg, track)
        comet.profile_begin()
        comet.dca_rss(track, dev.wire_ends, dev.wire_offsets, dev.drift, cfg, rss, ws)
        prof = comet.profile_end()
        full = S * dev.n_wires * P
        assert S * dev.n_wires * (P // 32) <= prof["scan_points"] <= 2 * full, far
        if far:
            assert prof["scan_points"] < 0.3 * full


@pytest.mark.parametrize("K", [1, 16, 300, 1501])
def test_fused_track_and_scan_equals_separate_calls(ev_signal, K):
    """comet_track_dca_rss (the radii taken while recording) gives the track and RSS of
    comet_extrapolate_seeds + comet_dca_rss bit for bit, in the uniform field and in a
    field map, for step counts with and without a partial last window and a ragged seed
    count; no wires gives zero RSS and still the track."""
    sc = synth.ScanConfig("fused", (3, 5, 7, 9), (5.0, 5.0, 0.05, 0.05), K, 2.0, 0.8)
    seeds = gpu_seeds(synth.grid_descriptor(ev_signal.ref_states[1], sc), _n(*sc.n))
    cfg = scan.config_for(ev_signal, sc)
    S = seeds.shape[1]
    dev = scan.DeviceEvent.from_event(ev_signal)
    d = dict(dtype=torch.float64, device="cuda")
    fm = comet.FieldMap(*synth.solenoid_map())
    fm_rkn = comet.FieldMap(*synth.solenoid_map(), stepper=1)
    uniform = None
    for field in (None, fm, fm_rkn):
        t1 = torch.empty(3, K + 1, S, **d)
        r1 = torch.empty(S, **d)
        if field is None:
            comet.extrapolate_seeds(seeds, cfg, t1)
        else:
            comet.extrapolate_seeds_field(seeds, cfg, field, t1)
        comet.dca_rss(t1, dev.wire_ends, dev.wire_offsets, dev.drift, cfg, r1,
                      comet.dca_workspace(S, K + 1, dev.n_wires))
        t2 = torch.full((3, K + 1, S), np.nan, **d)
        r2 = torch.full((S,), np.nan, **d)
        comet.track_dca_rss(seeds, dev.wire_ends, dev.wire_offsets, dev.drift, cfg, t2, r2,
                            comet.dca_workspace(S, K + 1, dev.n_wires), field=field)
        torch.cuda.synchronize()
        assert torch.equal(t1, t2) and torch.equal(r1, r2), (K, field is None)
        if field is None:
            uniform = t1
    empty = torch.zeros(0, 6, **d)
    t3 = torch.empty(3, K + 1, S, **d)
    r3 = torch.full((S,), np.nan, **d)
    comet.track_dca_rss(seeds, empty, torch.zeros(1, dtype=torch.int32, device="cuda"),
                        torch.zeros(0, **d), cfg, t3, r3, torch.zeros(1, **d))
    torch.cuda.synchronize()
    assert torch.equal(t3, uniform) and bool((r3 == 0).all())
