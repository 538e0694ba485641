"""The stage loop (Sec. 3.1) on the GPU vs the CPU reference: backward extrapolation to
the previous turn's entry, the next stage's grids, the exclusion of classified hits, and
the whole loop over several events (every stage's chosen seed and the stage of every
hit), bit for bit."""
import numpy as np
import pytest
import torch

from paper_1911_09340_amd import comet, scan, stages, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    torch.cuda.set_device(0)
    comet.load()
    comet.set_batch_variant(0)


def test_backward_seeds_match_cpu(orc):
    rng = np.random.default_rng(2)
    seeds = []
    for i in range(6):
        ev = synth.event_mix(i)
        for t in range(ev.n_turns):
            s = ev.ref_states[t].copy()
            s[3:] *= 1.0 + rng.normal(0.0, 0.003, 3)
            seeds.append(s)
    seeds.append(np.full(6, np.nan))                         # no seed: NaN out
    seeds = np.stack(seeds)
    cfg = comet.make_config(1.0, -1.0, 2.0, 1000, 0.8)
    d = dict(device="cuda")
    for max_steps in (4000, 300):                            # 300: too few for a turn
        out = torch.empty(len(seeds), 6, dtype=torch.float64, **d)
        steps = torch.empty(len(seeds), dtype=torch.int32, **d)
        comet.backward_seeds(torch.as_tensor(seeds, **d), cfg, synth.SEED_RADIUS, max_steps, out,
                             steps)
        torch.cuda.synchronize()
        got, gs = out.cpu().numpy(), steps.cpu().numpy()
        for i, s in enumerate(seeds):
            want, k = orc.backward_seed(s, 1.0, -1.0, 2.0, synth.SEED_RADIUS, max_steps)
            assert gs[i] == k, (i, max_steps)
            assert np.array_equal(got[i], want, equal_nan=True), (i, max_steps)
        if max_steps == 300:
            assert (gs == -1).all()
        else:
            assert (gs[:-1] > 0).all() and gs[-1] == -1


def test_stage_grids_match_cpu(orc):
    rng = np.random.default_rng(3)
    tr, ex = rng.normal(0, 100, (9, 6)), rng.normal(0, 100, (9, 6))
    half = (5.0, 5.0, 0.05, 0.05)
    g = torch.empty(9, 14, dtype=torch.float64, device="cuda")
    comet.stage_grids(torch.as_tensor(tr, device="cuda"), torch.as_tensor(ex, device="cuda"), half, g)
    torch.cuda.synchronize()
    got = g.cpu().numpy()
    for i in range(9):
        assert np.array_equal(got[i], orc.stage_grid(tr[i], ex[i], half)), i


@pytest.mark.parametrize("n_z,z_half", [(1, 4.0), (3, 6.0), (5, 10.0), (2, 0.0)])
def test_stage_grids_z_match_cpu(orc, n_z, z_half):
    rng = np.random.default_rng(5)
    tr, ex = rng.normal(0, 100, (7, 6)), rng.normal(0, 100, (7, 6))
    half = (5.0, 5.0, 0.05, 0.05)
    g = torch.empty(7, n_z, 14, dtype=torch.float64, device="cuda")
    comet.stage_grids_z(torch.as_tensor(tr, device="cuda"), torch.as_tensor(ex, device="cuda"),
                        half, n_z, z_half, g)
    torch.cuda.synchronize()
    got = g.cpu().numpy()
    for i in range(7):
        assert np.array_equal(got[i], orc.stage_grids_z(tr[i], ex[i], half, n_z, z_half)), i


def test_exclude_hits_match_cpu(orc):
    rng = np.random.default_rng(4)
    evs = []
    for i in range(5):
        ev = synth.event_mix(i)
        evs.extend(synth.half_events(ev, 0))
    src = stages.StagePacked.from_events(evs)
    n_h = int(src.drift.shape[0])
    ex = (rng.random(n_h) < 0.4).astype(np.uint8)
    h0 = 0
    for k, ev in enumerate(evs):                 # one event loses every hit, one none
        if k == 2:
            ex[h0:h0 + ev.n_hits] = 1
        if k == 3:
            ex[h0:h0 + ev.n_hits] = 0
        h0 += ev.n_hits
    dst = src.empty_like()
    comet.exclude_hits(src, torch.as_tensor(ex, device="cuda"), dst,
                       comet.exclude_workspace(len(evs)))
    torch.cuda.synchronize()
    ew = dst.event_wires.cpu().numpy()
    wo = dst.wire_offsets.cpu().numpy()
    dr, en, hi = dst.drift.cpu().numpy(), dst.wire_ends.cpu().numpy(), dst.hit_ids.cpu().numpy()
    h0 = 0
    for k, ev in enumerate(evs):
        o2, d2, e2, wm, hm = orc.exclude_hits(ev.wire_offsets, ev.drift, ev.wire_ends,
                                               ex[h0:h0 + ev.n_hits])
        a, b = ew[k], ew[k + 1]
        assert b - a == len(o2) - 1, k
        base = wo[a]
        assert np.array_equal(wo[a:b + 1] - base, o2), k
        assert np.array_equal(dr[base:base + len(d2)], d2), k
        assert np.array_equal(en[a:b], e2.reshape(-1, 6)), k
        assert np.array_equal(hi[base:base + len(hm)], hm + h0), k
        h0 += ev.n_hits
    assert ew[3] == ew[2]                        # the emptied event keeps no wire


def test_self_refine_matches_cpu(orc):
    """Fitted seeds near the truth, input masks from the CPU classification at another
    seed and random bits; a NaN seed keeps its classified bits, a row of an event out of
    range is left alone; in place and out of place."""
    rng = np.random.default_rng(5)
    evs = [synth.event_mix(i) for i in (1, 4, 6)]
    packed = stages.StagePacked.from_events(evs)
    cfg = comet.make_config(evs[0].bz, evs[0].charge, 2.0, 900, 0.8)
    ocfg = [evs[0].bz, evs[0].charge, 2.0, 0.8]
    rows, seeds, masks = [], [], []
    stride = max(ev.n_hits for ev in evs)
    for e, ev in enumerate(evs):
        for t in range(ev.n_turns):
            fit = ev.ref_states[t].copy()
            fit[3:] *= 1.0 + rng.normal(0.0, 0.002, 3)
            scan_seed = ev.ref_states[t].copy()
            scan_seed[3:] *= 1.0 + rng.normal(0.0, 0.004, 3)
            m, _, _ = orc.classify(scan_seed, ocfg, 900, ev.wire_ends, ev.wire_offsets, ev.drift)
            for mask in (m, rng.integers(0, 4, ev.n_hits).astype(np.uint8)):
                rows.append(e)
                seeds.append(fit)
                masks.append(np.pad(mask, (0, stride - ev.n_hits)))
    seeds.append(np.full(6, np.nan))
    rows.append(2)
    masks.append(np.pad(rng.integers(0, 4, evs[2].n_hits).astype(np.uint8),
                        (0, stride - evs[2].n_hits)))
    seeds.append(evs[0].ref_states[0])
    rows.append(-1)                                          # skipped row
    masks.append(np.full(stride, 7, np.uint8))
    m_in = np.stack(masks)
    d = dict(device="cuda")
    t_seeds = torch.as_tensor(np.stack(seeds), **d)
    t_rows = torch.as_tensor(np.array(rows, np.int32), **d)
    out = torch.full(m_in.shape, 9, dtype=torch.uint8, **d)
    t_in = torch.as_tensor(m_in, **d)
    comet.self_refine(t_seeds, t_rows, cfg, packed, 0.3, t_in, out)
    comet.self_refine(t_seeds, t_rows, cfg, packed, 0.3, t_in, t_in)     # in place
    torch.cuda.synchronize()
    got, got_in = out.cpu().numpy(), t_in.cpu().numpy()
    n_changed = 0
    for r, e in enumerate(rows):
        if e < 0:
            assert (got[r] == 9).all() and (got_in[r] == 7).all()
            continue
        ev = evs[e]
        want, _ = orc.self_refine(seeds[r], ocfg, 900, ev.wire_ends, ev.wire_offsets, ev.drift,
                                  m_in[r, :ev.n_hits], 0.3)
        assert np.array_equal(got[r, :ev.n_hits], want), r
        assert np.array_equal(got_in[r, :ev.n_hits], want), r
        assert (got[r, ev.n_hits:] == 9).all(), r
        n_changed += int((want != (m_in[r, :ev.n_hits] & 1)).sum())
    assert n_changed > 0


def _cfg(ev, sc):
    return [ev.bz, ev.charge, sc.step_mm, sc.lambda_mm]


def _oracle_scan_z(orc, ev, sc, ext, t, n_z, z_half):
    """The z-axis scan of one stage: every sub-grid scanned, the lowest RSS over all of
    them (lowest sub-grid, then seed index, on ties), that grid re-centred on it, then
    the partition path with the remaining re-scans."""
    n = np.array(sc.n, np.int32)
    gz = orc.stage_grids_z(ev.ref_states[t], ext, sc.half, n_z, z_half)
    rows = [orc.scan(orc.seed_grid(g, n), _cfg(ev, sc), sc.n_steps, ev.wire_ends, ev.wire_offsets,
                     ev.drift)[0] for g in gz]
    j = orc.argmin(np.concatenate(rows))
    u, i = divmod(j, sc.n_seeds)
    g = orc.refine_grid(gz[u], n, i)
    return g


def _oracle_stages(orc, ev, sc, max_stages, min_wires, max_back, fit_iters=0, eta=0.3,
                   mu0=1e-3, n_z=1, z_half=0.0):
    soh = np.full(ev.n_hits, -1, np.int32)
    off, drift, ends = ev.wire_offsets, ev.drift, ev.wire_ends
    ids = np.arange(ev.n_hits)
    ext = ev.ref_states[ev.n_turns - 1]
    active = ev.n_wires >= min_wires
    out = []
    for s in range(max_stages):
        if not active:
            break
        t = ev.n_turns - 1 - s
        if n_z > 1:
            evs = type("Ev", (), dict(ref_states=ev.ref_states, wire_ends=ends,
                                      wire_offsets=off, drift=drift, bz=ev.bz,
                                      charge=ev.charge))
            g = _oracle_scan_z(orc, evs, sc, ext, t, n_z, z_half)
            r = orc.scan_partition(g, np.array(sc.n, np.int32), _cfg(ev, sc), sc.n_steps,
                                   sc.n_refine - 1, ends, off, drift)
        else:
            g = orc.stage_grid(ev.ref_states[t], ext, sc.half)
            r = orc.scan_partition(g, np.array(sc.n, np.int32), _cfg(ev, sc), sc.n_steps,
                                   sc.n_refine, ends, off, drift)
        mask, fit = r["mask"] & 1, r["best_seed"]
        if fit_iters > 0:
            fit, _, _ = orc.lm_refine(fit, _cfg(ev, sc), sc.n_steps, ends, off, drift,
                                      fit_iters, mu0)
            mask, _ = orc.self_refine(fit, _cfg(ev, sc), sc.n_steps, ends, off, drift, mask, eta)
        cls = mask.astype(bool)
        soh[ids[cls]] = s
        off, drift, ends, _, hm = orc.exclude_hits(off, drift, ends, cls.astype(np.uint8))
        ids = ids[hm]
        ext, _ = orc.backward_seed(fit, ev.bz, ev.charge, sc.step_mm, synth.SEED_RADIUS,
                                   max_back)
        out.append((r["best"], r["best_seed"], fit))
        active = (r["best"] >= 0 and s + 1 < min(ev.n_turns, max_stages)
                  and len(off) - 1 >= min_wires)
    return soh, out


def test_stage_loop_matches_cpu(orc):
    events = [synth.event_mix(i) for i in (2, 3, 5, 8)]
    sc = synth.ScanConfig("stages", (3, 4, 5, 6), (5.0, 5.0, 0.05, 0.05), 800, 2.0, 0.8, 1)
    run = stages.StageRunner(events, sc, max_stages=5, min_wires=30, max_back_steps=3000)
    run.run()
    torch.cuda.synchronize()
    first = run.stage_of_hit.clone()
    run.run()                                   # a second run starts from the same events
    torch.cuda.synchronize()
    assert torch.equal(run.stage_of_hit, first)
    soh = run.stage_of_hit.cpu().numpy()
    best = run.best.cpu().numpy()
    seeds = run.seeds.cpu().numpy()
    h0 = 0
    n_stages = 0
    for e, ev in enumerate(events):
        want, per_stage = _oracle_stages(orc, ev, sc, 5, 30, 3000)
        assert np.array_equal(soh[h0:h0 + ev.n_hits], want), e
        for s, (b, seed, _) in enumerate(per_stage):
            assert best[s, e] == b, (e, s)
            assert np.array_equal(seeds[s, e], seed), (e, s)
        # stages after the event stopped are not scanned at all
        for s in range(len(per_stage), 5):
            assert best[s, e] == -1 and np.all(np.isnan(seeds[s, e])), (e, s)
        n_stages += len(per_stage)
        h0 += ev.n_hits
    assert n_stages > len(events)                # the loop went past the first stage


def test_stage_loop_with_fit_matches_cpu(orc):
    """The loop with the self-refining: every stage's chosen seed is refined by
    Levenberg-Marquardt (the fitted track), the hits are re-tested at it with lambda and
    eta, and the next stage starts from the fitted seed. Fitted seeds agree to the LM bar
    (1e-7 relative); the chosen grid indices and the stage of every hit exactly."""
    events = [synth.event_mix(i) for i in (2, 3, 5, 8)]
    sc = synth.ScanConfig("stages", (3, 4, 5, 6), (5.0, 5.0, 0.05, 0.05), 800, 2.0, 0.8, 1)
    run = stages.StageRunner(events, sc, max_stages=5, min_wires=30, max_back_steps=3000,
                             fit_iters=4, eta=0.3)
    run.run()
    torch.cuda.synchronize()
    soh = run.stage_of_hit.cpu().numpy()
    best = run.best.cpu().numpy()
    seeds, fitted = run.seeds.cpu().numpy(), run.fitted.cpu().numpy()
    h0, n_stages, n_moved = 0, 0, 0
    for e, ev in enumerate(events):
        want, per_stage = _oracle_stages(orc, ev, sc, 5, 30, 3000, fit_iters=4, eta=0.3)
        assert np.array_equal(soh[h0:h0 + ev.n_hits], want), e
        for s, (b, seed, fit) in enumerate(per_stage):
            assert best[s, e] == b, (e, s)
            np.testing.assert_allclose(seeds[s, e], seed, rtol=1e-7, atol=1e-9)
            np.testing.assert_allclose(fitted[s, e], fit, rtol=1e-7, atol=1e-9)
            n_moved += int(not np.array_equal(fit, seed))
        n_stages += len(per_stage)
        h0 += ev.n_hits
    assert n_stages > len(events) and n_moved > 0


def test_stage_loop_with_z_axis_matches_cpu(orc):
    """The seed's z as a fifth axis in every stage (three sub-grids over +-6 mm): the
    stage of every hit, every stage's chosen index and seed, bit for bit with the CPU
    chain (sub-grid scans, lowest RSS over them, re-centred grid, remaining re-scans)."""
    events = [synth.event_mix(i) for i in (2, 3, 5, 8)]
    sc = synth.ScanConfig("stages", (3, 4, 5, 6), (5.0, 5.0, 0.05, 0.05), 800, 2.0, 0.8, 1)
    run = stages.StageRunner(events, sc, max_stages=5, min_wires=30, max_back_steps=3000,
                             n_z=3, z_half=6.0)
    run.run()
    torch.cuda.synchronize()
    soh = run.stage_of_hit.cpu().numpy()
    best = run.best.cpu().numpy()
    seeds = run.seeds.cpu().numpy()
    h0, n_stages = 0, 0
    for e, ev in enumerate(events):
        want, per_stage = _oracle_stages(orc, ev, sc, 5, 30, 3000, n_z=3, z_half=6.0)
        assert np.array_equal(soh[h0:h0 + ev.n_hits], want), e
        for s, (b, seed, _) in enumerate(per_stage):
            assert best[s, e] == b, (e, s)
            assert np.array_equal(seeds[s, e], seed), (e, s)
        n_stages += len(per_stage)
        h0 += ev.n_hits
    assert n_stages > len(events)
