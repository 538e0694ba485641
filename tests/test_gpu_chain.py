"""The paper's per-stage chain (Sec. 3.1) on the GPU vs the CPU reference: the exit
half's seed, the split of a stage's hits into halves, the halves' wire layers, the union
of the best complete set, and the whole chain over several events and stages (every
stage's chosen pair and entrance seed, the stage of every hit), bit for bit; fitted
seeds within the LM bar."""
from dataclasses import replace

import numpy as np
import pytest
import torch

from paper_1911_09340_amd import chain, comet, stages, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    torch.cuda.set_device(0)
    comet.load()
    comet.set_batch_variant(0)


def test_exit_seeds_match_cpu(orc):
    """Entry states of many turns (perturbed), read directly (row stride 6) and as the
    reference state of grid descriptors (stride 14); a NaN row; too few steps."""
    rng = np.random.default_rng(7)
    states = []
    for i in range(8):
        ev = synth.event_mix(i)
        for t in range(ev.n_turns):
            s = ev.ref_states[t].copy()
            s[3:] *= 1.0 + rng.normal(0.0, 0.003, 3)
            s[2] += rng.normal(0.0, 5.0)
            states.append(s)
    states.append(np.full(6, np.nan))
    states = np.stack(states)
    n = len(states)
    grids = np.stack([orc.stage_grid(s, s, (5.0, 5.0, 0.05, 0.05)) for s in states])
    cfg = comet.make_config(1.0, -1.0, 2.0, 1000, 0.8)
    d = dict(device="cuda")
    for max_steps in (4000, 50):
        for src, stride in ((states, 6), (grids, 14)):
            out = torch.empty(n, 6, dtype=torch.float64, **d)
            steps = torch.empty(n, dtype=torch.int32, **d)
            comet.exit_seeds(torch.as_tensor(np.ascontiguousarray(src), **d), stride, cfg,
                             synth.SEED_RADIUS, max_steps, out, steps)
            torch.cuda.synchronize()
            got, gs = out.cpu().numpy(), steps.cpu().numpy()
            for i in range(n):
                want, k = orc.exit_seed(states[i], 1.0, -1.0, 2.0, synth.SEED_RADIUS, max_steps)
                assert gs[i] == k, (i, max_steps, stride)
                assert np.array_equal(got[i], want, equal_nan=True), (i, max_steps, stride)
            if max_steps == 50:
                assert (gs == -1).all()
            else:
                assert (gs[:-1] > 0).all() and gs[-1] == -1


def _excluded_packed(events, frac, seed):
    """Packed events after a random exclusion, so that hit ids are not the positions."""
    rng = np.random.default_rng(seed)
    src = stages.StagePacked.from_events(events)
    n_h = int(src.drift.shape[0])
    ex = (rng.random(n_h) < frac).astype(np.uint8)
    dst = src.empty_like()
    comet.exclude_hits(src, torch.as_tensor(ex, device="cuda"), dst,
                       comet.exclude_workspace(len(events)))
    return dst, n_h


def test_half_split_and_wire_layers_match_host():
    events = [synth.event_mix(i) for i in (1, 3, 4, 9)]
    packed, n_ids = _excluded_packed(events, 0.3, 1)
    rng = np.random.default_rng(2)
    side = (rng.random(n_ids) < 0.5).astype(np.uint8)
    layer = rng.integers(0, synth.N_LAYERS, n_ids).astype(np.int32)
    n_h = int(packed.drift.shape[0])
    ea = torch.full((n_h,), 7, dtype=torch.uint8, device="cuda")
    eb = torch.full((n_h,), 7, dtype=torch.uint8, device="cuda")
    comet.half_split(packed, torch.as_tensor(side, device="cuda"), ea, eb)
    torch.cuda.synchronize()
    ew = packed.event_wires.cpu().numpy()
    wo = packed.wire_offsets.cpu().numpy()
    used = wo[ew[-1]]
    ids = packed.hit_ids.cpu().numpy()[:used]
    assert np.array_equal(ea.cpu().numpy()[:used], (side[ids] == 0).astype(np.uint8))
    assert np.array_equal(eb.cpu().numpy()[:used], (side[ids] != 0).astype(np.uint8))
    assert (ea.cpu().numpy()[used:] == 7).all()            # past the used hits: untouched
    for k, ex in enumerate((ea, eb)):
        half = packed.empty_like()
        comet.exclude_hits(packed, ex, half, comet.exclude_workspace(len(events)))
        wl = torch.full((int(half.wire_ends.shape[0]),), -9, dtype=torch.int32, device="cuda")
        comet.wire_layers(half, torch.as_tensor(layer, device="cuda"), wl)
        torch.cuda.synchronize()
        hew = half.event_wires.cpu().numpy()
        hwo = half.wire_offsets.cpu().numpy()
        hids = half.hit_ids.cpu().numpy()
        nw = hew[-1]
        assert np.array_equal(wl.cpu().numpy()[:nw], layer[hids[hwo[:nw]]]), k
        assert (wl.cpu().numpy()[nw:] == -9).all()
        # every kept hit is on its side
        sh = side[hids[:hwo[nw]]]
        assert (sh == (1 if k == 0 else 0)).all()


def _host_union(pair, nc, F, packed, side, ma, mb, seeds_a, active, stride):
    ew = packed.event_wires.cpu().numpy()
    wo = packed.wire_offsets.cpu().numpy()
    ids = packed.hit_ids.cpu().numpy()
    E = len(active)
    masks = np.zeros((E, stride), np.uint8)
    seed = np.full((E, 6), np.nan)
    best = np.full(E, -1, np.int64)
    for e in range(E):
        if not active[e]:
            continue
        i, j = divmod(int(pair[e, 0]), F) if nc[e] > 0 else (0, 0)
        seed[e] = seeds_a[e * F + i]
        best[e] = -1 if np.isnan(seed[e, 0]) else i * F + j
        h0, h1 = wo[ew[e]], wo[ew[e + 1]]
        ca = cb = 0
        for h in range(h0, h1):
            if side[ids[h]]:
                masks[e, h - h0] = ma[e * F + i, ca] & 1
                ca += 1
            else:
                masks[e, h - h0] = mb[e * F + j, cb] & 1
                cb += 1
    return masks, seed, best


def test_union_halves_matches_host():
    """Random half masks (other bits set too), ranked pairs, events without a complete
    set (the lowest-RSS seed of each side), an inactive event, a NaN entrance seed."""
    events = [synth.event_mix(i) for i in (2, 5, 6, 7, 11)]
    packed, n_ids = _excluded_packed(events, 0.25, 3)
    E, F = len(events), 4
    rng = np.random.default_rng(4)
    side = (rng.random(n_ids) < 0.5).astype(np.uint8)
    stride = max(ev.n_hits for ev in events)
    ma = rng.integers(0, 4, (E * F, stride)).astype(np.uint8)
    mb = rng.integers(0, 4, (E * F, stride)).astype(np.uint8)
    seeds_a = rng.normal(0.0, 100.0, (E * F, 6))
    seeds_a[3 * F + 2] = np.nan
    pair = np.stack([rng.permutation(F * F) for _ in range(E)]).astype(np.int32)
    pair[3, 0] = 2 * F + 1                      # chooses the NaN seed
    nc = np.array([3, 0, 5, 1, 2], np.int32)    # event 1: no complete set
    active = np.array([1, 1, 1, 1, 0], np.int32)
    d = dict(device="cuda")
    mo = torch.full((E, stride), 9, dtype=torch.uint8, **d)
    so = torch.empty(E, 6, dtype=torch.float64, **d)
    bo = torch.empty(E, dtype=torch.int64, **d)
    comet.union_halves(torch.as_tensor(pair, **d), torch.as_tensor(nc, **d), F, packed,
                       torch.as_tensor(side, **d), torch.as_tensor(ma, **d),
                       torch.as_tensor(mb, **d), torch.as_tensor(seeds_a, **d),
                       torch.as_tensor(active, **d), mo, so, bo)
    torch.cuda.synchronize()
    wm, ws, wb = _host_union(pair, nc, F, packed, side, ma, mb, seeds_a, active, stride)
    ew = packed.event_wires.cpu().numpy()
    wo = packed.wire_offsets.cpu().numpy()
    got = mo.cpu().numpy()
    for e in range(E):
        n = wo[ew[e + 1]] - wo[ew[e]]
        if active[e]:
            assert np.array_equal(got[e, :n], wm[e, :n]), e
        else:
            assert (got[e] == 9).all(), e       # an inactive event's mask is left alone
        assert (got[e, n:] == 9).all(), e
    assert np.array_equal(so.cpu().numpy(), ws, equal_nan=True)
    assert np.array_equal(bo.cpu().numpy(), wb)
    assert wb[3] == -1 and wb[1] == 0 and wb[4] == -1


# ------------------------------------------------------------------ the whole chain
def _cfg(ev, sc, charge=None):
    return [ev.bz, ev.charge if charge is None else charge, sc.step_mm, sc.lambda_mm]


def _oracle_multiref(orc, csr, charge, bz, grid0, sc, n_fine, R, n_iter, F):
    """The several-reference chain of one half on the CPU: final indices, RSS, seeds and
    half sets (None for a missing seed)."""
    off, drift, ends = csr
    cfg = [bz, charge, sc.step_mm, sc.lambda_mm]

    def scan_grids(grids, n):
        out = []
        for g in grids:
            s = orc.seed_grid(g, np.asarray(n, np.int32))
            r, _ = orc.scan(s, cfg, sc.n_steps, ends, off, drift)
            out.append(r)
        return np.stack(out)

    grids, n = grid0[None, :], sc.n
    rss = scan_grids(grids, n)
    for _ in range(n_iter):
        _, _, ng, _ = orc.sparse_select(grids, rss, n, R)
        grids, n = ng, n_fine
        rss = scan_grids(grids, n)
    idx, frss, _, _ = orc.sparse_select(grids, rss, n, F)
    S = int(np.prod(n))
    seeds, masks = [], []
    for r in range(F):
        if idx[r] < 0:
            seeds.append(None)
            masks.append(None)
            continue
        s = orc.seed(grids[idx[r] // S], np.asarray(n, np.int32), int(idx[r] % S))
        m, _, _ = orc.classify(s, cfg, sc.n_steps, ends, off, drift)
        seeds.append(s)
        masks.append(m)
    return frss, seeds, masks


def _oracle_chain_stages(orc, ev, sc, max_stages, min_wires, max_back, n_fine, R, n_iter, F,
                         fit_iters, eta, mu0=1e-3):
    soh = np.full(ev.n_hits, -1, np.int32)
    off, drift, ends = ev.wire_offsets, ev.drift, ev.wire_ends
    ids = np.arange(ev.n_hits)
    counts = np.diff(ev.wire_offsets)
    hit_layer = np.repeat(synth.wire_layers(ev.wire_ids), counts)
    sc_half = replace(sc, n_steps=sc.n_steps // 2)
    ext = ev.ref_states[ev.n_turns - 1]
    active = ev.n_wires >= min_wires
    out = []
    for s in range(max_stages):
        if not active:
            break
        t = ev.n_turns - 1 - s
        side_hit = np.repeat(synth.entrance_sides(ev, t), counts)[ids]
        g_ent = orc.stage_grid(ev.ref_states[t], ext, sc.half)
        exit6, _ = orc.exit_seed(g_ent[:6], ev.bz, ev.charge, sc.step_mm, synth.SEED_RADIUS,
                                 max_back)
        ex = ev.exit_states[t]
        g_ext = orc.stage_grid(np.concatenate([ex[:3], -ex[3:]]), exit6, sc.half)
        res = []
        for k, (g, charge) in enumerate(((g_ent, ev.charge), (g_ext, -ev.charge))):
            keep = side_hit != 0 if k == 0 else side_hit == 0
            o2, d2, e2, _, hm = orc.exclude_hits(off, drift, ends, (~keep).astype(np.uint8))
            frss, seeds, masks = _oracle_multiref(orc, (o2, d2, e2.reshape(-1, 6)), charge,
                                                  ev.bz, g, sc_half, n_fine, R, n_iter, F)
            wl = hit_layer[ids[hm[o2[:-1]]]] if len(o2) > 1 else np.zeros(0, np.int32)
            veto = np.array([orc.layer_veto(m, o2, wl, synth.N_LAYERS) if m is not None else 1
                             for m in masks], np.int32)
            res.append((frss, seeds, masks, veto))
        (ra, sa, ma, va), (rb, _, mb, vb) = res
        pair, _, nc = orc.merge_halves(ra, va, rb, vb)
        i, j = divmod(int(pair[0]), F) if nc > 0 else (0, 0)
        seed = sa[i] if sa[i] is not None else np.full(6, np.nan)
        best = -1 if np.isnan(seed[0]) else i * F + j
        union = np.zeros(len(side_hit), np.uint8)
        ca = cb = 0
        for h in range(len(side_hit)):
            if side_hit[h]:
                union[h] = ma[i][ca] & 1 if ma[i] is not None else 0
                ca += 1
            else:
                union[h] = mb[j][cb] & 1 if mb[j] is not None else 0
                cb += 1
        fit = seed
        if fit_iters > 0:
            fit, _, _ = orc.lm_refine(seed, _cfg(ev, sc), sc.n_steps, ends, off, drift,
                                      fit_iters, mu0)
        mask, _ = orc.self_refine(fit, _cfg(ev, sc), sc.n_steps, ends, off, drift, union, eta)
        cls = mask.astype(bool)
        soh[ids[cls]] = s
        off, drift, ends, _, hm = orc.exclude_hits(off, drift, ends, cls.astype(np.uint8))
        ends = ends.reshape(-1, 6)
        ids = ids[hm]
        ext, _ = orc.backward_seed(fit, ev.bz, ev.charge, sc.step_mm, synth.SEED_RADIUS,
                                   max_back)
        out.append((best, seed, fit, nc))
        active = (best >= 0 and s + 1 < min(ev.n_turns, max_stages)
                  and len(off) - 1 >= min_wires)
    return soh, out


@pytest.mark.parametrize("fit_iters", [0, 4])
def test_stage_chain_matches_cpu(orc, fit_iters):
    events = [synth.event_mix(i) for i in (2, 3, 5, 8)]
    sc = synth.ScanConfig("chain", (3, 4, 5, 6), (5.0, 5.0, 0.05, 0.05), 800, 2.0, 0.8, 0)
    n_fine, R, n_iter, F = (2, 3, 3, 4), 4, 1, 5
    run = chain.StageChainRunner(events, sc, max_stages=5, min_wires=30, max_back_steps=3000,
                                 n_ref=R, n_iter=n_iter, n_fine=n_fine, n_final=F,
                                 fit_iters=fit_iters, eta=0.3)
    run.run()
    torch.cuda.synchronize()
    first = run.stage_of_hit.clone()
    run.run()                                   # a second run starts from the same events
    torch.cuda.synchronize()
    assert torch.equal(run.stage_of_hit, first)
    soh = run.stage_of_hit.cpu().numpy()
    best = run.best.cpu().numpy()
    chosen, fitted = run.chosen.cpu().numpy(), run.fitted.cpu().numpy()
    nc = run.n_complete_at.cpu().numpy()
    h0, n_stages, n_complete = 0, 0, 0
    for e, ev in enumerate(events):
        want, per_stage = _oracle_chain_stages(orc, ev, sc, 5, 30, 3000, n_fine, R, n_iter, F,
                                               fit_iters, 0.3)
        assert np.array_equal(soh[h0:h0 + ev.n_hits], want), e
        for s, (b, seed, fit, wnc) in enumerate(per_stage):
            assert best[s, e] == b, (e, s)
            assert nc[s, e] == wnc, (e, s)
            if fit_iters == 0:
                assert np.array_equal(chosen[s, e], seed, equal_nan=True), (e, s)
            else:
                np.testing.assert_allclose(chosen[s, e], seed, rtol=1e-7, atol=1e-9)
                np.testing.assert_allclose(fitted[s, e], fit, rtol=1e-7, atol=1e-9)
            n_complete += int(wnc > 0)
        n_stages += len(per_stage)
        h0 += ev.n_hits
    assert n_stages > len(events) and n_complete > 0


def test_stage_chain_bench_size_matches_cpu(orc):
    """The chain at the bench's sizes (each half: 8 x 16 x 16 x 16 first grid, 10
    references, two re-scans of 10 x 4 x 8 x 8 x 8, 10 final seeds, 500 x 2 mm; the fit
    with 8 LM iterations over 1000 x 2 mm) on a two-turn event: both stages' pairs,
    complete-set counts and seeds, and the stage of every hit."""
    events = [synth.event_mix(0)]
    sc = synth.C2
    F = 10
    run = chain.StageChainRunner(events, sc, n_ref=10, n_iter=2, n_fine=(4, 8, 8, 8),
                                 n_final=F, fit_iters=8, eta=0.3)
    run.run()
    torch.cuda.synchronize()
    want, per_stage = _oracle_chain_stages(orc, events[0], sc, 5, 30, 4000, (4, 8, 8, 8), 10, 2,
                                           F, 8, 0.3)
    assert np.array_equal(run.stage_of_hit.cpu().numpy(), want)
    best, nc = run.best.cpu().numpy(), run.n_complete_at.cpu().numpy()
    chosen, fitted = run.chosen.cpu().numpy(), run.fitted.cpu().numpy()
    assert len(per_stage) == 2
    for s, (b, seed, fit, wnc) in enumerate(per_stage):
        assert best[s, 0] == b and nc[s, 0] == wnc, s
        if s == 0:
            assert np.array_equal(chosen[s, 0], seed), s
        else:
            np.testing.assert_allclose(chosen[s, 0], seed, rtol=1e-7, atol=1e-9)
        np.testing.assert_allclose(fitted[s, 0], fit, rtol=1e-7, atol=1e-9)
