"""The seeded synthetic workloads have the shapes the measurements quote (CPU only)."""
import numpy as np
import pytest

from paper_1911_09340_amd import synth


def _valid_csr(ev):
    assert ev.wire_offsets[0] == 0 and ev.wire_offsets[-1] == ev.n_hits
    assert np.all(np.diff(ev.wire_offsets) >= 1)          # every wire holds a hit
    assert np.all(np.diff(ev.wire_ids) > 0)               # sorted, unique
    assert np.all((ev.drift >= 0.0) & (ev.drift <= synth.DRIFT_MAX))
    ends = ev.wire_ends
    assert np.all(np.abs(ends[:, 2]) == 750.0) and np.all(np.abs(ends[:, 5]) == 750.0)


def test_chamber_geometry():
    w = synth.chamber_wires()
    assert w.shape == (18 * 320, 6)
    mid = 0.5 * (w[:, :3] + w[:, 3:])
    r = np.hypot(mid[:, 0], mid[:, 1])
    for layer in (0, 9, 17):
        rl = r[layer * 320:(layer + 1) * 320]
        assert np.allclose(rl, 530.0 + layer * 300.0 / 17.0, rtol=0, atol=1e-9)


def test_plain_event_shape():
    ev = synth.event_plain(0)
    _valid_csr(ev)
    assert ev.n_turns == 1 and ev.n_hits == 42 and ev.n_wires == 42
    assert ev.meta["n_noise"] == 0
    p = np.linalg.norm(ev.ref_states[0, 3:])
    assert abs(p - 100.0) < 1e-9
    assert abs(np.hypot(*ev.ref_states[0, :2]) - synth.SEED_RADIUS) < 1e-3


def test_signal_event_shape():
    ev = synth.event_signal(0)
    _valid_csr(ev)
    assert ev.n_turns == 3 and ev.n_hits == 227 and ev.n_wires == 172
    n_sig = ev.meta["n_signal"]
    assert ev.meta["n_noise"] == round(0.10 * n_sig)
    for t in range(3):
        assert 40 <= np.sum(ev.hit_turn == t) <= 110
    r = np.hypot(ev.ref_states[:, 0], ev.ref_states[:, 1])
    assert np.all(np.abs(r - synth.SEED_RADIUS) < 1e-3)


@pytest.mark.parametrize("seed", range(12))
def test_mix_event_shape(seed):
    ev = synth.event_mix(seed)
    _valid_csr(ev)
    assert 40 <= ev.n_hits <= 400
    assert 1 <= ev.n_turns <= 5
    n_sig, n_noise = ev.meta["n_signal"], ev.meta["n_noise"]
    assert n_noise == round(0.25 * n_sig)                 # 20 % of the total
    assert np.sum(ev.hit_turn < 0) == n_noise


def test_mix_is_seeded():
    a, b = synth.event_mix(3), synth.event_mix(3)
    assert np.array_equal(a.drift, b.drift) and np.array_equal(a.wire_ids, b.wire_ids)
    assert not np.array_equal(synth.event_mix(4).drift[:10], a.drift[:10])


def test_grid_descriptor_layout():
    ev = synth.event_plain(0)
    g = synth.grid_descriptor(ev.ref_states[0], synth.C0)
    assert g.shape == (14,)
    assert np.array_equal(g[:6], ev.ref_states[0])
    assert g[6] == 0.0 and abs(g[7] - 100.0) < 1e-9 and g[8] == 0.0 and g[9] == 0.0
    assert np.array_equal(g[10:], [5.0, 5.0, 0.05, 0.05])
    assert synth.C1.n_seeds == 65536 and synth.C2.n_seeds == 32768
    assert synth.C3_FINE.n_seeds == 32 ** 4 and synth.C3_COARSE.n_seeds == 8 ** 4


def test_exit_states_and_half_split():
    """The exit seed sits on r = 500 mm moving inward, mirrors the entrance point across
    the line through the axis and the circle centre, and the two halves partition the
    event's wires and hits."""
    for seed in range(4):
        ev = synth.event_mix(seed)
        for t in range(ev.n_turns):
            ref, ext = ev.ref_states[t], ev.exit_states[t]
            assert abs(np.hypot(ext[0], ext[1]) - synth.SEED_RADIUS) < 1e-6
            assert ext[0] * ext[3] + ext[1] * ext[4] < 0          # inward
            assert ref[0] * ref[3] + ref[1] * ref[4] > 0          # outward
            c = synth.circle_centre(ref, ev.charge, ev.bz)
            cx = synth.circle_centre(ext, ev.charge, ev.bz)
            assert np.allclose(c, cx, atol=1e-6)                  # same circle
            u = c / np.linalg.norm(c)
            mirror = 2.0 * np.dot(ref[:2], u) * u - ref[:2]
            assert np.allclose(mirror, ext[:2], atol=1e-6)
            a, b = synth.half_events(ev, t)
            assert a.n_wires + b.n_wires == ev.n_wires
            assert sorted(np.concatenate([a.wire_ids, b.wire_ids]).tolist()) == ev.wire_ids.tolist()
            hits = np.concatenate([a.meta["hits"], b.meta["hits"]])
            assert sorted(hits.tolist()) == list(range(ev.n_hits))
            assert np.array_equal(a.drift, ev.drift[a.meta["hits"]])
            assert np.array_equal(b.ref_states[0], np.concatenate([ext[:3], -ext[3:]]))
            assert b.charge == -ev.charge and a.charge == ev.charge
            # the flipped exit seed retraces the turn backwards: same circle centre
            assert np.allclose(synth.circle_centre(b.ref_states[0], b.charge, b.bz), c, atol=1e-6)
            # each half holds a good share of the turn's own hits
            own = np.sum(ev.hit_turn == t)
            assert np.sum(a.hit_turn == t) > 0.25 * own and np.sum(b.hit_turn == t) > 0.25 * own
