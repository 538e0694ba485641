"""The allocation-free entry point (comet_track_dca_rss_static) against the entry point
with a caller's workspace (comet_track_dca_rss): track and RSS bit for bit, on two calls
in a row, the second smaller than the first (the fixed array keeps the first call's
contents), in the uniform field and in a field map; sizes past the fixed array are
rejected before any device work."""
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


def _seeds(ev, sc, turn, count):
    g = torch.as_tensor(synth.grid_descriptor(ev.ref_states[turn], sc), device="cuda")
    seeds = torch.empty(6, sc.n_seeds, dtype=torch.float64, device="cuda")
    comet.seed_grid(g, np.array(sc.n, np.int32), seeds)
    return seeds[:, :count].contiguous()


def _both(ev, seeds, cfg, field=None):
    dev = scan.DeviceEvent.from_event(ev)
    S, P = int(seeds.shape[1]), cfg.n_steps + 1
    out = []
    for static in (False, True):
        track = torch.full((3, P, S), float("nan"), dtype=torch.float64, device="cuda")
        rss = torch.full((S,), float("nan"), dtype=torch.float64, device="cuda")
        if static:
            comet.track_dca_rss_static(seeds, dev.wire_ends, dev.wire_offsets, dev.drift, cfg,
                                       track, rss, field=field)
        else:
            ws = comet.dca_workspace(S, P, dev.n_wires)
            comet.track_dca_rss(seeds, dev.wire_ends, dev.wire_offsets, dev.drift, cfg, track,
                                rss, ws, field=field)
        torch.cuda.synchronize()
        out.append((track.cpu().numpy(), rss.cpu().numpy()))
    return out


def test_static_workspace_matches_caller_workspace_two_calls():
    ev1, sc1 = synth.event_signal(0), synth.C1
    cfg1 = scan.config_for(ev1, sc1)
    S1 = 8192
    assert comet.dca_workspace_bytes(S1, sc1.n_steps + 1, ev1.n_wires) <= \
        comet.static_scratch_bytes()
    (t_ws, r_ws), (t_st, r_st) = _both(ev1, _seeds(ev1, sc1, 1, S1), cfg1)
    assert np.all(np.isfinite(r_ws))
    assert np.array_equal(t_st, t_ws) and np.array_equal(r_st, r_ws)
    # a second, smaller call: other event, fewer seeds, wires and steps
    ev2, sc2 = synth.event_plain(0), synth.C0
    cfg2 = scan.config_for(ev2, sc2)
    (t_ws, r_ws), (t_st, r_st) = _both(ev2, _seeds(ev2, sc2, 0, 1000), cfg2)
    assert np.all(np.isfinite(r_ws))
    assert np.array_equal(t_st, t_ws) and np.array_equal(r_st, r_ws)


@pytest.mark.parametrize("stepper", [0, 1])
def test_static_workspace_in_field_map(stepper):
    ev, sc = synth.event_signal(0), synth.C1
    cfg = scan.config_for(ev, sc)
    fmap = comet.FieldMap(*synth.solenoid_map(g=0.3, z_scale=1000.0, half_xy=700.0,
                                              half_z=900.0), stepper=stepper)
    (t_ws, r_ws), (t_st, r_st) = _both(ev, _seeds(ev, sc, 0, 2000), cfg, field=fmap)
    assert np.all(np.isfinite(r_ws))
    assert np.array_equal(t_st, t_ws) and np.array_equal(r_st, r_ws)


def test_static_workspace_rejects_oversize():
    ev, sc = synth.event_signal(0), synth.C1
    cfg = scan.config_for(ev, sc)
    S = sc.n_seeds   # 65536 seeds x 1501 points x 172 wires: ~140 MB of workspace
    assert comet.dca_workspace_bytes(S, sc.n_steps + 1, ev.n_wires) > comet.static_scratch_bytes()
    dev = scan.DeviceEvent.from_event(ev)
    seeds = torch.zeros(6, S, dtype=torch.float64, device="cuda")
    track = torch.zeros(3, sc.n_steps + 1, S, dtype=torch.float64, device="cuda")
    rss = torch.full((S,), 7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(comet.CometError) as e:
        comet.track_dca_rss_static(seeds, dev.wire_ends, dev.wire_offsets, dev.drift, cfg, track,
                                   rss)
    assert e.value.status == -2 and "split the seeds" in str(e.value)
    torch.cuda.synchronize()
    assert bool((rss == 7.0).all())
