"""Tracking in a field map (Sec. 2.2.1) on the GPU vs the CPU reference: RK4 tracks in
the synthetic solenoid map bit for bit (tracks that leave the map's grid included), and
the RSS of a partition scanned with map tracks."""
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


@pytest.fixture(scope="module")
def fmap():
    return synth.solenoid_map(g=0.3, z_scale=1000.0, half_xy=700.0, half_z=900.0)


def _gpu_tracks(seeds, cfg, fmap):
    f = comet.FieldMap(*fmap)
    S = seeds.shape[1]
    track = torch.empty(3, cfg.n_steps + 1, S, dtype=torch.float64, device="cuda")
    comet.extrapolate_seeds_field(torch.as_tensor(np.ascontiguousarray(seeds), device="cuda"),
                                  cfg, f, track)
    torch.cuda.synchronize()
    return track


def test_field_tracks_match_cpu(orc, fmap):
    ev = synth.event_mix(1)
    sc = synth.ScanConfig("field", (2, 3, 4, 5), (5.0, 5.0, 0.05, 0.05), 700, 2.0, 0.8, 0)
    g = synth.grid_descriptor(ev.ref_states[0], sc)
    seeds = orc.seed_grid(g, np.array(sc.n, np.int32))          # 120 seeds, ragged tiles
    # two seeds that start outside the map's grid (clamped field) and one inside it
    extra = np.array([[900.0, 0.0, 0.0, 0.0, 80.0, 20.0], [0.0, -100.0, 1200.0, 60.0, 0.0, -30.0],
                      [100.0, 50.0, -300.0, -40.0, 70.0, 10.0]]).T
    seeds = np.concatenate([seeds, extra], axis=1)
    cfg = comet.make_config(1.0, ev.charge, sc.step_mm, sc.n_steps, sc.lambda_mm)
    got = _gpu_tracks(seeds, cfg, fmap).cpu().numpy()
    for s in range(seeds.shape[1]):
        want = orc.track_field(seeds[:, s], fmap, ev.charge, sc.step_mm, sc.n_steps)
        assert np.array_equal(got[:, :, s].T, want), s


def test_field_partition_rss_matches_cpu(orc, fmap):
    """A 3x4x5x6 grid scanned with map tracks: every RSS and the argmin, bit for bit."""
    ev = synth.event_mix(4)
    sc = synth.ScanConfig("field-p", (3, 4, 5, 6), (5.0, 5.0, 0.05, 0.05), 600, 2.0, 0.8, 0)
    cfg = scan.config_for(ev, sc)
    f = comet.FieldMap(*fmap)
    r = scan.PartitionScanner(sc.n, cfg, ev.n_wires, ev.n_hits, field=f)
    dev = scan.DeviceEvent.from_event(ev)
    r.run(dev, scan.grid_tensor(ev.ref_states[0], sc), 0)
    torch.cuda.synchronize()
    got = r.rss.cpu().numpy()
    g = synth.grid_descriptor(ev.ref_states[0], sc)
    seeds = orc.seed_grid(g, np.array(sc.n, np.int32))
    want = np.array([orc.rss_track(orc.track_field(seeds[:, s], fmap, ev.charge, sc.step_mm,
                                                   sc.n_steps),
                                   ev.wire_ends, ev.wire_offsets, ev.drift, sc.lambda_mm)
                     for s in range(seeds.shape[1])])
    assert np.array_equal(got, want)
    assert int(r.best.item()) == int(np.argmin(want))
