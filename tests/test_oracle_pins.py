"""The CPU reference against its pins (closed forms, hand cases, invariants, brute force)."""
import pytest

import pins


@pytest.mark.parametrize("check", pins.ALL_SIMPLE, ids=lambda f: f.__name__)
def test_simple_pin(orc, check):
    check(orc)


def test_far_seed(orc, ev_plain):
    pins.pin_far_seed(orc, ev_plain)


def test_truth_seed_exact_drift(orc, ev_plain_exact):
    pins.pin_truth_seed(orc, ev_plain_exact)


def test_grid_argmin_is_truth(orc, ev_plain_exact):
    pins.pin_grid_argmin(orc, ev_plain_exact)


def test_rotation_invariance(orc, ev_plain):
    pins.pin_rotation(orc, ev_plain)


def test_brute_force_long_double(orc, ev_plain):
    pins.pin_brute_force(orc, ev_plain)


def test_scan_threads_deterministic(orc, ev_signal):
    """The CPU result does not depend on the thread count (Sec. 4.1)."""
    import numpy as np
    from paper_1911_09340_amd import synth
    cfg = synth.ScanConfig("t", (2, 2, 3, 5), (5.0, 5.0, 0.05, 0.05), 300, 2.0, 0.8)
    grid = synth.grid_descriptor(ev_signal.ref_states[1], cfg)
    seeds = orc.seed_grid(grid, np.array(cfg.n, dtype=np.int32))
    c = [ev_signal.bz, ev_signal.charge, 2.0, 0.8]
    r1, used1 = orc.scan(seeds, c, 300, ev_signal.wire_ends, ev_signal.wire_offsets,
                         ev_signal.drift, n_threads=1)
    r4, used4 = orc.scan(seeds, c, 300, ev_signal.wire_ends, ev_signal.wire_offsets,
                         ev_signal.drift, n_threads=4)
    assert used1 == 1
    assert np.array_equal(r1, r4)


def test_gradient_vs_central_differences(orc, ev_plain):
    pins.pin_gradient_fd(orc, ev_plain)


def test_lm_recovers_truth(orc, ev_plain_exact):
    pins.pin_lm_truth(orc, ev_plain_exact)
