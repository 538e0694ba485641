"""Hit-classification efficiency and purity (Sec. 3.2.1) on hand-made masks."""
import numpy as np

from paper_1911_09340_amd import quality


def test_turn_metrics_hand_cases():
    hit_turn = np.array([0, 0, 0, 1, 1, -1, -1, 2])
    # classified: two of turn 0, one of turn 1, one noise -> turn 0 represented
    mask = np.array([1, 1, 0, 1, 0, 1, 0, 0], np.uint8)
    e, p, t = quality.turn_metrics(mask, hit_turn)
    assert t == 0 and e == 2 / 3 and p == 2 / 4
    # bit 1 alone (borderline) is not a classification
    e, p, t = quality.turn_metrics(np.array([2, 2, 2, 0, 0, 0, 0, 0], np.uint8), hit_turn)
    assert (e, t) == (0.0, -1) and np.isnan(p)
    # only noise classified: efficiency 0, purity 0
    e, p, t = quality.turn_metrics(np.array([0, 0, 0, 0, 0, 1, 1, 0], np.uint8), hit_turn)
    assert (e, p, t) == (0.0, 0.0, -1)
    # a tie between turns 1 and 0 goes to the lower index; all of turn 2
    e, p, t = quality.turn_metrics(np.array([1, 0, 0, 1, 0, 0, 0, 0], np.uint8), hit_turn)
    assert t == 0 and e == 1 / 3 and p == 1 / 2
    e, p, t = quality.turn_metrics(np.array([0, 0, 0, 0, 0, 0, 0, 3], np.uint8), hit_turn)
    assert (e, p, t) == (1.0, 1.0, 2)


def test_classification_over_partitions():
    class Ev:
        def __init__(self, hit_turn, n_turns):
            self.hit_turn = np.asarray(hit_turn)
            self.n_hits = self.hit_turn.size
            self.n_turns = n_turns

    events = [Ev([0, 0, 1, -1], 2), Ev([0, 0, 0], 1)]
    mask = np.zeros((3, 4), np.uint8)
    mask[0, :2] = 1          # turn 0 of event 0: perfect
    mask[1, 1:3] = 1         # turn 1 of event 0: one of turn 0, one of turn 1 -> turn 0
    mask[2, :3] = 1          # event 1: perfect
    mask[2, 3] = 1           # past the event's hits: ignored
    q = quality.classification(mask, events)
    assert q["partitions"] == 3
    assert q["represents_own_turn"] == 2 / 3
    assert np.isclose(q["efficiency_mean"], (1 + 0.5 + 1) / 3)
    assert np.isclose(q["purity_mean"], (1 + 0.5 + 1) / 3)
    assert np.isclose(q["eff_and_purity_above_0.9"], 2 / 3)
