"""Pins of the F1 metric (Sec. IV-B, IoU threshold 0.3) and of the whole
oracle against planted ground truth from the seeded simulator."""
import numpy as np
import pytest
from scipy.optimize import linear_sum_assignment

import oracle
from oracle.metrics import _assign
from synth import preset, simulate


@pytest.mark.parametrize("seed", range(6))
def test_assignment_matches_scipy(seed):
    rng = np.random.default_rng(seed)
    w = rng.random((4 + seed, 6))
    pairs = _assign(w)
    r, c = linear_sum_assignment(w, maximize=True)
    assert abs(sum(w[i, j] for i, j in pairs) - w[r, c].sum()) < 1e-12
    assert len({i for i, _ in pairs}) == len(pairs) == min(w.shape)


def test_f1_hand_worked():
    H = W = 10
    ref = np.zeros((2, H, W), bool)
    ref[0, 0:4, 0:4] = True
    ref[1, 6:10, 6:10] = True
    pred = np.zeros((3, H, W), bool)
    pred[0, 0:4, 0:3] = True     # IoU 12/16 = 0.75 with ref 0
    pred[1, 6:10, 9:10] = True   # IoU 4/16 = 0.25 < 0.3: no match
    pred[2, 5:6, 5:6] = True
    f = oracle.match_f1(pred, ref, 0.3)
    assert f["precision"] == pytest.approx(1 / 3)
    assert f["recall"] == pytest.approx(1 / 2)
    assert f["f1"] == pytest.approx(0.4)
    assert f["matches"] == [(0, 0, 0.75)]


def test_f1_empty_cases():
    z = np.zeros((0, 4, 4), bool)
    one = np.ones((1, 4, 4), bool)
    assert oracle.match_f1(z, z)["f1"] == 1.0
    assert oracle.match_f1(one, z)["f1"] == 0.0
    assert oracle.match_f1(z, one)["f1"] == 0.0


def _masks(res, shape):
    return (np.array([f["mask"] for f in res.footprints])
            if res.footprints else np.zeros((0,) + shape, bool))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_planted_truth_config1(seed):
    v, truth = simulate(preset(1), seed)
    res = oracle.segment(v, with_corr=False)
    f = oracle.match_f1(_masks(res, v.shape[1:]), truth.masks(), 0.3)
    assert f["f1"] == 1.0, f


@pytest.mark.parametrize("seed", [2000, 2001])
def test_planted_truth_config2_style(seed):
    cfg = preset(2, height=128, width=128, frames=2000, n_neurons=8, n_overlap=2)
    v, truth = simulate(cfg, seed)
    res = oracle.segment(v, with_corr=False)
    f = oracle.match_f1(_masks(res, v.shape[1:]), truth.masks(), 0.3)
    assert f["f1"] >= 0.85, f


@pytest.mark.parametrize("seed", [10, 11, 12, 13])
def test_zero_activity_yields_no_neurons(seed):
    # neurons present but silent, and no neurons at all
    cfg = preset(1, rate_range=(0.0, 0.0)) if seed % 2 else preset(1, n_neurons=0)
    v, _ = simulate(cfg, seed)
    res = oracle.segment(v, with_corr=False)
    assert res.n_comp == 0 and res.footprints == []


def test_zero_activity_structured_background():
    cfg = preset(2, height=128, width=128, frames=2000, n_neurons=0, n_overlap=0)
    v, _ = simulate(cfg, 2100)
    res = oracle.segment(v, with_corr=False)
    assert res.footprints == []


def test_trailing_partial_segment_dropped():
    v, _ = simulate(preset(1, frames=1050), 3)
    a = oracle.segment(v[:1000], with_corr=False)
    b = oracle.segment(v[:1025], with_corr=False)
    assert b.T.shape[0] == 20
    np.testing.assert_array_equal(a.T, b.T)
    np.testing.assert_array_equal(a.labels, b.labels)
