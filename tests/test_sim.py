"""Seeded simulator: determinism and its Poisson-Gaussian statistics."""
import numpy as np

from synth import draw, preset, simulate, simulate_frames, session_mix


def test_deterministic_any_thread_count():
    a, _ = simulate(preset(1, frames=300), 4, threads=1)
    b, _ = simulate(preset(1, frames=300), 4, threads=8)
    assert np.array_equal(a, b)


def test_frame_ranges_match_whole_video():
    cfg = preset(1, frames=400)
    v, _ = simulate(cfg, 5)
    bundle = draw(cfg, 5)
    part = simulate_frames(cfg, 5, 150, 300, bundle)
    assert np.array_equal(part, v[150:300])


def test_flat_background_poisson_gaussian_moments():
    # no neurons, flat background, no drift: V ~ round(Poisson(1000) + N(0, 25))
    cfg = preset(1, n_blobs=0, n_neurons=0, drift=0.0, frames=200)
    v, truth = simulate(cfg, 6)
    x = v.astype(np.float64)
    n = x.size
    mean_expect = 1000.0
    var_expect = 1000.0 + 25.0 + 1.0 / 12.0
    assert abs(x.mean() - mean_expect) < 4 * np.sqrt(var_expect / n)
    # sample variance SE ~ var * sqrt(2 / n)
    assert abs(x.var() - var_expect) < 4 * var_expect * np.sqrt(2.0 / n) + 1.0


def test_spike_counts_poisson_rate():
    cfg = preset(1, frames=20000, n_neurons=4)
    from synth.simulate import draw as d
    truth = d(cfg, 7)[0]
    p = 10.0 / cfg.fps
    for s in truth.spikes:
        assert abs(len(s) - p * cfg.frames) < 5 * np.sqrt(p * (1 - p) * cfg.frames)


def test_segment_masks_and_mix():
    v, truth = simulate(preset(1), 0)
    sm = truth.segment_masks(50)
    assert sm.shape == (20, 64, 64) and sm.any()
    mix = session_mix(16, 5000)
    assert len(mix) == 16
    assert all((m["height"], m["width"]) in [(128, 128), (256, 256), (512, 128), (512, 512)] for m in mix)
    assert all(mix[i]["arrival"] <= mix[i + 1]["arrival"] for i in range(15))
