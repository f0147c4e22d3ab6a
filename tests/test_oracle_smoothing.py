"""Pins of the oracle's Gaussian pre-smoothing (the smoothing inside Eq. 2,
Sec. III-B: a Gaussian filter of standard deviation 3 pixels)."""
import json
import os

import numpy as np
import pytest
import scipy.ndimage as ndi

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_paper_constants_fixture():
    g = json.load(open(os.path.join(GOLD, "paper_constants.json")))
    prm = oracle.Params()
    assert prm.seg_len == g["segment_length_L"]["value"]
    assert prm.sigma == g["gaussian_sigma_px"]["value"]
    # 1,000 frames give 20 summary pairs: non-overlapping segments
    assert g["training_video_frames"]["value"] // prm.seg_len == g["summary_pairs_per_video"]["value"]


def test_weights_closed_form():
    w = oracle.gaussian_weights(3.0, 12)
    assert w.shape == (25,)
    assert abs(w.sum() - 1.0) < 1e-15
    k = np.arange(-12, 13)
    np.testing.assert_allclose(w / w[12], np.exp(-k * k / 18.0), rtol=1e-15)
    np.testing.assert_array_equal(w, w[::-1])


@pytest.mark.parametrize("j,n,expect", [(-1, 4, 0), (-2, 4, 1), (-4, 4, 3), (-5, 4, 3),
                                        (-8, 4, 0), (4, 4, 3), (5, 4, 2), (7, 4, 0),
                                        (8, 4, 0), (12, 4, 3), (0, 1, 0), (-3, 1, 0),
                                        (13, 5, 3)])
def test_reflect_index_hand_worked(j, n, expect):
    # half-sample symmetric extension of [a b c d]: ... d c b a | a b c d | d c b a ...
    assert oracle.reflect_index(j, n) == expect


@pytest.mark.parametrize("shape", [(1, 64, 64), (3, 17, 13), (2, 5, 4), (1, 1, 7), (2, 30, 2)])
def test_matches_scipy_reflect(shape):
    rng = np.random.default_rng(1)
    f = rng.integers(0, 65535, size=shape).astype(np.float64)
    got = oracle.smooth_frames(f, 3.0, 12)
    for t in range(shape[0]):
        ref = ndi.gaussian_filter(f[t], 3.0, mode="reflect", truncate=4.0)
        np.testing.assert_allclose(got[t], ref, rtol=0, atol=1e-9 * np.abs(f).max())


def _brute(frame, w, r):
    H, W = frame.shape
    out = np.zeros((H, W))
    for y in range(H):
        for x in range(W):
            acc = 0.0
            for dy in range(-r, r + 1):
                for dx in range(-r, r + 1):
                    yy = oracle.reflect_index(y + dy, H)
                    xx = oracle.reflect_index(x + dx, W)
                    acc += w[dy + r] * w[dx + r] * frame[yy, xx]
            out[y, x] = acc
    return out


@pytest.mark.parametrize("shape", [(13, 17), (5, 4), (3, 26)])
def test_brute_force_2d(shape):
    rng = np.random.default_rng(2)
    f = rng.integers(0, 4000, size=shape).astype(np.float64)
    w = oracle.gaussian_weights(3.0, 12)
    np.testing.assert_allclose(oracle.smooth_frames(f[None], 3.0, 12)[0], _brute(f, w, 12),
                               rtol=1e-12, atol=1e-9)


def test_constant_frame_unchanged():
    f = np.full((1, 9, 31), 777.0)
    np.testing.assert_allclose(oracle.smooth_frames(f), f, rtol=1e-14)


def test_impulse_response_interior():
    f = np.zeros((1, 41, 41))
    f[0, 20, 20] = 1.0
    w = oracle.gaussian_weights(3.0, 12)
    out = oracle.smooth_frames(f)[0]
    np.testing.assert_allclose(out[8:33, 8:33], np.outer(w, w), atol=1e-16)
    assert abs(out.sum() - 1.0) < 1e-13


def test_gaussian_blob_continuous_limit():
    # a sampled Gaussian blob of sd s smoothed by sd 3 is close to a Gaussian of
    # variance s^2 + 9 with amplitude s^2 / (s^2 + 9) (loose sanity pin)
    s = 4.0
    yy, xx = np.mgrid[0:81, 0:81] - 40.0
    blob = np.exp(-(xx ** 2 + yy ** 2) / (2 * s * s))
    out = oracle.smooth_frames(blob[None])[0]
    v = s * s + 9.0
    expect = (s * s / v) * np.exp(-(xx ** 2 + yy ** 2) / (2 * v))
    assert np.abs(out - expect).max() < 2e-3
