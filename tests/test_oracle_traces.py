"""Pins of the trace-extraction oracle (mean intensity inside each ROI per
frame, Sec. II) against closed forms and brute force."""
import numpy as np

from oracle.traces import extract_traces


def test_constant_video_gives_the_constant():
    v = np.full((7, 5, 6), 1234, np.uint16)
    m = np.zeros((2, 5, 6), bool)
    m[0, 1:3, 2:5] = True
    m[1, 4, 0] = True
    assert np.array_equal(extract_traces(v, m), np.full((2, 7), 1234.0))


def test_single_pixel_mask_is_that_pixel():
    rng = np.random.default_rng(1)
    v = rng.integers(0, 65536, size=(20, 8, 9), dtype=np.uint16)
    m = np.zeros((1, 8, 9), bool)
    m[0, 3, 7] = True
    assert np.array_equal(extract_traces(v, m)[0], v[:, 3, 7].astype(np.float64))


def test_hand_worked_mean():
    v = np.zeros((2, 3, 3), np.uint16)
    v[0] = [[1, 2, 3], [4, 5, 6], [7, 8, 9]]
    v[1] = 10 * v[0]
    m = np.zeros((1, 3, 3), bool)
    m[0, 0, 0] = m[0, 1, 1] = m[0, 2, 1] = True          # 1, 5, 8
    assert np.allclose(extract_traces(v, m)[0], [14 / 3, 140 / 3], rtol=0, atol=1e-12)


def test_affine_maps_exactly():
    """trace(a V + b) = a trace(V) + b for integers (exact in the integer sum)."""
    rng = np.random.default_rng(2)
    v = rng.integers(0, 1000, size=(15, 10, 10), dtype=np.uint16)
    m = rng.random((3, 10, 10)) < 0.3
    t = extract_traces(v, m)
    w = (3 * v.astype(np.int64) + 17).astype(np.uint16)
    assert np.allclose(extract_traces(w, m), 3 * t + 17, rtol=1e-15, atol=1e-9)


def test_brute_force_and_empty_mask():
    rng = np.random.default_rng(3)
    v = rng.integers(0, 65536, size=(6, 4, 5), dtype=np.uint16)
    m = rng.random((3, 4, 5)) < 0.5
    m[2] = False
    t = extract_traces(v, m)
    for j in range(2):
        for f in range(6):
            vals = [int(v[f, y, x]) for y in range(4) for x in range(5) if m[j, y, x]]
            assert t[j, f] == sum(vals) / len(vals)
    assert np.array_equal(t[2], np.zeros(6))
