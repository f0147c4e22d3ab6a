"""Pins of the motion-correction oracle (patch-wise ZNCC, Sec. II) against a
library routine, closed forms, brute force and planted motion."""
import numpy as np

import oracle.motion as om
from synth import move_frames, plant_motion, preset, simulate


def test_zncc_is_pearson_correlation():
    rng = np.random.default_rng(0)
    for _ in range(20):
        a = rng.integers(0, 65536, 441)
        b = rng.integers(0, 65536, 441) + (a // 3)
        assert abs(om.zncc(a, b) - np.corrcoef(a, b)[0, 1]) <= 1e-12


def test_zncc_closed_forms():
    rng = np.random.default_rng(1)
    a = rng.normal(size=(21, 21))
    assert abs(om.zncc(a, a) - 1.0) <= 1e-12
    assert abs(om.zncc(a, -a) + 1.0) <= 1e-12
    b = rng.normal(size=(21, 21))
    assert abs(om.zncc(3.5 * a + 100.0, b) - om.zncc(a, b)) <= 1e-12
    assert abs(om.zncc(a, b) - om.zncc(b, a)) <= 1e-15
    assert om.zncc(np.full((21, 21), 7.0), b) == 0.0
    assert om.zncc(a, np.zeros((21, 21))) == 0.0


def test_template_rounds_half_up():
    f = np.array([[[1]], [[2]]], np.uint16)            # mean 1.5 -> 2
    assert om.make_template(f)[0, 0] == 2
    f = np.array([[[1]], [[1]], [[2]]], np.uint16)     # mean 1.33 -> 1
    assert om.make_template(f)[0, 0] == 1
    f = np.array([[[65535]], [[65534]]], np.uint16)    # 65534.5 -> 65535
    assert om.make_template(f)[0, 0] == 65535
    rng = np.random.default_rng(2)
    g = rng.integers(0, 65536, size=(50, 8, 8), dtype=np.uint16)
    mean = g.astype(np.float64).mean(0)
    assert np.array_equal(om.make_template(g), np.floor(mean + 0.5).astype(np.uint16))


def test_patch_grid_and_vectors():
    assert om.patch_grid(64, 64, 4) == [(11, 11), (11, 32), (32, 11), (32, 32)]
    g = om.patch_grid(256, 256, 8)
    assert len(g) == 121 and g[0] == (12, 12) and g[-1] == (222, 222)
    # 40 - 4 = 36 leaves 15 rows beside one tile, 100 - 4 = 96 leaves 12 beside four
    assert om.patch_grid(40, 100, 2) == [(2 + 15 // 2, 2 + 12 // 2 + 21 * j) for j in range(4)]
    for (y, x) in g:                                    # every shifted window is inside
        assert y - 8 >= 0 and x - 8 >= 0 and y + 21 + 8 <= 256 and x + 21 + 8 <= 256
    v = om.vectors(2)
    assert len(v) == 25 and v[0] == (-2, -2) and v[1] == (-2, -1) and v[12] == (0, 0)


def test_table_against_brute_force():
    rng = np.random.default_rng(3)
    R = 2
    tmpl = rng.integers(500, 1500, size=(30, 52), dtype=np.uint16)
    frame = rng.integers(500, 1500, size=(30, 52), dtype=np.uint16)
    grid = om.patch_grid(30, 52, R)
    assert len(grid) == 2
    z = om.zncc_table(frame, tmpl, R)
    for k, (y, x) in enumerate(grid):
        for v, (dy, dx) in enumerate(om.vectors(R)):
            fp = [float(frame[y + i, x + j]) for i in range(21) for j in range(21)]
            tp = [float(tmpl[y + dy + i, x + dx + j]) for i in range(21) for j in range(21)]
            mf, mt = sum(fp) / 441, sum(tp) / 441
            num = sum((a - mf) * (b - mt) for a, b in zip(fp, tp))
            den = (sum((a - mf) ** 2 for a in fp) * sum((b - mt) ** 2 for b in tp)) ** 0.5
            assert abs(z[k, v] - num / den) <= 1e-12
    s = om.scores(frame, tmpl, R)
    assert np.allclose(s, z.sum(0), rtol=0, atol=1e-13)


def _texture(H, W, seed):
    """Smooth random texture (sum of Gaussian bumps) as uint16."""
    rng = np.random.default_rng(seed)
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    img = np.full((H, W), 1000.0)
    for _ in range(60):
        cy, cx, s, a = rng.uniform(0, H), rng.uniform(0, W), rng.uniform(2, 6), rng.uniform(-300, 300)
        img += a * np.exp(-((yy - cy) ** 2 + (xx - cx) ** 2) / (2 * s * s))
    return np.clip(np.rint(img), 0, 65535).astype(np.uint16)


def test_planted_shift_recovered_exactly_on_a_texture():
    R = 4
    tmpl = _texture(80, 96, 4)
    shifts = np.array([(dy, dx) for dy in range(-R, R + 1) for dx in range(-R, R + 1)], np.int32)
    frames = move_frames(np.repeat(tmpl[None], len(shifts), 0), shifts)
    got, sc = om.estimate(frames, tmpl, R)
    assert np.array_equal(got, shifts)
    # the best vector reaches the patch count (every patch correlates to 1)
    P = len(om.patch_grid(80, 96, R))
    assert np.allclose(sc.max(axis=1), P, rtol=0, atol=1e-9)
    corr = om.apply_shifts(frames, got, tmpl)
    assert np.array_equal(corr[:, R:-R, R:-R], np.repeat(tmpl[None], len(shifts), 0)[:, R:-R, R:-R])


def test_apply_shifts_closed_forms():
    rng = np.random.default_rng(5)
    f = rng.integers(0, 65536, size=(3, 9, 11), dtype=np.uint16)
    tm = rng.integers(0, 65536, size=(9, 11), dtype=np.uint16)
    assert np.array_equal(om.apply_shifts(f, np.zeros((3, 2), np.int32), tm), f)
    s = np.array([[1, 0], [0, -2], [3, 3]], np.int32)
    out = om.apply_shifts(f, s, tm)
    assert np.array_equal(out[0, :-1], f[0, 1:]) and np.array_equal(out[0, -1], tm[-1])
    assert np.array_equal(out[1, :, 2:], f[1, :, :-2]) and np.array_equal(out[1, :, :2], tm[:, :2])
    assert out[2, 0, 0] == f[2, 3, 3] and out[2, -1, -1] == tm[-1, -1]
    assert np.array_equal(out[2, :6, :8], f[2, 3:, 3:])
    assert np.array_equal(out[2, 6:], tm[6:]) and np.array_equal(out[2, :, 8:], tm[:, 8:])
    # brute force
    for t in range(3):
        for y in range(9):
            for x in range(11):
                sy, sx = y + s[t, 0], x + s[t, 1]
                want = f[t, sy, sx] if 0 <= sy < 9 and 0 <= sx < 11 else tm[y, x]
                assert out[t, y, x] == want
    # undoes planted motion away from the borders
    back = om.apply_shifts(move_frames(f, s), s, tm)
    assert np.array_equal(back[:, 3:-3, 3:-3], f[:, 3:-3, 3:-3])


def test_simulated_recording_motion_recovered():
    """A 256x256 recording of the benchmark kind with planted drift up to
    6 px: the oracle recovers every displacement."""
    video, _ = simulate(preset(2, frames=100), 5)
    moved, planted = plant_motion(video, 6, 2)
    corr, shifts, tmpl = om.correct(moved, R=8)
    assert np.array_equal(shifts, planted)
    assert np.array_equal(corr[:, 8:-8, 8:-8], video[:, 8:-8, 8:-8])
