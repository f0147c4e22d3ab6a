"""Pins of the oracle's segment summaries: Eq. 1 (S), Eq. 2 (T), the noise
scale D and the correlation image, against closed forms, brute force and
invariants."""
import numpy as np
import pytest
from scipy import integrate, special, stats

import oracle

L = 50


def const_video(values, H=6, W=7):
    """Spatially constant video: frame t equals values[t] everywhere."""
    v = np.asarray(values, dtype=np.uint16)
    return np.broadcast_to(v[:, None, None], (len(v), H, W)).copy()


def test_constant():
    r = oracle.summarize_segment(const_video([1234] * L))
    assert np.all(r["S"] == 1234.0)
    assert np.abs(r["T"]).max() < 1e-9
    assert np.abs(r["D"]).max() < 1e-9


def test_single_raised_frame():
    vals = [1000] * L
    vals[17] = 1000 + 80
    r = oracle.summarize_segment(const_video(vals))
    np.testing.assert_allclose(r["T"], 80.0, atol=1e-9)
    np.testing.assert_allclose(r["S"], 1000 + 80 / L, rtol=1e-15)
    assert np.abs(r["D"]).max() < 1e-9


def test_ramp_closed_form():
    k = 3
    r = oracle.summarize_segment(const_video([500 + k * t for t in range(1, L + 1)]))
    np.testing.assert_allclose(r["T"], 24.5 * k, atol=1e-8)
    np.testing.assert_allclose(r["D"], 6.25 * k, atol=1e-8)
    np.testing.assert_allclose(r["S"], 500 + k * 25.5, rtol=1e-15)


@pytest.mark.parametrize("m,expect", [(1, 40.0), (24, 40.0), (25, 20.0), (26, 0.0), (49, 0.0)])
def test_square_wave(m, expect):
    vals = [2000] * L
    for t in range(m):
        vals[(7 * t) % L] = 2040
    r = oracle.summarize_segment(const_video(vals))
    np.testing.assert_allclose(r["T"], expect, atol=1e-8)


def test_impulse_gives_kernel():
    H, W = 40, 40
    seg = np.full((L, H, W), 900, np.uint16)
    seg[9, 20, 20] += 500
    r = oracle.summarize_segment(seg)
    w = oracle.gaussian_weights(3.0, 12)
    np.testing.assert_allclose(r["T"][8:33, 8:33], 500 * np.outer(w, w), atol=1e-8)
    S = np.full((H, W), 900.0)
    S[20, 20] += 500 / L
    np.testing.assert_array_equal(r["S"], S)


def _brute_summary(seg):
    Lh, H, W = seg.shape
    w = oracle.gaussian_weights(3.0, 12)
    vb = np.zeros((Lh, H, W))
    for t in range(Lh):
        for y in range(H):
            for x in range(W):
                acc = 0.0
                for dy in range(-12, 13):
                    for dx in range(-12, 13):
                        acc += (w[dy + 12] * w[dx + 12] *
                                float(seg[t, oracle.reflect_index(y + dy, H), oracle.reflect_index(x + dx, W)]))
                vb[t, y, x] = acc
    T = np.zeros((H, W))
    D = np.zeros((H, W))
    S = np.zeros((H, W))
    for y in range(H):
        for x in range(W):
            vals = sorted(vb[:, y, x].tolist())
            med = 0.5 * (vals[Lh // 2 - 1] + vals[Lh // 2])
            T[y, x] = vals[-1] - med
            D[y, x] = sum(max(0.0, med - v) for v in vb[:, y, x]) / Lh
            S[y, x] = sum(int(v) for v in seg[:, y, x]) / Lh
    return S, T, D


@pytest.mark.parametrize("shape", [(L, 5, 4), (L, 7, 9)])
def test_brute_force_tiny(shape):
    rng = np.random.default_rng(5)
    seg = rng.poisson(1000, size=shape).astype(np.uint16)
    S, T, D = _brute_summary(seg)
    r = oracle.summarize_segment(seg)
    np.testing.assert_allclose(r["S"], S, rtol=1e-15)
    np.testing.assert_allclose(r["T"], T, rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(r["D"], D, rtol=1e-10, atol=1e-10)


def test_shift_invariance():
    rng = np.random.default_rng(6)
    seg = rng.poisson(800, size=(L, 12, 10)).astype(np.uint16)
    a = oracle.summarize_segment(seg)
    b = oracle.summarize_segment(seg + np.uint16(3000))
    np.testing.assert_allclose(a["T"], b["T"], atol=1e-9)
    np.testing.assert_allclose(a["D"], b["D"], atol=1e-9)
    np.testing.assert_allclose(b["S"] - a["S"], 3000.0, atol=1e-12)


def test_spike_robust_noise_scale():
    # raising values that sit above the median changes neither median nor D
    H, W = 3, 3
    rng = np.random.default_rng(7)
    vals = rng.permutation(np.arange(1000, 1000 + L)).astype(np.uint16)
    seg = const_video(vals, H, W)
    a = oracle.summarize_segment(seg)
    seg2 = seg.copy()
    top = np.argsort(vals)[-10:]
    seg2[top] += 300
    b = oracle.summarize_segment(seg2)
    np.testing.assert_allclose(a["med"], b["med"], atol=1e-9)
    np.testing.assert_allclose(a["D"], b["D"], atol=1e-9)
    np.testing.assert_allclose(b["T"] - a["T"], 300.0, atol=1e-8)


def _expected_normal_D(n):
    """E[(1/n) sum_t max(0, med - X_t)] for X iid N(0, 1), n even, from the
    expected order statistics E[X_(k)] (numerical integration)."""
    def ek(k):
        c = special.gammaln(n + 1) - special.gammaln(k) - special.gammaln(n - k + 1)
        f = lambda x: x * np.exp(c + (k - 1) * stats.norm.logcdf(x) +
                                 (n - k) * stats.norm.logsf(x) + stats.norm.logpdf(x))
        return integrate.quad(f, -12, 12, epsabs=1e-13)[0]
    half = n // 2
    return -sum(ek(k) for k in range(1, half + 1)) / n


def test_noise_scale_statistics():
    # with a near-delta kernel (sd 0.01) the smoothing is the identity, so for
    # iid N(0, s^2) noise E[sqrt(2 pi) D] = s sqrt(2 pi) E_D(50)
    s = 40.0
    rng = np.random.default_rng(8)
    noise = rng.standard_normal((L, 64, 64)) * s
    seg = np.rint(10000 + noise).astype(np.uint16)
    r = oracle.summarize_segment(seg, oracle.Params(sigma=0.01))
    est = np.sqrt(2 * np.pi) * r["D"]
    expect = s * np.sqrt(2 * np.pi) * _expected_normal_D(L)
    se = est.std() / np.sqrt(est.size)
    assert abs(est.mean() - expect) < 4 * se + 0.01
    assert 0.97 < expect / s < 0.995   # the finite-L bias (about 1.7% low)


def test_noise_scale_with_smoothing_gain():
    # with the sd-3 kernel, iid noise of sd s has smoothed sd s * sum_k w_k^2
    s = 50.0
    rng = np.random.default_rng(9)
    seg = np.rint(20000 + s * rng.standard_normal((L, 96, 96))).astype(np.uint16)
    r = oracle.summarize_segment(seg)
    w = oracle.gaussian_weights(3.0, 12)
    expect = s * (w * w).sum() * np.sqrt(2 * np.pi) * _expected_normal_D(L)
    est = np.sqrt(2 * np.pi) * r["D"][20:76, 20:76]
    assert abs(est.mean() / expect - 1.0) < 0.02


# ---------------------------------------------------------------- correlation

def test_correlation_rank1_positive():
    rng = np.random.default_rng(10)
    H, W = 7, 6
    a = rng.integers(500, 1500, size=(H, W))
    b = rng.integers(1, 4, size=(H, W))
    s = rng.integers(0, 200, size=2 * L)
    v = (a[None] + b[None] * s[:, None, None]).astype(np.uint16)
    C = oracle.segment_moments(v[:L]) + oracle.segment_moments(v[L:])
    np.testing.assert_allclose(oracle.correlation_image(C), 1.0, atol=1e-12)


def test_correlation_checkerboard_signs():
    # sign (-1)^(x+y): 4-neighbours anti-correlated, diagonals correlated
    H, W = 6, 5
    rng = np.random.default_rng(11)
    yy, xx = np.mgrid[0:H, 0:W]
    sgn = np.where((xx + yy) % 2 == 0, 1, -1)
    s = rng.integers(0, 100, size=L)
    v = (1000 + sgn[None] * s[:, None, None]).astype(np.uint16)
    R = oracle.correlation_image(oracle.segment_moments(v))
    np.testing.assert_allclose(R[1:-1, 1:-1], 0.0, atol=1e-12)
    np.testing.assert_allclose(R[0, 0], (-1 - 1 + 1) / 3.0, atol=1e-12)     # corner: 3 neighbours
    np.testing.assert_allclose(R[0, 2], (-1 - 1 - 1 + 1 + 1) / 5.0, atol=1e-12)  # edge: 5 neighbours


def test_correlation_pooling_removes_segment_offsets():
    rng = np.random.default_rng(12)
    base = rng.poisson(1000, size=(2 * L, 8, 8)).astype(np.int64)
    shifted = base.copy()
    shifted[L:] += 700          # a jump between segments
    Ca = oracle.segment_moments(base[:L].astype(np.uint16)) + oracle.segment_moments(base[L:].astype(np.uint16))
    Cb = oracle.segment_moments(shifted[:L].astype(np.uint16)) + oracle.segment_moments(shifted[L:].astype(np.uint16))
    np.testing.assert_allclose(Ca, Cb, rtol=1e-12, atol=1e-6)


def test_correlation_independent_noise_small():
    rng = np.random.default_rng(13)
    K = 8
    v = rng.poisson(1000, size=(K * L, 20, 20)).astype(np.uint16)
    C = sum(oracle.segment_moments(v[i * L:(i + 1) * L]) for i in range(K))
    R = oracle.correlation_image(C)
    assert np.abs(R).max() < 4.0 / np.sqrt(K * (L - 1))


def test_segment_moments_brute():
    rng = np.random.default_rng(14)
    seg = rng.poisson(100, size=(L, 4, 5)).astype(np.uint16)
    got = oracle.segment_moments(seg)
    m = seg.astype(np.float64).mean(axis=0)
    offs = [(0, 0), (0, 1), (1, 0), (1, 1), (1, -1)]
    for k, (dy, dx) in enumerate(offs):
        for y in range(4):
            for x in range(5):
                yy, xx = y + dy, x + dx
                if 0 <= yy < 4 and 0 <= xx < 5:
                    ref = sum((float(seg[t, y, x]) - m[y, x]) * (float(seg[t, yy, xx]) - m[yy, xx]) for t in range(L))
                else:
                    ref = 0.0
                assert abs(got[k, y, x] - ref) < 1e-8
