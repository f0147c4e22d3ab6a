"""Closed forms of the network references' forward operators (oracle/nn_ref.py,
used by oracle/unet_st.py): each operator on inputs whose result can be
written down by hand, so a wrong stride, padding, weight layout or
normalisation fails here and not only as a gradient mismatch.

  * 3x3 convolution with a one-hot kernel = a shift with zero fill;
  * transposed 2x2 convolution with a one-hot weight row = a scatter into
    one of the four sub-grids;
  * temporal convolutions (kernel 5, strides 5, 2, 1, padding 0, 2, 0):
    50 -> 10 -> 5 -> 1 samples, a one-hot tap picks sample j s - p + k;
  * a hand-worked 2x2 max pool, with the first of equal maxima winning;
  * the per-pixel normalisation (V - mean) / sqrt(mean + 25) on hand values;
  * the BF16 numerics mode equals the exact one on operands that BF16
    represents exactly and sums FP32 holds exactly.
"""
import numpy as np
import pytest

from oracle import nn_ref, unet_st


def _onehot_conv3(co, ci, o, c, ky, kx):
    W = np.zeros((co, ci * 9))
    W[o, c * 9 + 3 * ky + kx] = 1.0
    return W


@pytest.mark.parametrize("ky,kx", [(0, 0), (1, 1), (2, 0), (0, 2), (1, 2)])
def test_conv3_one_hot_kernel_is_a_shift(ky, kx):
    rng = np.random.default_rng(ky * 3 + kx)
    x = rng.integers(-9, 10, size=(2, 3, 5, 7)).astype(np.float64)
    W = _onehot_conv3(4, 3, 2, 1, ky, kx)
    b = np.array([0.0, 0.0, 0.5, 0.0])
    y = nn_ref.conv3(x, W, b)
    want = np.zeros((2, 5, 7))
    for yy in range(5):
        for xx in range(7):
            sy, sx = yy + ky - 1, xx + kx - 1
            if 0 <= sy < 5 and 0 <= sx < 7:
                want[:, yy, xx] = x[:, 1, sy, sx]
    assert np.array_equal(y[:, 2], want + 0.5)
    assert np.array_equal(y[:, [0, 1, 3]], np.zeros((2, 3, 5, 7)))


def test_conv3_sums_channels_and_taps():
    """All-ones kernel on a constant input of value v over C channels: 9 C v
    inside, fewer taps at the borders (zero padding): 4 C v in a corner and
    6 C v along an edge."""
    C, v = 3, 2.0
    x = np.full((1, C, 4, 5), v)
    y = nn_ref.conv3(x, np.ones((1, C * 9)), np.zeros(1))[0, 0]
    assert y[1, 1] == 9 * C * v and y[0, 0] == 4 * C * v and y[0, 2] == 6 * C * v and y[2, 0] == 6 * C * v


@pytest.mark.parametrize("a,bb", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_transposed_conv_one_hot_row_is_a_scatter(a, bb):
    rng = np.random.default_rng(10 + 2 * a + bb)
    x = rng.integers(-5, 6, size=(2, 3, 4, 6)).astype(np.float64)
    Co, Ci = 2, 3
    W = np.zeros((Co * 4, Ci))
    W[1 * 4 + 2 * a + bb, 2] = 1.0                 # output channel 1 <- input channel 2
    y = nn_ref.up(x, W, np.zeros(Co))
    assert y.shape == (2, Co, 8, 12)
    want = np.zeros((2, 8, 12))
    want[:, a::2, bb::2] = x[:, 2]
    assert np.array_equal(y[:, 1], want)
    assert not y[:, 0].any()
    # the bias is per output channel, added to all four sub-grids
    yb = nn_ref.up(x, W, np.array([0.0, 1.5]))
    assert np.array_equal(yb[:, 1] - y[:, 1], np.full((2, 8, 12), 1.5))


@pytest.mark.parametrize("stride,pad,tin,tout", [(5, 0, 50, 10), (2, 2, 10, 5), (1, 0, 5, 1)])
def test_temporal_conv_strides(stride, pad, tin, tout):
    """A one-hot tap k picks input sample j stride - pad + k (zero outside);
    the three layers take 50 samples to 10, 5 and 1."""
    x = (np.arange(tin, dtype=np.float64) + 1.0)[None, None, :, None, None] * np.ones((1, 1, tin, 2, 3))
    for k in range(5):
        W = np.zeros((1, 5))
        W[0, k] = 1.0
        y = nn_ref.tconv(x, W, np.zeros(1), stride, pad, tout)
        assert y.shape == (1, 1, tout, 2, 3)
        for j in range(tout):
            t = j * stride - pad + k
            want = t + 1.0 if 0 <= t < tin else 0.0
            assert np.all(y[0, 0, j] == want), (k, j)
    # all taps: window sums of the ramp 1..tin
    y = nn_ref.tconv(x, np.ones((1, 5)), np.zeros(1), stride, pad, tout)
    for j in range(tout):
        ts = [j * stride - pad + k for k in range(5)]
        assert y[0, 0, j, 0, 0] == sum(t + 1.0 for t in ts if 0 <= t < tin)


def test_temporal_stack_collapses_50_frames():
    frames = np.full((1, 50, 4, 4), 1000, np.uint16)
    _, c, _ = nn_ref.forward(nn_ref.init(0), frames)
    assert c["a1"].shape[2] == 10 and c["a2"].shape[2] == 5 and c["a3"].shape == (1, 32, 4, 4)


def test_pool_hand_worked():
    x = np.array([[1, 2, 5, 3],
                  [4, 0, 1, 1],
                  [9, 9, 0, 0],
                  [2, 8, 0, 7]], np.float64)[None, None]
    y, arg = nn_ref.pool(x)
    assert np.array_equal(y[0, 0], [[4, 5], [9, 7]])
    assert np.array_equal(arg[0, 0], [[2, 0], [0, 3]])      # (1,0); (0,0); tie -> first; (1,1)
    d = nn_ref.pool_bwd(np.array([[[[1.0, 2.0], [3.0, 4.0]]]]), arg, x.shape)
    want = np.zeros((4, 4))
    want[1, 0], want[0, 2], want[2, 0], want[3, 3] = 1.0, 2.0, 3.0, 4.0
    assert np.array_equal(d[0, 0], want)


def test_frame_normalisation_hand_values():
    """(V - mean) / sqrt(mean + 25) per pixel over the 50 frames: a constant
    pixel gives 0; 49 frames of 975 and one of 1025 have mean 976, so the
    raised frame gives 49 / sqrt(1001) and the others -1 / sqrt(1001)."""
    f = np.full((1, 50, 2, 2), 975, np.uint16)
    f[0, 7, 1, 0] = 1025
    x = nn_ref.normalise(f)
    assert np.array_equal(x[0, :, 0, 0], np.zeros(50))
    assert abs(x[0, 7, 1, 0] - 49.0 / np.sqrt(1001.0)) < 1e-15
    assert np.allclose(np.delete(x[0, :, 1, 0], 7), -1.0 / np.sqrt(1001.0), rtol=0, atol=1e-15)


def test_bf16_mode_is_exact_on_representable_operands():
    """Small integers and halves are BF16 values and their FP32 sums are
    exact, so the BF16 numerics mode reproduces the exact one."""
    rng = np.random.default_rng(3)
    nm = nn_ref.Numerics(bf16=True)
    x = rng.integers(-8, 9, size=(2, 3, 6, 6)).astype(np.float64) / 2
    W = rng.integers(-4, 5, size=(5, 27)).astype(np.float64)
    b = rng.integers(-3, 4, size=5).astype(np.float64)
    assert np.array_equal(nn_ref.conv3(x, W, b, nm), nn_ref.conv3(x, W, b))
    Wu = rng.integers(-4, 5, size=(8, 3)).astype(np.float64)
    assert np.array_equal(nn_ref.up(x, Wu, b[:2], nm), nn_ref.up(x, Wu, b[:2]))
    dy = rng.integers(-4, 5, size=(2, 5, 6, 6)).astype(np.float64)
    for a, e in zip(nn_ref.conv3_bwd(x, W, dy, nm), nn_ref.conv3_bwd(x, W, dy)):
        assert np.array_equal(a, e)
    # and it does round where BF16 cannot represent an operand
    x2 = x + 1.0 / 1024
    assert not np.array_equal(nn_ref.conv3(x2, W, b, nm), nn_ref.conv3(x2, W, b))


def test_bf16_mode_rounds_operands_not_sums():
    """One product of two operands that BF16 rounds: the mode's result is the
    exact product of the rounded operands."""
    nm = nn_ref.Numerics(bf16=True)
    x = np.zeros((1, 1, 1, 1))
    x[0, 0, 0, 0] = 1.0 + 5.0 / 512                # BF16 (8 significant bits) -> 1 + 1/128
    W = np.zeros((1, 9))
    W[0, 4] = 3.0 + 5.0 / 512                      # -> 3 + 1/64
    y = nn_ref.conv3(x, W, np.zeros(1), nm)[0, 0, 0, 0]
    assert y == (1 + 1 / 128) * (3 + 1 / 64)       # exact in FP32 as well
    assert nn_ref.conv3(x, W, np.zeros(1))[0, 0, 0, 0] == (1 + 5 / 512) * (3 + 5 / 512)


def test_summary_unet_reference_uses_the_same_operators():
    """The summary U-Net's first layer is nn_ref's 3x3 convolution on the
    normalised two-channel patch."""
    rng = np.random.default_rng(9)
    st = np.stack([rng.uniform(800, 1200, (1, 8, 8)), rng.uniform(0, 50, (1, 8, 8))], axis=1)
    theta = unet_st.init(1)
    _, c, p = unet_st.forward(theta, st)
    e1a = np.maximum(nn_ref.conv3(unet_st.normalise(st), p["e1a.w"], p["e1a.b"]), 0.0)
    assert np.array_equal(c["e1a"], e1a)


def test_bf16_mode_normalisation_is_single_precision():
    """In the BF16 mode the normalisation is evaluated in FP32 (each operation
    rounded): on the hand values above it stays within a few FP32 ulps of the
    exact one and is itself representable in FP32."""
    f = np.full((1, 50, 2, 2), 975, np.uint16)
    f[0, 7, 1, 0] = 1025
    x = nn_ref.normalise(f, nn_ref.Numerics(bf16=True))
    assert np.array_equal(x, x.astype(np.float32).astype(np.float64))
    assert np.array_equal(x[0, :, 0, 0], np.zeros(50))
    assert abs(x[0, 7, 1, 0] - 49.0 / np.sqrt(1001.0)) < 4 * np.spacing(np.float32(1.55))
