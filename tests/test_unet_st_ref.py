"""Pins of the summary-image U-Net reference (oracle/unet_st.py): analytic
gradients against central differences, and closed forms of the patch grid,
input normalisation and weighted merge."""
import numpy as np
import pytest

from oracle import unet_st


@pytest.fixture(scope="module")
def case():
    rng = np.random.default_rng(4)
    S = rng.uniform(800, 1200, size=(2, 8, 8))
    T = rng.uniform(0, 60, size=(2, 8, 8))
    T[0, 2:5, 3:6] += 200
    st = np.stack([S, T], axis=1)
    labels = (rng.random((2, 8, 8)) < 0.3).astype(np.float64)
    theta = unet_st.init(2)
    theta += 0.01 * rng.standard_normal(theta.size)
    loss, g = unet_st.loss_and_grad(theta, st, labels)
    return st, labels, theta, loss, g


def _loss(theta, st, labels):
    logit, _, _ = unet_st.forward(theta, st)
    from oracle import nn_ref
    return nn_ref.bce(logit, labels)[0]


def test_directional_derivatives(case):
    st, labels, theta, loss, g = case
    rng = np.random.default_rng(5)
    for _ in range(3):
        v = rng.standard_normal(theta.size)
        v /= np.linalg.norm(v)
        h = 1e-6
        fd = (_loss(theta + h * v, st, labels) - _loss(theta - h * v, st, labels)) / (2 * h)
        assert abs(fd - g @ v) <= 1e-6 * max(1.0, abs(fd)), (fd, g @ v)


def test_coordinates_of_every_layer(case):
    st, labels, theta, loss, g = case
    from oracle import nn_ref
    at = 0
    for name, r, c in unet_st.LAYERS:
        for idx in (at + (r * c) // 3, at + r * c):       # a weight and the first bias
            e = np.zeros_like(theta)
            e[idx] = 1.0
            h = 1e-6
            fd = (_loss(theta + h * e, st, labels) - _loss(theta - h * e, st, labels)) / (2 * h)
            assert abs(fd - g[idx]) <= 1e-6 + 1e-4 * abs(fd), (name, idx, fd, g[idx])
        at += r * c + nn_ref.bias_len(name, r)


def test_origins_and_patches():
    assert unet_st.origins(64) == [0]
    assert unet_st.origins(100) == [0, 32, 36]
    assert unet_st.origins(256) == [0, 32, 64, 96, 128, 160, 192]
    assert unet_st.origins(128) == [0, 32, 64]
    rng = np.random.default_rng(6)
    S, T = rng.random((100, 70)), rng.random((100, 70))
    p = unet_st.patches(S, T)
    assert p.shape == (3 * 2, 2, 64, 64)
    assert np.array_equal(p[0, 0], S[:64, :64]) and np.array_equal(p[1, 1], T[:64, 6:70])
    assert np.array_equal(p[5, 0], S[36:100, 6:70])


def test_normalisation_closed_forms():
    rng = np.random.default_rng(7)
    st = np.stack([rng.uniform(500, 1500, (3, 64, 64)), rng.uniform(0, 50, (3, 64, 64))], axis=1)
    x = unet_st.normalise(st)
    assert np.allclose(x[:, 0].mean(axis=(1, 2)), 0.0, atol=1e-12)
    assert np.allclose(x[:, 0].std(axis=(1, 2)), 1.0, atol=1e-12)
    assert np.allclose(x[:, 1], st[:, 1] / np.sqrt(st[:, 0] + 25.0), rtol=1e-15)
    flat = np.stack([np.full((1, 64, 64), 900.0), np.full((1, 64, 64), 30.0)], axis=1)
    y = unet_st.normalise(flat)
    assert np.array_equal(y[:, 0], np.zeros((1, 64, 64))) and np.allclose(y[:, 1], 30.0 / np.sqrt(925.0))


def test_merge_closed_forms():
    w = unet_st.tent()
    assert w.min() > 0 and np.allclose(w, w.T) and np.allclose(w, w[::-1, ::-1])
    assert abs(w[31, 31] - (1 - 0.5 / 32) ** 2) < 1e-15
    # constant probabilities merge to the constant
    n = len(unet_st.origins(100)) * len(unet_st.origins(150))
    assert np.allclose(unet_st.merge(np.full((n, 64, 64), 0.3), 100, 150), 0.3, rtol=0, atol=1e-15)
    # patches cut from one map merge back to that map
    rng = np.random.default_rng(8)
    m = rng.random((100, 150))
    cut = unet_st.patches(m, m)[:, 0]
    assert np.allclose(unet_st.merge(cut, 100, 150), m, rtol=0, atol=1e-14)
    # a pixel covered by one patch takes that patch's value
    prob = rng.random((n, 64, 64))
    out = unet_st.merge(prob, 100, 150)
    assert out[0, 0] == prob[0, 0, 0]
