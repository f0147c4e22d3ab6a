"""The FP64 surrogate reference: analytic gradients vs central differences,
and the parameter layout it shares with the library."""
import numpy as np
import pytest

from oracle import nn_ref


@pytest.fixture(scope="module")
def case():
    rng = np.random.default_rng(0)
    frames = rng.poisson(1000, size=(2, 50, 8, 8)).astype(np.uint16)
    frames[0, 20:22, 3:5, 3:5] += 300
    labels = (rng.random((2, 8, 8)) < 0.3).astype(np.float64)
    theta = nn_ref.init(1)
    theta += 0.01 * rng.standard_normal(theta.size)     # nonzero biases too
    loss, g = nn_ref.loss_and_grad(theta, frames, labels)
    return frames, labels, theta, loss, g


def _loss(theta, frames, labels):
    logit, _, _ = nn_ref.forward(theta, frames)
    return nn_ref.bce(logit, labels)[0]


def test_directional_derivatives(case):
    frames, labels, theta, loss, g = case
    rng = np.random.default_rng(2)
    for _ in range(3):
        v = rng.standard_normal(theta.size)
        v /= np.linalg.norm(v)
        h = 1e-6
        fd = (_loss(theta + h * v, frames, labels) - _loss(theta - h * v, frames, labels)) / (2 * h)
        assert abs(fd - g @ v) <= 1e-6 * max(1.0, abs(fd)), (fd, g @ v)


def test_coordinates_of_every_layer(case):
    frames, labels, theta, loss, g = case
    at = 0
    for name, r, c in nn_ref.LAYERS:
        idx = at + (r * c) // 3                       # one weight per layer
        e = np.zeros_like(theta)
        e[idx] = 1.0
        h = 1e-6
        fd = (_loss(theta + h * e, frames, labels) - _loss(theta - h * e, frames, labels)) / (2 * h)
        assert abs(fd - g[idx]) <= 1e-6 + 1e-4 * abs(fd), (name, fd, g[idx])
        at += r * c + nn_ref.bias_len(name, r)


def test_layout_matches_library():
    from paper_2403_16438_amd import surrogate
    assert surrogate.param_count() == nn_ref.n_params()
    at = 0
    for (name, r, c), (n2, r2, c2, wo, bo) in zip(nn_ref.LAYERS, surrogate.param_layout()):
        assert (name, r, c) == (n2, r2, c2) and wo == at and bo == at + r * c
        at += r * c + nn_ref.bias_len(name, r)


def test_bf16_rounding():
    x = np.array([1.0, 1.00390625, 1.005859375, 3.14159, -2.5e-3], np.float32)
    r = nn_ref.bf16_round(x)
    assert r[0] == 1.0 and r[1] == 1.0                 # tie to even
    assert r[2] == 1.0078125
    assert abs(r[3] - 3.140625) < 1e-12
