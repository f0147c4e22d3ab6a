"""FP64 reference of the summary-image U-Net (test infrastructure).

The paper's spiking-pixel identifier (Sec. III-C) is a U-Net whose input is
a 64 x 64 patch of the segment's two summary images (S_i, T_i); over a whole
frame it runs on sliding patches whose outputs are merged by weighted
averaging. Layer sizes appear only in a figure, so the network here is the
depth-3 U-Net of oracle/nn_ref.py (32 / 64 / 128 channels) with a 2-channel
first convolution. Readings where the paper is silent:
  * input channel 0: S standardised over the patch, (S - mean) / sd (sd
    floored at 1e-3); channel 1: T / sqrt(S + 25) pixel by pixel (the
    shot-noise scale of the mean intensity);
  * patch origins every 32 pixels, the last one flush with the far edge;
  * merge weight of patch pixel (u, v): w(u) w(v), w(u) = 1 - |u - 31.5| / 32
    (a tent that is largest in the middle of the patch and positive at its
    border); a frame pixel's probability is the weighted mean over the
    patches that contain it.
Only the test suite uses this module; it shares no code with the GPU path.
"""
from __future__ import annotations

import numpy as np

from . import nn_ref

P = 64
STRIDE = 32

LAYERS = [("e1a", 32, 18), ("e1b", 32, 288), ("e2a", 64, 288), ("e2b", 64, 576),
          ("e3a", 128, 576), ("e3b", 128, 1152), ("u2", 256, 128),
          ("d2a", 64, 1152), ("d2b", 64, 576), ("u1", 128, 64),
          ("d1a", 32, 576), ("d1b", 32, 288), ("out", 1, 32)]


def n_params():
    return sum(r * c + nn_ref.bias_len(n, r) for n, r, c in LAYERS)


def unpack(theta):
    p, at = {}, 0
    for n, r, c in LAYERS:
        p[n + ".w"] = theta[at:at + r * c].reshape(r, c)
        at += r * c
        bl = nn_ref.bias_len(n, r)
        p[n + ".b"] = theta[at:at + bl]
        at += bl
    return p


def pack(grads):
    return np.concatenate([np.concatenate([grads[n + ".w"].ravel(), grads[n + ".b"].ravel()])
                           for n, _, _ in LAYERS])


def init(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    out = []
    for n, r, c in LAYERS:
        out.append(rng.standard_normal(r * c) * np.sqrt(2.0 / c) * scale)
        out.append(np.zeros(nn_ref.bias_len(n, r)))
    return np.concatenate(out)


def origins(n: int) -> list:
    """Patch origins along an axis of n >= 64 pixels."""
    o = list(range(0, n - P + 1, STRIDE))
    if o[-1] != n - P:
        o.append(n - P)
    return o


def patches(S: np.ndarray, T: np.ndarray) -> np.ndarray:
    """Raw summary patches [n_patch][2][64][64] in raster order of origins."""
    H, W = S.shape
    out = []
    for y in origins(H):
        for x in origins(W):
            out.append(np.stack([S[y:y + P, x:x + P], T[y:y + P, x:x + P]]))
    return np.array(out, np.float64)


def normalise(st: np.ndarray, nm=nn_ref.EXACT) -> np.ndarray:
    """[B][2][64][64] raw (S, T) -> network input."""
    s = st[:, 0].astype(np.float64)
    t = st[:, 1].astype(np.float64)
    m = s.mean(axis=(1, 2), keepdims=True)
    sd = np.maximum(s.std(axis=(1, 2), keepdims=True), 1e-3)
    return nm.s(np.stack([(s - m) / sd, t / np.sqrt(np.maximum(s, 0.0) + 25.0)], axis=1))


def tent() -> np.ndarray:
    u = np.arange(P, dtype=np.float64)
    w = 1.0 - np.abs(u - (P - 1) / 2.0) / (P / 2.0)
    return np.outer(w, w)


def merge(prob: np.ndarray, H: int, W: int) -> np.ndarray:
    """Weighted mean of patch probabilities [n_patch][64][64] over the frame."""
    num = np.zeros((H, W))
    den = np.zeros((H, W))
    w = tent()
    k = 0
    for y in origins(H):
        for x in origins(W):
            num[y:y + P, x:x + P] += w * prob[k]
            den[y:y + P, x:x + P] += w
            k += 1
    return num / den


def forward(theta, st, nm=nn_ref.EXACT):
    """Logits [B][64][64] of raw patches st [B][2][64][64], and the cache
    (nm: where the arithmetic rounds, see nn_ref.Numerics)."""
    p = unpack(np.asarray(theta, np.float64))
    c = {}
    c["x"] = normalise(st, nm)
    relu = lambda v: np.maximum(v, 0.0)
    c["e1a"] = relu(nn_ref.conv3(c["x"], p["e1a.w"], p["e1a.b"], nm))
    c["s1"] = relu(nn_ref.conv3(c["e1a"], p["e1b.w"], p["e1b.b"], nm))
    c["p1"], c["arg1"] = nn_ref.pool(c["s1"])
    c["e2a"] = relu(nn_ref.conv3(c["p1"], p["e2a.w"], p["e2a.b"], nm))
    c["s2"] = relu(nn_ref.conv3(c["e2a"], p["e2b.w"], p["e2b.b"], nm))
    c["p2"], c["arg2"] = nn_ref.pool(c["s2"])
    c["e3a"] = relu(nn_ref.conv3(c["p2"], p["e3a.w"], p["e3a.b"], nm))
    c["b3"] = relu(nn_ref.conv3(c["e3a"], p["e3b.w"], p["e3b.b"], nm))
    c["cat2"] = np.concatenate([nn_ref.up(c["b3"], p["u2.w"], p["u2.b"], nm), c["s2"]], axis=1)
    c["d2a"] = relu(nn_ref.conv3(c["cat2"], p["d2a.w"], p["d2a.b"], nm))
    c["d2"] = relu(nn_ref.conv3(c["d2a"], p["d2b.w"], p["d2b.b"], nm))
    c["cat1"] = np.concatenate([nn_ref.up(c["d2"], p["u1.w"], p["u1.b"], nm), c["s1"]], axis=1)
    c["d1a"] = relu(nn_ref.conv3(c["cat1"], p["d1a.w"], p["d1a.b"], nm))
    c["d1"] = relu(nn_ref.conv3(c["d1a"], p["d1b.w"], p["d1b.b"], nm))
    logit = nm.s(np.einsum("c,bcyx->byx", nm.q(p["out.w"][0]), nm.q(c["d1"])) + p["out.b"][0])
    return logit, c, p


def loss_and_grad(theta, st, labels, nm=nn_ref.EXACT):
    """Mean binary cross-entropy and its gradient with respect to theta."""
    logit, c, p = forward(theta, st, nm)
    loss, dl = nn_ref.bce(logit, labels.astype(np.float64), nm)
    g = {}
    g["out.w"] = nm.s(np.einsum("byx,bcyx->c", nm.q(dl), nm.q(c["d1"])))[None]
    g["out.b"] = nm.s(np.array([dl.sum()]))
    dd1 = nm.s(nm.q(p["out.w"][0])[None, :, None, None] * nm.q(dl)[:, None]) * (c["d1"] > 0)
    dd1a, g["d1b.w"], g["d1b.b"] = nn_ref.conv3_bwd(c["d1a"], p["d1b.w"], dd1, nm)
    dd1a = dd1a * (c["d1a"] > 0)
    dcat1, g["d1a.w"], g["d1a.b"] = nn_ref.conv3_bwd(c["cat1"], p["d1a.w"], dd1a, nm)
    dd2, g["u1.w"], g["u1.b"] = nn_ref.up_bwd(c["d2"], p["u1.w"], dcat1[:, :32], nm)
    ds1 = dcat1[:, 32:]
    dd2 = dd2 * (c["d2"] > 0)
    dd2a, g["d2b.w"], g["d2b.b"] = nn_ref.conv3_bwd(c["d2a"], p["d2b.w"], dd2, nm)
    dd2a = dd2a * (c["d2a"] > 0)
    dcat2, g["d2a.w"], g["d2a.b"] = nn_ref.conv3_bwd(c["cat2"], p["d2a.w"], dd2a, nm)
    db3, g["u2.w"], g["u2.b"] = nn_ref.up_bwd(c["b3"], p["u2.w"], dcat2[:, :64], nm)
    ds2 = dcat2[:, 64:]
    db3 = db3 * (c["b3"] > 0)
    de3a, g["e3b.w"], g["e3b.b"] = nn_ref.conv3_bwd(c["e3a"], p["e3b.w"], db3, nm)
    de3a = de3a * (c["e3a"] > 0)
    dp2, g["e3a.w"], g["e3a.b"] = nn_ref.conv3_bwd(c["p2"], p["e3a.w"], de3a, nm)
    ds2 = nm.s(ds2 + nn_ref.pool_bwd(dp2, c["arg2"], c["s2"].shape)) * (c["s2"] > 0)
    de2a, g["e2b.w"], g["e2b.b"] = nn_ref.conv3_bwd(c["e2a"], p["e2b.w"], ds2, nm)
    de2a = de2a * (c["e2a"] > 0)
    dp1, g["e2a.w"], g["e2a.b"] = nn_ref.conv3_bwd(c["p1"], p["e2a.w"], de2a, nm)
    ds1 = nm.s(ds1 + nn_ref.pool_bwd(dp1, c["arg1"], c["s1"].shape)) * (c["s1"] > 0)
    de1a, g["e1b.w"], g["e1b.b"] = nn_ref.conv3_bwd(c["e1a"], p["e1b.w"], ds1, nm)
    de1a = de1a * (c["e1a"] > 0)
    _, g["e1a.w"], g["e1a.b"] = nn_ref.conv3_bwd(c["x"], p["e1a.w"], de1a, nm)
    return loss, pack(g)
