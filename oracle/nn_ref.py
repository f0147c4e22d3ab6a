"""FP64 reference of the learned surrogate detector, forward and backward.

TEST INFRASTRUCTURE: used only to check the GPU network's gradients. Written
from the architecture description (the spiking-pixel identifier of Sec. III-C
with temporal convolutions in front of a depth-3 U-Net, binary cross-entropy
loss); it shares no code with the GPU kernels. Tensors are [batch][channel]
[row][col] (the GPU uses channel-major); the flat parameter vector follows the
layer order and shapes below, which is the interface both sides agree on.
"""
from __future__ import annotations

import numpy as np

# name, weight rows, weight cols; bias length = rows (rows / 4 for the
# transposed convolutions, whose rows are out_channel * 4 + 2a + b)
LAYERS = [("t1", 32, 5), ("t2", 32, 160), ("t3", 32, 160),
          ("e1a", 32, 288), ("e1b", 32, 288), ("e2a", 64, 288), ("e2b", 64, 576),
          ("e3a", 128, 576), ("e3b", 128, 1152), ("u2", 256, 128),
          ("d2a", 64, 1152), ("d2b", 64, 576), ("u1", 128, 64),
          ("d1a", 32, 576), ("d1b", 32, 288), ("out", 1, 32)]


def bias_len(name, rows):
    return rows // 4 if name in ("u2", "u1") else rows


def n_params():
    return sum(r * c + bias_len(n, r) for n, r, c in LAYERS)


def unpack(theta):
    p, at = {}, 0
    for n, r, c in LAYERS:
        p[n + ".w"] = theta[at:at + r * c].reshape(r, c)
        at += r * c
        bl = bias_len(n, r)
        p[n + ".b"] = theta[at:at + bl]
        at += bl
    return p


def pack(grads):
    return np.concatenate([np.concatenate([grads[n + ".w"].ravel(), grads[n + ".b"].ravel()])
                           for n, _, _ in LAYERS])


def init(seed, scale=1.0):
    """He-normal weights, zero biases."""
    rng = np.random.default_rng(seed)
    out = []
    for n, r, c in LAYERS:
        fan_in = c if n not in ("u2", "u1") else c
        out.append(rng.standard_normal(r * c) * np.sqrt(2.0 / fan_in) * scale)
        out.append(np.zeros(bias_len(n, r)))
    return np.concatenate(out)


# ---------------------------------------------------------------- numerics

def bf16_round(a):
    """Round float values to the nearest BF16 (ties to even), as float64."""
    u = np.asarray(a, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


class Numerics:
    """Where the arithmetic rounds.

    Numerics() is exact FP64 throughout. Numerics(bf16=True) rounds as a
    network with BF16 matrix products and FP32 storage does: both operands of
    every product (weights, activations, gradients) to BF16, and every
    stored activation, gradient and product result to FP32; sums stay FP64
    (the products' FP32 accumulation differs from that by rounding only)."""

    def __init__(self, bf16: bool = False):
        self.bf16 = bf16

    def q(self, a):
        """A product operand."""
        return bf16_round(a) if self.bf16 else a

    def s(self, a):
        """A stored tensor."""
        return np.asarray(a, np.float32).astype(np.float64) if self.bf16 else a


EXACT = Numerics()


# ---------------------------------------------------------------- ops

def normalise(frames, nm=EXACT):
    """(V - mean) / sqrt(mean + 25) per pixel over the segment's frames. In
    the BF16 mode each operation rounds to FP32 as a single-precision
    evaluation does: the integer sum (exact), mean = sum / T, the reciprocal
    root of mean + 25, then (V - mean) times it."""
    if nm.bf16:
        f32 = np.float32
        v = frames.astype(f32)
        m = (v.sum(axis=1, keepdims=True, dtype=np.float64).astype(f32) / f32(frames.shape[1])).astype(f32)
        inv = (f32(1.0) / np.sqrt(m + f32(25.0))).astype(f32)
        return ((v - m) * inv).astype(f32).astype(np.float64)
    v = frames.astype(np.float64)                    # [B][T][H][W]
    m = v.mean(axis=1, keepdims=True)
    return (v - m) / np.sqrt(m + 25.0)


def tconv(x, W, b, stride, pad, tout, nm=EXACT):
    """x [B][Ci][Tin][H][W] -> [B][Co][tout][H][W], kernel 5: output sample j
    reads input samples j * stride - pad .. j * stride - pad + 4 (zero
    outside)."""
    B, Ci, Tin, H, Wd = x.shape
    Co = W.shape[0]
    Wk = nm.q(W.reshape(Co, Ci, 5))
    xp = np.zeros((B, Ci, Tin + 2 * pad + 5, H, Wd))
    xp[:, :, pad:pad + Tin] = nm.q(x)
    y = np.zeros((B, Co, tout, H, Wd))
    for j in range(tout):
        seg = xp[:, :, j * stride:j * stride + 5]          # [B][Ci][5][H][W]
        y[:, :, j] = np.einsum("ock,bckyx->boyx", Wk, seg)
    return nm.s(y + b[None, :, None, None, None])


def tconv_bwd(x, W, dy, stride, pad, nm=EXACT):
    B, Ci, Tin, H, Wd = x.shape
    Co, tout = dy.shape[1], dy.shape[2]
    Wk = nm.q(W.reshape(Co, Ci, 5))
    xp = np.zeros((B, Ci, Tin + 2 * pad + 5, H, Wd))
    xp[:, :, pad:pad + Tin] = nm.q(x)
    dq = nm.q(dy)
    dxp = np.zeros_like(xp)
    dW = np.zeros_like(Wk)
    for j in range(tout):
        seg = xp[:, :, j * stride:j * stride + 5]
        dW += np.einsum("boyx,bckyx->ock", dq[:, :, j], seg)
        dxp[:, :, j * stride:j * stride + 5] += nm.s(np.einsum("ock,boyx->bckyx", Wk, dq[:, :, j]))
    return (nm.s(dxp[:, :, pad:pad + Tin]), nm.s(dW.reshape(Co, Ci * 5)),
            nm.s(dy.sum(axis=(0, 2, 3, 4))))


def _cols3(x):
    B, C, H, W = x.shape
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1)))
    cols = np.empty((B, C, 9, H, W))
    for ky in range(3):
        for kx in range(3):
            cols[:, :, ky * 3 + kx] = xp[:, :, ky:ky + H, kx:kx + W]
    return cols.reshape(B, C * 9, H, W)


def conv3(x, W, b, nm=EXACT):
    """3x3 convolution, zero padding 1: W [Co][Ci * 9], column ci * 9 + 3 ky + kx
    weighs input (ci, y + ky - 1, x + kx - 1)."""
    return nm.s(np.einsum("ok,bkyx->boyx", nm.q(W), nm.q(_cols3(x))) + b[None, :, None, None])


def conv3_bwd(x, W, dy, nm=EXACT):
    B, C, H, Wd = x.shape
    cols = nm.q(_cols3(x))
    dq = nm.q(dy)
    dW = np.einsum("boyx,bkyx->ok", dq, cols)
    dcols = nm.s(np.einsum("ok,boyx->bkyx", nm.q(W), dq)).reshape(B, C, 9, H, Wd)
    dxp = np.zeros((B, C, H + 2, Wd + 2))
    for ky in range(3):
        for kx in range(3):
            dxp[:, :, ky:ky + H, kx:kx + Wd] += dcols[:, :, ky * 3 + kx]
    return nm.s(dxp[:, :, 1:H + 1, 1:Wd + 1]), nm.s(dW), nm.s(dy.sum(axis=(0, 2, 3)))


def pool(x):
    """2x2 max pool; argmax order (0,0), (0,1), (1,0), (1,1), first wins."""
    B, C, H, W = x.shape
    q = np.stack([x[:, :, 0::2, 0::2], x[:, :, 0::2, 1::2], x[:, :, 1::2, 0::2], x[:, :, 1::2, 1::2]])
    a = np.argmax(q, axis=0)
    return np.take_along_axis(q, a[None], 0)[0], a


def pool_bwd(dy, a, shape):
    dx = np.zeros(shape)
    for k, (oy, ox) in enumerate([(0, 0), (0, 1), (1, 0), (1, 1)]):
        dx[:, :, oy::2, ox::2] = np.where(a == k, dy, 0.0)
    return dx


def up(x, W, b, nm=EXACT):
    """2x2 stride-2 transposed convolution; W rows = co * 4 + 2a + bb: input
    pixel (y, x) writes output pixel (2y + a, 2x + bb) of channel co."""
    B, Ci, h, w = x.shape
    Co = W.shape[0] // 4
    z = np.einsum("rc,bcyx->bryx", nm.q(W), nm.q(x)).reshape(B, Co, 2, 2, h, w)
    y = np.zeros((B, Co, 2 * h, 2 * w))
    for a in range(2):
        for bb in range(2):
            y[:, :, a::2, bb::2] = z[:, :, a, bb]
    return nm.s(y + b[None, :, None, None])


def up_bwd(x, W, dy, nm=EXACT):
    B, Ci, h, w = x.shape
    Co = W.shape[0] // 4
    dz = np.zeros((B, Co, 2, 2, h, w))
    for a in range(2):
        for bb in range(2):
            dz[:, :, a, bb] = dy[:, :, a::2, bb::2]
    dz = nm.q(dz.reshape(B, 4 * Co, h, w))
    return (nm.s(np.einsum("rc,bryx->bcyx", nm.q(W), dz)), nm.s(np.einsum("bryx,bcyx->rc", dz, nm.q(x))),
            nm.s(dy.sum(axis=(0, 2, 3))))


relu = lambda v: np.maximum(v, 0.0)


def forward(theta, frames, nm=EXACT):
    """Logits [B][H][W] and the cache for backward (nm: where it rounds)."""
    p = unpack(np.asarray(theta, np.float64))
    c = {}
    x = normalise(frames, nm)[:, None]                        # [B][1][50][H][W]
    c["x"] = x
    c["a1"] = relu(tconv(x, p["t1.w"], p["t1.b"], 5, 0, 10, nm))
    c["a2"] = relu(tconv(c["a1"], p["t2.w"], p["t2.b"], 2, 2, 5, nm))
    c["a3"] = relu(tconv(c["a2"], p["t3.w"], p["t3.b"], 1, 0, 1, nm))[:, :, 0]
    c["e1a"] = relu(conv3(c["a3"], p["e1a.w"], p["e1a.b"], nm))
    c["s1"] = relu(conv3(c["e1a"], p["e1b.w"], p["e1b.b"], nm))
    c["p1"], c["arg1"] = pool(c["s1"])
    c["e2a"] = relu(conv3(c["p1"], p["e2a.w"], p["e2a.b"], nm))
    c["s2"] = relu(conv3(c["e2a"], p["e2b.w"], p["e2b.b"], nm))
    c["p2"], c["arg2"] = pool(c["s2"])
    c["e3a"] = relu(conv3(c["p2"], p["e3a.w"], p["e3a.b"], nm))
    c["b3"] = relu(conv3(c["e3a"], p["e3b.w"], p["e3b.b"], nm))
    c["cat2"] = np.concatenate([up(c["b3"], p["u2.w"], p["u2.b"], nm), c["s2"]], axis=1)
    c["d2a"] = relu(conv3(c["cat2"], p["d2a.w"], p["d2a.b"], nm))
    c["d2"] = relu(conv3(c["d2a"], p["d2b.w"], p["d2b.b"], nm))
    c["cat1"] = np.concatenate([up(c["d2"], p["u1.w"], p["u1.b"], nm), c["s1"]], axis=1)
    c["d1a"] = relu(conv3(c["cat1"], p["d1a.w"], p["d1a.b"], nm))
    c["d1"] = relu(conv3(c["d1a"], p["d1b.w"], p["d1b.b"], nm))
    logit = nm.s(np.einsum("c,bcyx->byx", nm.q(p["out.w"][0]), nm.q(c["d1"])) + p["out.b"][0])
    return logit, c, p


def bce(logit, y, nm=EXACT):
    """mean of max(z, 0) - z y + log(1 + exp(-|z|)) and its gradient."""
    n = logit.size
    loss = (np.maximum(logit, 0) - logit * y + np.log1p(np.exp(-np.abs(logit)))).sum() / n
    return loss, nm.s((1.0 / (1.0 + np.exp(-logit)) - y) / n)


def loss_and_grad(theta, frames, labels, nm=EXACT):
    logit, c, p = forward(theta, frames, nm)
    loss, dl = bce(logit, labels.astype(np.float64), nm)
    g = {}
    g["out.w"] = nm.s(np.einsum("byx,bcyx->c", nm.q(dl), nm.q(c["d1"])))[None]
    g["out.b"] = nm.s(np.array([dl.sum()]))
    dd1 = nm.s(nm.q(p["out.w"][0])[None, :, None, None] * nm.q(dl)[:, None])
    dd1 = dd1 * (c["d1"] > 0)
    dd1a, g["d1b.w"], g["d1b.b"] = conv3_bwd(c["d1a"], p["d1b.w"], dd1, nm)
    dd1a = dd1a * (c["d1a"] > 0)
    dcat1, g["d1a.w"], g["d1a.b"] = conv3_bwd(c["cat1"], p["d1a.w"], dd1a, nm)
    dd2, g["u1.w"], g["u1.b"] = up_bwd(c["d2"], p["u1.w"], dcat1[:, :32], nm)
    ds1 = dcat1[:, 32:]
    dd2 = dd2 * (c["d2"] > 0)
    dd2a, g["d2b.w"], g["d2b.b"] = conv3_bwd(c["d2a"], p["d2b.w"], dd2, nm)
    dd2a = dd2a * (c["d2a"] > 0)
    dcat2, g["d2a.w"], g["d2a.b"] = conv3_bwd(c["cat2"], p["d2a.w"], dd2a, nm)
    db3, g["u2.w"], g["u2.b"] = up_bwd(c["b3"], p["u2.w"], dcat2[:, :64], nm)
    ds2 = dcat2[:, 64:]
    db3 = db3 * (c["b3"] > 0)
    de3a, g["e3b.w"], g["e3b.b"] = conv3_bwd(c["e3a"], p["e3b.w"], db3, nm)
    de3a = de3a * (c["e3a"] > 0)
    dp2, g["e3a.w"], g["e3a.b"] = conv3_bwd(c["p2"], p["e3a.w"], de3a, nm)
    ds2 = nm.s(ds2 + pool_bwd(dp2, c["arg2"], c["s2"].shape)) * (c["s2"] > 0)
    de2a, g["e2b.w"], g["e2b.b"] = conv3_bwd(c["e2a"], p["e2b.w"], ds2, nm)
    de2a = de2a * (c["e2a"] > 0)
    dp1, g["e2a.w"], g["e2a.b"] = conv3_bwd(c["p1"], p["e2a.w"], de2a, nm)
    ds1 = nm.s(ds1 + pool_bwd(dp1, c["arg1"], c["s1"].shape)) * (c["s1"] > 0)
    de1a, g["e1b.w"], g["e1b.b"] = conv3_bwd(c["e1a"], p["e1b.w"], ds1, nm)
    de1a = de1a * (c["e1a"] > 0)
    da3, g["e1a.w"], g["e1a.b"] = conv3_bwd(c["a3"], p["e1a.w"], de1a, nm)
    da3 = (da3 * (c["a3"] > 0))[:, :, None]
    da2, g["t3.w"], g["t3.b"] = tconv_bwd(c["a2"], p["t3.w"], da3, 1, 0, nm)
    da2 = da2 * (c["a2"] > 0)
    da1, g["t2.w"], g["t2.b"] = tconv_bwd(c["a1"], p["t2.w"], da2, 2, 2, nm)
    da1 = da1 * (c["a1"] > 0)
    _, g["t1.w"], g["t1.b"] = tconv_bwd(c["x"], p["t1.w"], da1, 5, 0, nm)
    return loss, pack(g)

