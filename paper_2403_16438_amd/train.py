"""Training of the surrogate detector on simulated segments (Sec. III-C trains
its U-Net on synthetic videos with binary cross-entropy and RMSProp).

A training example is one 50-frame segment of a 64 x 64 video drawn from the
simulator's config-4 scenes (2,000 frames each, 1-3 neurons... see
synth.preset(4)); its label is the ground-truth mask of the neurons that spike
in that segment (footprint >= 0.25 of peak). Frames are rendered on the GPU
from the scene (synth.gpu); the forward, loss, backward and RMSProp update run
in libseg.so.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from .surrogate import Surrogate, he_init

SEG = 50


class SceneBank:
    """n simulated training videos (config 4: 64x64x2000) on the GPU; the
    spike amplitudes alternate between the two dF/F references of the
    simulator (relative to the local total fluorescence, and the dimmer one
    relative to the neuron's own), so that the network sees events on both
    sides of the plain method's threshold."""

    def __init__(self, n: int, seed0: int = 40000, device="cuda", mixed: bool = True, **overrides):
        from synth import preset
        from synth.gpu import GpuScene
        self.scenes = []
        self.labels = []
        for k in range(n):
            mode = {"dff_reference": "neuron" if mixed and k % 2 else "total"}
            cfg = preset(4, **dict(mode, **overrides))
            sc = GpuScene(cfg, seed0 + k, device)
            self.scenes.append(sc)
            self.labels.append(torch.from_numpy(sc.truth.segment_masks(SEG).astype(np.float32)).to(device))
        self.K = self.scenes[0].cfg.frames // SEG
        self.H, self.W = self.scenes[0].cfg.height, self.scenes[0].cfg.width
        self.device = torch.device(device)

    def batch(self, rng, B):
        frames = torch.empty((B, SEG, self.H, self.W), dtype=torch.int16, device=self.device)
        labels = torch.empty((B, self.H, self.W), dtype=torch.float32, device=self.device)
        for b in range(B):
            k = int(rng.integers(len(self.scenes)))
            i = int(rng.integers(self.K))
            self.scenes[k].render(i * SEG, (i + 1) * SEG, out=frames[b])
            labels[b] = self.labels[k][i]
        return frames, labels


def train(steps: int = 400, batch: int = 16, lr: float = 1e-3, n_videos: int = 200, seed: int = 0,
          device="cuda", log=None, bank: SceneBank | None = None):
    """Train a fresh surrogate; returns (Surrogate, losses)."""
    bank = bank or SceneBank(n_videos, device=device)
    net = Surrogate(batch, bank.H, bank.W, he_init(seed), device)
    rng = np.random.default_rng(seed)
    losses = []
    t0 = time.time()
    for s in range(steps):
        frames, labels = bank.batch(rng, batch)
        loss, _ = net.backward(frames, labels)
        net.step(lr=lr)
        losses.append(loss)
        if log and (s % 50 == 0 or s == steps - 1):
            log(f"step {s} loss {loss:.4f} ({time.time() - t0:.1f}s)")
    return net, losses


def for_frames(net: Surrogate, height: int, width: int, device="cuda") -> Surrogate:
    """A batch-1 network for other frame sizes with the same weights."""
    return Surrogate(1, height, width, net.theta(), device)


# ---- the paper's input: summary-image patches --------------------------------

class SummaryBank:
    """Summary pairs (S_i, T_i) of n simulated 128 x 128 x 1,000 videos (the
    training videos of Sec. III-C: 20 pairs each), computed on the GPU by a
    plain session, with the mask of the neurons spiking in each segment as
    the label. Training patches are random 64 x 64 crops of the pairs."""

    def __init__(self, n: int, seed0: int = 60000, device="cuda", **overrides):
        from synth import preset
        from synth.gpu import GpuScene
        from . import abi
        from .session import Session
        self.device = torch.device(device)
        cfg0 = preset(4, **dict(dict(height=128, width=128, frames=1000, n_neurons=8, n_overlap=2,
                                     edge_margin=10.0), **overrides))
        self.H, self.W = cfg0.height, cfg0.width
        K = cfg0.frames // SEG
        self.S = torch.empty((n * K, self.H, self.W), dtype=torch.float32, device=self.device)
        self.T = torch.empty_like(self.S)
        self.Y = torch.empty_like(self.S)
        for k in range(n):
            cfg = preset(4, **dict(dict(height=128, width=128, frames=1000, n_neurons=8, n_overlap=2,
                                        edge_margin=10.0,
                                        dff_reference="neuron" if k % 2 else "total"), **overrides))
            sc = GpuScene(cfg, seed0 + k, self.device)
            sess = Session(self.H, self.W, cfg.frames, self.device)
            sess.push(sc.render(0, cfg.frames))
            self.S[k * K:(k + 1) * K] = sess.segment_maps(abi.SEG_MAP_S)
            self.T[k * K:(k + 1) * K] = sess.segment_maps(abi.SEG_MAP_T)
            self.Y[k * K:(k + 1) * K] = torch.from_numpy(sc.truth.segment_masks(SEG).astype(np.float32))
            sess.close()

    def batch(self, rng, B):
        st = torch.empty((B, 2, 64, 64), dtype=torch.float32, device=self.device)
        y = torch.empty((B, 64, 64), dtype=torch.float32, device=self.device)
        for b in range(B):
            i = int(rng.integers(self.S.shape[0]))
            oy, ox = int(rng.integers(self.H - 63)), int(rng.integers(self.W - 63))
            st[b, 0] = self.S[i, oy:oy + 64, ox:ox + 64]
            st[b, 1] = self.T[i, oy:oy + 64, ox:ox + 64]
            y[b] = self.Y[i, oy:oy + 64, ox:ox + 64]
        return st, y


def train_unet(steps: int = 2000, batch: int = 32, lr: float = 1e-3, n_videos: int = 100, seed: int = 0,
               device="cuda", log=None, bank: SummaryBank | None = None):
    """Train a fresh summary-image U-Net; returns (SummaryUNet, losses)."""
    from .unet import SummaryUNet, he_init as st_init
    bank = bank or SummaryBank(n_videos, device=device)
    net = SummaryUNet(batch, 64, 64, st_init(seed), device)
    rng = np.random.default_rng(seed)
    losses = []
    t0 = time.time()
    for s in range(steps):
        st, y = bank.batch(rng, batch)
        loss, _ = net.backward(st, y)
        net.step(lr=lr)
        losses.append(loss)
        if log and (s % 100 == 0 or s == steps - 1):
            log(f"step {s} loss {loss:.4f} ({time.time() - t0:.1f}s)")
    return net, losses
