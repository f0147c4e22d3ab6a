"""Seeded voltage-imaging simulator (input generator only).

Photon rate at pixel x and frame t:

    lam(x, t) = flick(t) * [ B(x) * (1 + drift * t / T)
                 + sum_j g_j(x) * ( F_j * (1 + sub_j(t)) + dF_j * s_j(t) ) ]

* B(x)   smooth background: Gaussian blobs, optional vessel ridges and a
         linear spatial gradient, scaled to a mean level (~1000 counts).
* g_j    unit-peak (elliptical) Gaussian footprint of neuron j.
* F_j    resting fluorescence = amplitude_j * B(centre_j).
* sub_j  subthreshold sinusoid (relative amplitude, 1-5 Hz).
* s_j    spike train convolved with the kernel (1, 0.5): a spike at frame s
         adds 1 * dF_j at frame s and 0.5 * dF_j at frame s + 1.
* dF_j   dff_j * (B(c_j) + F_j) when dff is relative to the total baseline at
         the footprint centre ("total", the default), or dff_j * F_j when it
         is relative to the neuron's own fluorescence ("neuron", hard mode).

Observation: V = clip(round(Poisson(lam) + N(0, read_noise^2)), 0, 65535),
stored as uint16 [T][H][W] with W fastest.

Every random draw comes from numpy's PCG64 generator seeded with `seed`; frame
chunks use child generators spawned from one SeedSequence, so the video is
identical for any thread count.
"""
from __future__ import annotations

from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field, replace
import os

import numpy as np

CHUNK = 50  # frames per independently seeded chunk


@dataclass(frozen=True)
class SimConfig:
    height: int = 64
    width: int = 64
    frames: int = 1000
    fps: float = 500.0
    mean_level: float = 1000.0
    # background
    n_blobs: int = 1
    blob_sigma: tuple = (15.0, 25.0)
    blob_amp: tuple = (0.3, 0.6)
    n_vessels: tuple = (0, 0)
    vessel_gain: float = 0.2
    vessel_sigma: float = 1.0
    gradient: float = 0.0          # total relative change across the frame width
    drift: float = 0.0             # relative change over the whole video
    flicker: float = 0.0           # sd of the per-frame multiplicative flicker
    # neurons
    n_neurons: int = 4
    n_overlap: int = 0             # neurons placed 1-2 sigma from a partner
    sigma_range: tuple = (3.0, 3.0)
    elliptical: bool = False
    amp_range: tuple = (0.10, 0.10)
    rate_range: tuple = (10.0, 10.0)   # Hz
    dff_range: tuple = (0.15, 0.15)
    sub_amp: float = 0.0
    sub_freq: tuple = (1.0, 5.0)
    min_sep: float = 18.0          # centre distance for non-overlapping neurons
    edge_margin: float = 9.0
    spike_kernel: tuple = (1.0, 0.5)
    read_noise: float = 5.0
    dff_reference: str = "total"   # "total" or "neuron"


@dataclass
class Truth:
    centers: np.ndarray          # [N, 2] (x, y)
    sigmas: np.ndarray           # [N, 2]
    angles: np.ndarray           # [N]
    footprints: np.ndarray       # [N, H, W] float32, unit peak
    spikes: list                 # N arrays of spike frame indices
    amplitude: np.ndarray        # F_j
    dF: np.ndarray               # per-spike fluorescence change dF_j
    background: np.ndarray       # B(x) float64 [H, W]
    partner: np.ndarray          # index of the partner for overlap neurons, else -1
    cfg: SimConfig = field(default=None)

    def masks(self, level: float = 0.25) -> np.ndarray:
        """Binary footprint masks g_j >= level * peak, [N, H, W] bool."""
        return self.footprints >= level

    def segment_masks(self, seg_len: int, level: float = 0.25) -> np.ndarray:
        """[K, H, W] bool: union of masks of neurons spiking in segment i."""
        n_seg = self.cfg.frames // seg_len
        out = np.zeros((n_seg, self.cfg.height, self.cfg.width), bool)
        m = self.masks(level)
        for j, s in enumerate(self.spikes):
            for i in np.unique(np.asarray(s) // seg_len):
                if i < n_seg:
                    out[i] |= m[j]
        return out


def preset(n: int, **overrides) -> SimConfig:
    """The five workload shapes of the benchmark suite (1-based).

    1: 64x64x1000 at 500 fps, 4 round neurons, one background blob, 1% drift.
    2: 256x256x10000 at 741 fps, 30 elliptical neurons (6 overlapping), blobs
       and vessel ridges, dim amplitudes, subthreshold sinusoids.
    3: 512x512x20000 at 1000 fps, 120 neurons (36 touching or overlapping),
       5% spatial gradient and 0.5% per-frame flicker.
    4: 64x64x2000 training videos with config-2 parameter ranges.
    5: one streaming session of config-2 style (frame size set by the caller).
    """
    if n == 1:
        c = SimConfig()
        c = replace(c, drift=0.01)
    elif n in (2, 5):
        c = SimConfig(height=256, width=256, frames=10000, fps=741.0,
                      n_blobs=5, blob_sigma=(30.0, 80.0), blob_amp=(0.2, 0.6),
                      n_vessels=(3, 5), n_neurons=30, n_overlap=6,
                      sigma_range=(3.0, 6.0), elliptical=True,
                      amp_range=(0.03, 0.10), rate_range=(5.0, 20.0),
                      dff_range=(0.05, 0.15), sub_amp=0.01, min_sep=24.0,
                      edge_margin=12.0)
    elif n == 3:
        c = SimConfig(height=512, width=512, frames=20000, fps=1000.0,
                      n_blobs=12, blob_sigma=(30.0, 80.0), blob_amp=(0.2, 0.6),
                      n_vessels=(6, 10), gradient=0.05, flicker=0.005,
                      n_neurons=120, n_overlap=36, sigma_range=(3.0, 6.0),
                      elliptical=True, amp_range=(0.03, 0.10),
                      rate_range=(5.0, 20.0), dff_range=(0.05, 0.15),
                      sub_amp=0.01, min_sep=24.0, edge_margin=12.0)
    elif n == 4:
        c = SimConfig(height=64, width=64, frames=2000, fps=741.0,
                      n_blobs=2, blob_sigma=(15.0, 40.0), blob_amp=(0.2, 0.6),
                      n_vessels=(0, 2), n_neurons=4, n_overlap=1,
                      sigma_range=(3.0, 6.0), elliptical=True,
                      amp_range=(0.03, 0.10), rate_range=(5.0, 20.0),
                      dff_range=(0.05, 0.15), sub_amp=0.01, min_sep=20.0,
                      edge_margin=10.0)
    else:
        raise ValueError(f"no preset {n}")
    return replace(c, **overrides) if overrides else c


def _background(cfg: SimConfig, rng) -> np.ndarray:
    H, W = cfg.height, cfg.width
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    field_ = np.ones((H, W))
    for _ in range(cfg.n_blobs):
        cx, cy = rng.uniform(0, W), rng.uniform(0, H)
        s = rng.uniform(*cfg.blob_sigma)
        a = rng.uniform(*cfg.blob_amp)
        field_ += a * np.exp(-((xx - cx) ** 2 + (yy - cy) ** 2) / (2 * s * s))
    nv = int(rng.integers(cfg.n_vessels[0], cfg.n_vessels[1] + 1))
    for _ in range(nv):
        ang = rng.uniform(0, np.pi)
        px, py = rng.uniform(0, W), rng.uniform(0, H)
        dist = np.abs(-(xx - px) * np.sin(ang) + (yy - py) * np.cos(ang))
        field_ *= 1.0 + cfg.vessel_gain * np.exp(-dist ** 2 / (2 * cfg.vessel_sigma ** 2))
    if cfg.gradient:
        field_ *= 1.0 + cfg.gradient * (xx / max(W - 1, 1) - 0.5)
    return field_ * (cfg.mean_level / field_.mean())


def _place(cfg: SimConfig, rng, sig):
    """Centres: n_overlap neurons 1-2 sigma from a partner, the rest apart."""
    H, W = cfg.height, cfg.width
    N = cfg.n_neurons
    n_free = N - cfg.n_overlap
    m = cfg.edge_margin
    centers = np.zeros((N, 2))
    partner = -np.ones(N, dtype=np.int64)
    placed = 0
    tries = 0
    while placed < n_free:
        tries += 1
        if tries > 200000:
            raise RuntimeError("could not place neurons; frame too small")
        c = rng.uniform([m, m], [W - 1 - m, H - 1 - m])
        if placed and np.min(np.hypot(*(centers[:placed] - c).T)) < cfg.min_sep:
            continue
        centers[placed] = c
        placed += 1
    for j in range(n_free, N):
        for _ in range(100000):
            p = int(rng.integers(0, n_free))
            d = rng.uniform(1.0, 2.0) * max(sig[p].mean(), sig[j].mean())
            a = rng.uniform(0, 2 * np.pi)
            c = centers[p] + d * np.array([np.cos(a), np.sin(a)])
            if not (m <= c[0] <= W - 1 - m and m <= c[1] <= H - 1 - m):
                continue
            others = [k for k in range(j) if k != p]
            if others and np.min(np.hypot(*(centers[others] - c).T)) < d:
                continue
            centers[j] = c
            partner[j] = p
            break
        else:
            raise RuntimeError("could not place an overlapping neuron")
    return centers, partner


def draw(cfg: SimConfig, seed: int):
    """Scene parameters, activity traces, flicker and per-chunk seeds."""
    rng = np.random.default_rng(seed)
    H, W, T = cfg.height, cfg.width, cfg.frames
    B = _background(cfg, rng)
    N = cfg.n_neurons
    sig = rng.uniform(cfg.sigma_range[0], cfg.sigma_range[1], size=(N, 2))
    if not cfg.elliptical:
        sig[:, 1] = sig[:, 0]
    ang = rng.uniform(0, np.pi, size=N) if cfg.elliptical else np.zeros(N)
    centers, partner = _place(cfg, rng, sig)
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    fp = np.zeros((N, H, W), np.float32)
    for j in range(N):
        dx, dy = xx - centers[j, 0], yy - centers[j, 1]
        c, s = np.cos(ang[j]), np.sin(ang[j])
        u, v = c * dx + s * dy, -s * dx + c * dy
        fp[j] = np.exp(-0.5 * ((u / sig[j, 0]) ** 2 + (v / sig[j, 1]) ** 2))
    bc = np.array([B[int(round(cy)), int(round(cx))] for cx, cy in centers])
    amp = rng.uniform(*cfg.amp_range, size=N) * bc
    dff = rng.uniform(*cfg.dff_range, size=N)
    dF = dff * (bc + amp) if cfg.dff_reference == "total" else dff * amp
    rate = rng.uniform(*cfg.rate_range, size=N)
    spikes = [np.flatnonzero(rng.random(T) < r / cfg.fps) for r in rate]
    sub_f = rng.uniform(*cfg.sub_freq, size=N)
    sub_ph = rng.uniform(0, 2 * np.pi, size=N)
    flick = 1.0 + cfg.flicker * rng.standard_normal(T) if cfg.flicker else np.ones(T)
    # per-neuron temporal multiplier on g_j: F_j (1 + sub_j(t)) + dF_j s_j(t)
    t = np.arange(T)
    act = np.empty((N, T))
    for j in range(N):
        s = np.zeros(T)
        for k, kv in enumerate(cfg.spike_kernel):
            idx = spikes[j] + k
            idx = idx[idx < T]
            np.add.at(s, idx, kv)
        sub = cfg.sub_amp * np.sin(2 * np.pi * sub_f[j] * t / cfg.fps + sub_ph[j])
        act[j] = amp[j] * (1.0 + sub) + dF[j] * s
    truth = Truth(centers=centers, sigmas=sig, angles=ang, footprints=fp,
                  spikes=spikes, amplitude=amp, dF=dF, background=B,
                  partner=partner, cfg=cfg)
    chunk_seeds = np.random.SeedSequence([seed, 0x5EED]).spawn((T + CHUNK - 1) // CHUNK)
    return truth, act, flick, chunk_seeds


def _render_chunk(cfg, truth, act, flick, t0, t1, ss):
    rng = np.random.default_rng(ss)
    T = cfg.frames
    B = truth.background.ravel()
    fp = truth.footprints.reshape(len(truth.footprints), cfg.height * cfg.width).astype(np.float64)
    n = t1 - t0
    lam = np.empty((n, cfg.height * cfg.width))
    for k in range(n):
        t = t0 + k
        base = B * (1.0 + cfg.drift * t / T)
        lam[k] = flick[t] * (base + act[:, t] @ fp) if len(fp) else flick[t] * base
    np.maximum(lam, 0.0, out=lam)
    v = rng.poisson(lam).astype(np.float64)
    v += cfg.read_noise * rng.standard_normal(lam.shape)
    np.rint(v, out=v)
    np.clip(v, 0, 65535, out=v)
    return v.reshape(n, cfg.height, cfg.width).astype(np.uint16)


def simulate_frames(cfg: SimConfig, seed: int, t0: int, t1: int, bundle=None,
                    threads: int | None = None) -> np.ndarray:
    """Frames [t0, t1) of the video as uint16 [t1 - t0, H, W].

    t0 must be a multiple of the 50-frame chunk; `bundle` is the result of
    `draw(cfg, seed)` when the caller renders several ranges of one video."""
    if t0 % CHUNK:
        raise ValueError("t0 must be a multiple of 50")
    truth, act, flick, seeds = bundle or draw(cfg, seed)
    buf = np.empty((t1 - t0, cfg.height, cfg.width), np.uint16)
    jobs = [(c * CHUNK, min((c + 1) * CHUNK, t1), seeds[c])
            for c in range(t0 // CHUNK, (t1 + CHUNK - 1) // CHUNK)]

    def run(j):
        a, b, ss = j
        buf[a - t0:b - t0] = _render_chunk(cfg, truth, act, flick, a, b, ss)[:b - a]

    threads = threads or min(16, os.cpu_count() or 1)
    if threads > 1 and len(jobs) > 1:
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(run, jobs))
    else:
        for j in jobs:
            run(j)
    return buf


def simulate(cfg: SimConfig, seed: int, threads: int | None = None):
    """Whole video and its ground truth: (uint16 [T, H, W], Truth)."""
    bundle = draw(cfg, seed)
    video = simulate_frames(cfg, seed, 0, cfg.frames, bundle, threads)
    return video, bundle[0]


def session_mix(n_sessions: int = 16, seed: int = 5000, blocks: int = 20,
                block_frames: int = 500, mean_gap_s: float = 0.5):
    """Streaming-session schedule: list of dicts with frame size, fps,
    arrival time (Poisson arrivals) and the simulator config of each session.
    Neuron density is scaled by frame area relative to 256 x 256."""
    rng = np.random.default_rng(seed)
    sizes = [(128, 128), (256, 256), (512, 128), (512, 512)]
    t = 0.0
    out = []
    for s in range(n_sessions):
        h, w = sizes[int(rng.integers(0, len(sizes)))]
        fps = float(rng.uniform(500.0, 1000.0))
        scale = h * w / 65536.0
        n_neu = max(2, int(round(30 * scale)))
        n_ov = int(round(0.2 * n_neu))
        cfg = preset(5, height=h, width=w, frames=blocks * block_frames, fps=fps,
                     n_neurons=n_neu, n_overlap=n_ov,
                     n_blobs=max(1, int(round(5 * scale))))
        out.append(dict(session=s, seed=seed + s, height=h, width=w, fps=fps,
                        arrival=t, cfg=cfg, block_frames=block_frames,
                        blocks=blocks))
        t += float(rng.exponential(mean_gap_s))
    return out
