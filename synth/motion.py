"""Seeded rigid motion planted into a video (input generator).

The recording is still for its first `still` frames (the frames a template
is taken from), then drifts by integer steps of one pixel in y or x, with an
occasional jump to a random position within the bound: brain motion and
stage drift at imaging rates, reduced to rigid integer translations.

A frame moved by (dy, dx) shows at (y, x) what the still frame shows at
(y - dy, x - dx); pixels that enter from outside repeat the nearest edge.
"""
from __future__ import annotations

import numpy as np


def draw_motion(frames: int, max_px: int, seed: int, still: int = 50,
                step_prob: float = 0.05, jump_prob: float = 0.002) -> np.ndarray:
    """int32 [frames, 2] displacements (dy, dx), |dy|, |dx| <= max_px."""
    rng = np.random.default_rng(seed)
    out = np.zeros((frames, 2), np.int32)
    cur = np.zeros(2, np.int64)
    for t in range(still, frames):
        if rng.random() < jump_prob:
            cur = rng.integers(-max_px, max_px + 1, size=2)
        else:
            step = (rng.random(2) < step_prob) * rng.choice([-1, 1], size=2)
            cur = np.clip(cur + step, -max_px, max_px)
        out[t] = cur
    return out


def move_frames(video: np.ndarray, shifts: np.ndarray) -> np.ndarray:
    """Frames of `video` [T, H, W] displaced by `shifts` [T, 2] (edge repeat)."""
    T, H, W = video.shape
    out = np.empty_like(video)
    ys, xs = np.arange(H), np.arange(W)
    for t in range(T):
        dy, dx = int(shifts[t, 0]), int(shifts[t, 1])
        iy = np.clip(ys - dy, 0, H - 1)
        ix = np.clip(xs - dx, 0, W - 1)
        out[t] = video[t][iy][:, ix]
    return out


def plant_motion(video: np.ndarray, max_px: int, seed: int, still: int = 50):
    """(moved video, displacements) for a still video."""
    shifts = draw_motion(video.shape[0], max_px, seed, still)
    return move_frames(video, shifts), shifts
