"""Voltage trace extraction (test infrastructure: FP64 CPU oracle).

The paper's third stage takes, for every detected neuron, the mean pixel
intensity inside its region of interest in each frame of the (motion
corrected) video (Sec. II). Here the region of interest of a footprint is its
mask (footprint >= 0.25 of its peak, Sec. III-D reading).

trace_j(t) = (1 / |R_j|) * sum_{x in R_j} V(x, t)

The sum over the mask is exact in integers (uint16 pixels), the division is
one FP64 operation; the result is rounded to FP32 for comparison with the GPU,
which stores FP32 traces.
"""
from __future__ import annotations

import numpy as np


def extract_traces(video: np.ndarray, masks: np.ndarray) -> np.ndarray:
    """video uint16 [T, H, W], masks bool [N, H, W] -> FP64 traces [N, T]."""
    T = video.shape[0]
    flat = video.reshape(T, -1)
    out = np.zeros((masks.shape[0], T))
    for j, m in enumerate(masks.reshape(masks.shape[0], -1)):
        idx = np.flatnonzero(m)
        if len(idx) == 0:
            continue
        out[j] = flat[:, idx].astype(np.int64).sum(axis=1) / float(len(idx))
    return out
