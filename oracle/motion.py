"""Rigid motion correction by patch-wise ZNCC (test infrastructure: FP64 CPU oracle).

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark use this module; the GPU library shares no code with it.

The paper's first stage (Sec. II) measures the similarity of two images by
their zero-mean normalised cross-correlation (ZNCC). Patches of 21 x 21
pixels tile the image; ZNCC is evaluated for every patch and every candidate
motion vector, and the patch values are then aggregated into the single most
likely motion vector of the frame.

Readings where the paper is silent:
  * template: the per-pixel mean of the first 50 frames (one segment),
    rounded half up to an integer;
  * candidate vectors: every integer d = (dy, dx) with |dy|, |dx| <= R
    (R = 8), ordered by dy, then dx;
  * patch grid: (H - 2R) // 21 rows and (W - 2R) // 21 columns of tiles,
    centred in the frame minus an R-pixel margin, so that every shifted
    template window lies inside the frame;
  * ZNCC of the frame's patch at tile origin p with the template's window at
    p + d, and 0 where either has zero variance;
  * aggregation: the sum over patches in raster order of the tiles; the
    vector with the largest sum wins, ties going to the first in order;
  * the reported motion is m = -d, the displacement of the frame's content
    relative to the template; the corrected frame is
    C(y, x) = F(y + my, x + mx) where that pixel lies in the frame, and the
    template's T(y, x) where it does not (no measurement exists there, and a
    repeated edge would vary with the motion like activity).
"""
from __future__ import annotations

import numpy as np
from numpy.lib.stride_tricks import sliding_window_view

PATCH = 21
TEMPLATE_FRAMES = 50


def make_template(frames: np.ndarray) -> np.ndarray:
    """uint16 [n, H, W] -> uint16 [H, W]: mean rounded half up."""
    n = frames.shape[0]
    s = frames.astype(np.int64).sum(axis=0)
    return ((s + n // 2) // n).astype(np.uint16)


def patch_grid(H: int, W: int, R: int, patch: int = PATCH) -> list:
    """Tile origins (y, x) in raster order."""
    ny, nx = (H - 2 * R) // patch, (W - 2 * R) // patch
    oy = R + ((H - 2 * R) - patch * ny) // 2
    ox = R + ((W - 2 * R) - patch * nx) // 2
    return [(oy + patch * i, ox + patch * j) for i in range(ny) for j in range(nx)]


def vectors(R: int) -> list:
    return [(dy, dx) for dy in range(-R, R + 1) for dx in range(-R, R + 1)]


def zncc(a: np.ndarray, b: np.ndarray) -> float:
    """Zero-mean normalised cross-correlation of two equal-size arrays."""
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    a = a - a.mean()
    b = b - b.mean()
    den = np.sqrt((a * a).sum() * (b * b).sum())
    return 0.0 if den == 0.0 else float((a * b).sum() / den)


def zncc_table(frame: np.ndarray, tmpl: np.ndarray, R: int, patch: int = PATCH) -> np.ndarray:
    """[P, V] ZNCC of every patch (raster order) with every shifted template window."""
    H, W = frame.shape
    grid = patch_grid(H, W, R, patch)
    V = (2 * R + 1) ** 2
    out = np.zeros((len(grid), V))
    t64 = tmpl.astype(np.float64)
    for k, (y, x) in enumerate(grid):
        f = frame[y:y + patch, x:x + patch].astype(np.float64).ravel()
        f = f - f.mean()
        # windows[dy + R, dx + R] is the template at (y + dy, x + dx)
        region = t64[y - R:y + R + patch, x - R:x + R + patch]
        win = sliding_window_view(region, (patch, patch)).reshape(V, patch * patch)
        win = win - win.mean(axis=1, keepdims=True)
        num = win @ f
        den = np.sqrt((win * win).sum(axis=1) * (f * f).sum())
        out[k] = np.where(den == 0.0, 0.0, num / np.where(den == 0.0, 1.0, den))
    return out


def scores(frame: np.ndarray, tmpl: np.ndarray, R: int) -> np.ndarray:
    """[V] per-vector sum of the patch ZNCCs, summed in patch order."""
    z = zncc_table(frame, tmpl, R)
    s = np.zeros(z.shape[1])
    for row in z:
        s = s + row
    return s


def estimate(frames: np.ndarray, tmpl: np.ndarray, R: int):
    """Motion (my, mx) per frame, int32 [n, 2], and the scores [n, V]."""
    vec = vectors(R)
    n = frames.shape[0]
    shifts = np.zeros((n, 2), np.int32)
    sc = np.zeros((n, len(vec)))
    for t in range(n):
        sc[t] = scores(frames[t], tmpl, R)
        dy, dx = vec[int(np.argmax(sc[t]))]          # first maximum wins ties
        shifts[t] = (-dy, -dx)
    return shifts, sc


def apply_shifts(frames: np.ndarray, shifts: np.ndarray, tmpl: np.ndarray) -> np.ndarray:
    """C_t(y, x) = F_t(y + my, x + mx) inside the frame, else T(y, x)."""
    n, H, W = frames.shape
    out = np.empty_like(frames)
    y, x = np.mgrid[0:H, 0:W]
    for t in range(n):
        sy, sx = y + int(shifts[t, 0]), x + int(shifts[t, 1])
        inside = (sy >= 0) & (sy < H) & (sx >= 0) & (sx < W)
        src = frames[t][np.clip(sy, 0, H - 1), np.clip(sx, 0, W - 1)]
        out[t] = np.where(inside, src, tmpl)
    return out


def correct(frames: np.ndarray, R: int = 8, tmpl: np.ndarray | None = None):
    """Template (from the first 50 frames unless given), motion, corrected frames."""
    if tmpl is None:
        tmpl = make_template(frames[:TEMPLATE_FRAMES])
    shifts, sc = estimate(frames, tmpl, R)
    return apply_shifts(frames, shifts, tmpl), shifts, tmpl
