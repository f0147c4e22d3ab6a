"""Hand-built test videos (input generators only; no step of the method)."""
import numpy as np


def ring_video(n_cells=6, radius=7.0, sigma=3.0, frames=1000, seed=0):
    """n_cells Gaussian cells on a ring around the centre of a 64 x 64 frame,
    neighbours overlapping, so they form one connected component; cell j
    fires (two frames, +40% and +20% of its footprint) in segments j,
    j + n_cells, ..., so every cell spikes alone in some segments and the
    component's detection matrix has rank n_cells. Poisson-Gaussian noise
    (read noise sd 5) around 1000 counts."""
    rng = np.random.default_rng(seed)
    yy, xx = np.mgrid[0:64, 0:64].astype(np.float64)
    cells = []
    for j in range(n_cells):
        ang = 2 * np.pi * j / n_cells
        cx, cy = 32 + radius * np.cos(ang), 32 + radius * np.sin(ang)
        cells.append(np.exp(-((xx - cx) ** 2 + (yy - cy) ** 2) / (2 * sigma ** 2)))
    cells = np.array(cells)
    act = np.zeros((frames, n_cells))
    for j in range(n_cells):
        for seg in range(j, frames // 50, n_cells):
            act[seg * 50 + 20 + j, j] = 1.0
            act[seg * 50 + 21 + j, j] = 0.5
    mean = 1000.0 * (1.0 + 0.4 * np.tensordot(act, cells, axes=1))
    v = rng.poisson(mean) + rng.normal(0.0, 5.0, mean.shape)
    return np.clip(np.rint(v), 0, 65535).astype(np.uint16)
