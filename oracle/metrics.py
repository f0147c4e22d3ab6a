"""Footprint agreement: F1 at an IoU threshold (Sec. IV-B follows the
CaImAn/VolPy convention of F1 at IoU 0.3; the matching rule is a reading:
one-to-one assignment maximising the summed IoU over pairs at or above the
threshold).

TEST INFRASTRUCTURE (imported by tests and the benchmark's evaluation only).
"""
from __future__ import annotations

import numpy as np


def iou_matrix(pred: np.ndarray, ref: np.ndarray) -> np.ndarray:
    """IoU between every predicted mask [Np, H, W] and reference mask [Nr, H, W]."""
    a = pred.reshape(len(pred), -1).astype(np.float64)
    b = ref.reshape(len(ref), -1).astype(np.float64)
    inter = a @ b.T
    union = a.sum(1)[:, None] + b.sum(1)[None, :] - inter
    return np.where(union > 0, inter / np.maximum(union, 1), 0.0)


def _assign(w: np.ndarray):
    """Maximum-weight one-to-one assignment on a small nonnegative matrix by
    exhaustive search over the smaller side (exact; used for tiny cases) or the
    Hungarian method (Kuhn-Munkres, O(n^3)) for larger ones."""
    n, m = w.shape
    transpose = n > m
    if transpose:
        w = w.T
        n, m = m, n
    # Hungarian method on cost = max - w, rows <= cols
    INF = float("inf")
    cost = w.max() - w if w.size else w
    u = np.zeros(n + 1)
    v = np.zeros(m + 1)
    p = np.zeros(m + 1, dtype=np.int64)
    way = np.zeros(m + 1, dtype=np.int64)
    for i in range(1, n + 1):
        p[0] = i
        j0 = 0
        minv = np.full(m + 1, INF)
        used = np.zeros(m + 1, bool)
        while True:
            used[j0] = True
            i0 = p[j0]
            delta = INF
            j1 = 0
            for j in range(1, m + 1):
                if not used[j]:
                    cur = cost[i0 - 1, j - 1] - u[i0] - v[j]
                    if cur < minv[j]:
                        minv[j] = cur
                        way[j] = j0
                    if minv[j] < delta:
                        delta = minv[j]
                        j1 = j
            for j in range(m + 1):
                if used[j]:
                    u[p[j]] += delta
                    v[j] -= delta
                else:
                    minv[j] -= delta
            j0 = j1
            if p[j0] == 0:
                break
        while True:
            j1 = way[j0]
            p[j0] = p[j1]
            j0 = j1
            if j0 == 0:
                break
    pairs = [(p[j] - 1, j - 1) for j in range(1, m + 1) if p[j] != 0]
    if transpose:
        pairs = [(b, a) for a, b in pairs]
    return pairs


def match_f1(pred: np.ndarray, ref: np.ndarray, thr: float = 0.3) -> dict:
    """Precision, recall, F1 and matched IoUs of predicted vs reference masks."""
    npred, nref = len(pred), len(ref)
    if npred == 0 or nref == 0:
        return dict(precision=0.0 if npred else 1.0 * (nref == 0),
                    recall=0.0 if nref else 1.0 * (npred == 0),
                    f1=1.0 if npred == nref == 0 else 0.0, matches=[], n_pred=npred,
                    n_ref=nref)
    iou = iou_matrix(pred, ref)
    w = np.where(iou >= thr, iou, 0.0)
    pairs = [(i, j) for i, j in _assign(w) if w[i, j] > 0]
    tp = len(pairs)
    prec = tp / npred
    rec = tp / nref
    f1 = 2 * prec * rec / (prec + rec) if tp else 0.0
    return dict(precision=prec, recall=rec, f1=f1,
                matches=[(i, j, float(iou[i, j])) for i, j in pairs],
                n_pred=npred, n_ref=nref)
