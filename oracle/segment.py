"""FP64 oracle of the neuron-segmentation stage (Bando et al., 2023, Sec. III).

TEST INFRASTRUCTURE: imported only by tests, the smoke check and the benchmark's
CPU-baseline leg. Written from the paper's definitions and the readings listed
below; slow on purpose, no blocking or fusion.

Steps, in the paper's order:

  segmentation   V is cut into non-overlapping segments V_i of L = 50 frames
                 (Sec. III-B; 1,000 frames give 20 summary pairs in Sec. III-C).
                 A trailing partial segment is dropped.
  Eq. 1          S_i(x) = (1/L) sum_t V_i(x, t)                   (Sec. III-B)
  Eq. 2          T_i(x) = max_t Vbar_i(x, t) - median_t Vbar_i(x, t), with
                 Vbar_i = G * V_i, G a Gaussian of sd 3 px       (Sec. III-B)
  noise scale    D_i(x) = (1/L) sum_t max(0, med_i(x) - Vbar_i(x, t)),
                 sigma(x) = sqrt(2 pi) * (1/K) sum_i D_i(x)      (reading)
  events         z_i = T_i / sigma, e_i = [z_i >= theta], p_i = max(0, z_i - theta)
                 stand where the paper thresholds its probability maps
                 (Sec. III-D).
  shape filter   8-connected regions of e_i kept by area, solidity (the
                 paper's "concaveness") and eccentricity       (Sec. III-D)
  aggregation    b(x) = [sum_i b_i(x) >= c_min]; c_min = 1 is the paper's OR
                 (Sec. III-D); the plain detector uses c_min = 2.
  components     8-connected components of b, numbered by minimum raster index
  NMF            per component, P_c ~ F A (Eq. 3, Sec. III-D): SPA picks the
                 rank and initial footprints, then HALS sweeps.
  correlation    8-neighbour Pearson correlation of the raw video, pooled
                 within segments (the summary image of Sec. III-A).

Readings where the paper is silent (each also listed in the design notes):
  * Gaussian: sampled taps exp(-k^2 / (2 sigma^2)) for |k| <= 12 (4 sigma),
    normalised to sum 1, separable; half-sample-symmetric reflection at the
    frame border (index j -> j mod 2n, then 2n - 1 - j if >= n).
  * median of an even count is the mean of the two middle order statistics.
  * shape filter: area in [16, 1600], solidity >= 0.75 with the convex hull of
    the pixel-square corners, eccentricity <= 0.95 from the covariance of the
    pixel centres, compared as lambda_min / lambda_max >= 1 - ecc_max^2.
  * NMF: SPA on the raw nonzero columns of P_c (stop when the largest residual
    column norm is below delta = 0.3 times the first pick's norm, or at max
    rank 6). Raw columns, not l1-normalised ones: after l1 normalisation a
    segment where a single pixel barely crosses the threshold becomes a unit
    vertex that SPA picks first, which then stops the rank search. Initial
    footprints = the picked raw columns scaled to max 1, A = 0, one HALS
    A-update then `nmf_sweeps` HALS sweeps (rows of A, then columns of F),
    footprints scaled to max 1, masks f >= 0.25, masks smaller than area_min
    dropped, ordered by component then by raster index of the footprint peak.
"""
from __future__ import annotations

from collections import deque
from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class Params:
    seg_len: int = 50
    sigma: float = 3.0
    radius: int = 12
    event_z: float = 5.0
    min_event_segs: int = 2
    area_min: int = 16
    area_max: int = 1600
    solidity_min: float = 0.75
    ecc_max: float = 0.95
    nmf_max_rank: int = 6
    nmf_sweeps: int = 200
    spa_delta: float = 0.3
    footprint_level: float = 0.25
    sigma_floor: float = 1e-3


# ----------------------------------------------------------------------------
# Gaussian pre-smoothing (Sec. III-B, the smoothing inside Eq. 2)
# ----------------------------------------------------------------------------

def gaussian_weights(sigma: float, radius: int) -> np.ndarray:
    """Taps w_k, k = -radius..radius: exp(-k^2 / (2 sigma^2)) normalised to 1."""
    k = np.arange(-radius, radius + 1, dtype=np.float64)
    w = np.exp(-(k * k) / (2.0 * sigma * sigma))
    return w / w.sum()


def reflect_index(j: int, n: int) -> int:
    """Half-sample-symmetric reflection of index j into [0, n)."""
    j = j % (2 * n)
    return 2 * n - 1 - j if j >= n else j


def smoothing_matrix(n: int, sigma: float, radius: int) -> np.ndarray:
    """The 1-D smoothing operator along an axis of length n as an n x n matrix:
    out[a] = sum_k w_k in[reflect(a + k)]."""
    w = gaussian_weights(sigma, radius)
    G = np.zeros((n, n))
    for a in range(n):
        for k in range(-radius, radius + 1):
            G[a, reflect_index(a + k, n)] += w[k + radius]
    return G


def smooth_frames(frames: np.ndarray, sigma: float = 3.0, radius: int = 12) -> np.ndarray:
    """Vbar = G * V for every frame: Gy @ V_t @ Gx^T, FP64. frames: [L, H, W]."""
    L, H, W = frames.shape
    Gy = smoothing_matrix(H, sigma, radius)
    Gx = smoothing_matrix(W, sigma, radius)
    f = frames.astype(np.float64)
    return np.matmul(np.matmul(Gy, f), Gx.T)


# ----------------------------------------------------------------------------
# Segment summaries: Eq. 1, Eq. 2, noise scale
# ----------------------------------------------------------------------------

def summarize_segment(seg: np.ndarray, prm: Params = Params()) -> dict:
    """Summaries of one segment seg: uint16 [L, H, W].

    S   Eq. 1, temporal mean of the raw segment.
    T   Eq. 2, max minus median over time of the smoothed segment.
    D   mean over time of max(0, median - smoothed value): the per-segment
        noise-scale term (reading; the paper has no noise normalisation).
    """
    L = seg.shape[0]
    S = seg.astype(np.int64).sum(axis=0) / float(L)
    vbar = smooth_frames(seg, prm.sigma, prm.radius)
    srt = np.sort(vbar, axis=0)
    if L % 2:
        med = srt[L // 2]
    else:
        med = 0.5 * (srt[L // 2 - 1] + srt[L // 2])
    mx = srt[-1]
    T = mx - med
    D = np.maximum(0.0, med[None] - vbar).sum(axis=0) / float(L)
    return dict(S=S, T=T, D=D, med=med, max=mx)


OFFSETS = ((0, 0), (0, 1), (1, 0), (1, 1), (1, -1))  # (dy, dx): self, right, down, down-right, down-left


def segment_moments(seg: np.ndarray) -> np.ndarray:
    """Centred co-moments of one raw segment, [5, H, W] FP64:
    C_o(x) = sum_t (V(x,t) - S(x)) (V(x+o,t) - S(x+o)) for the offsets o in
    OFFSETS; zero where x + o leaves the frame."""
    v = seg.astype(np.float64)
    c = v - v.mean(axis=0)
    L, H, W = v.shape
    out = np.zeros((5, H, W))
    for k, (dy, dx) in enumerate(OFFSETS):
        ys = slice(0, H - dy)
        yd = slice(dy, H)
        if dx >= 0:
            xs, xd = slice(0, W - dx), slice(dx, W)
        else:
            xs, xd = slice(-dx, W), slice(0, W + dx)
        out[k, ys, xs] = (c[:, ys, xs] * c[:, yd, xd]).sum(axis=0)
    return out


def correlation_image(C: np.ndarray) -> np.ndarray:
    """R(x): mean over the in-frame 8-neighbours y of
    rho(x, y) = C(x, y) / sqrt(C(x, x) C(y, y)), rho = 0 if a variance is 0.
    C: pooled co-moments [5, H, W] as produced by segment_moments."""
    _, H, W = C.shape
    var = C[0]
    acc = np.zeros((H, W))
    cnt = np.zeros((H, W))
    for k, (dy, dx) in enumerate(OFFSETS[1:], start=1):
        for sgn in (1, -1):
            # pair (x, x + o) stored at x; the reverse pair (y, y - o) at y - o
            ddy, ddx = sgn * dy, sgn * dx
            for y in range(H):
                yy = y + ddy
                if not 0 <= yy < H:
                    continue
                for x in range(W):
                    xx = x + ddx
                    if not 0 <= xx < W:
                        continue
                    if sgn == 1:
                        cov = C[k, y, x]
                    else:
                        cov = C[k, yy, xx]
                    d = var[y, x] * var[yy, xx]
                    acc[y, x] += cov / np.sqrt(d) if d > 0 else 0.0
                    cnt[y, x] += 1
    return acc / cnt


# ----------------------------------------------------------------------------
# Events (stand-in for thresholding the probability maps, Sec. III-D)
# ----------------------------------------------------------------------------

def event_maps(T: np.ndarray, sigma: np.ndarray, prm: Params = Params()) -> dict:
    """z = T / sigma (0 where sigma < floor), e = [z >= theta],
    p = max(0, z - theta), count c(x) = sum_i e_i(x), margin |z - theta|."""
    ok = sigma >= prm.sigma_floor
    safe = np.where(ok, sigma, 1.0)
    z = np.where(ok[None], T / safe[None], 0.0)
    e = z >= prm.event_z
    p = np.maximum(0.0, z - prm.event_z)
    return dict(z=z, e=e, p=p, count=e.sum(axis=0), margin=np.abs(z - prm.event_z))


# ----------------------------------------------------------------------------
# Connected components, region shape (Sec. III-D)
# ----------------------------------------------------------------------------

def label8(mask: np.ndarray):
    """8-connected components by breadth-first flood fill.

    Pixels are scanned in raster order and each unlabelled foreground pixel
    starts a new component, so components are numbered 1..n by their minimum
    raster index. Returns (labels int32 [H, W] with 0 = background, n)."""
    H, W = mask.shape
    lab = np.zeros((H, W), np.int32)
    n = 0
    ys, xs = np.nonzero(mask)
    for y0, x0 in zip(ys.tolist(), xs.tolist()):
        if lab[y0, x0]:
            continue
        n += 1
        lab[y0, x0] = n
        q = deque([(y0, x0)])
        while q:
            y, x = q.popleft()
            for dy in (-1, 0, 1):
                yy = y + dy
                if not 0 <= yy < H:
                    continue
                for dx in (-1, 0, 1):
                    xx = x + dx
                    if 0 <= xx < W and mask[yy, xx] and not lab[yy, xx]:
                        lab[yy, xx] = n
                        q.append((yy, xx))
    return lab, n


def hull_area2(points) -> int:
    """Twice the area of the convex hull of integer points (monotone chain,
    exact integer shoelace)."""
    pts = sorted(set(map(tuple, points)))
    if len(pts) < 3:
        return 0

    def cross(o, a, b):
        return (a[0] - o[0]) * (b[1] - o[1]) - (a[1] - o[1]) * (b[0] - o[0])

    lower, upper = [], []
    for p in pts:
        while len(lower) >= 2 and cross(lower[-2], lower[-1], p) <= 0:
            lower.pop()
        lower.append(p)
    for p in reversed(pts):
        while len(upper) >= 2 and cross(upper[-2], upper[-1], p) <= 0:
            upper.pop()
        upper.append(p)
    hull = lower[:-1] + upper[:-1]
    a2 = 0
    for i in range(len(hull)):
        x0, y0 = hull[i]
        x1, y1 = hull[(i + 1) % len(hull)]
        a2 += x0 * y1 - x1 * y0
    return abs(a2)


def region_stats(ys: np.ndarray, xs: np.ndarray) -> dict:
    """Shape of one region given its pixel rows ys and columns xs.

    area      pixel count n
    ratio     lambda_min / lambda_max of the pixel-centre covariance (1 when
              both are 0); eccentricity = sqrt(1 - ratio)
    hull2     twice the area of the convex hull of the pixel-square corners;
              only each row's leftmost and rightmost pixel contribute corners
    solidity  n / (hull2 / 2)
    """
    n = int(len(xs))
    X = [int(v) for v in xs]
    Y = [int(v) for v in ys]
    sx, sy = sum(X), sum(Y)
    sxx = sum(v * v for v in X)
    syy = sum(v * v for v in Y)
    sxy = sum(a * b for a, b in zip(X, Y))
    a = n * sxx - sx * sx      # n^2 var_x   (exact integers)
    b = n * syy - sy * sy      # n^2 var_y
    c = n * sxy - sx * sy      # n^2 cov_xy
    p = float(a + b)
    s = float(np.sqrt(float(a - b) * float(a - b) + 4.0 * float(c) * float(c)))
    ratio = (p - s) / (p + s) if p + s > 0 else 1.0
    rows = {}
    for yv, xv in zip(Y, X):
        lo, hi = rows.get(yv, (xv, xv))
        rows[yv] = (min(lo, xv), max(hi, xv))
    corners = []
    for yv, (lo, hi) in rows.items():
        corners += [(lo, yv), (lo, yv + 1), (hi + 1, yv), (hi + 1, yv + 1)]
    h2 = hull_area2(corners)
    return dict(area=n, ratio=ratio, ecc=float(np.sqrt(max(0.0, 1.0 - ratio))),
                hull2=h2, solidity=2.0 * n / h2 if h2 else 1.0)


def shape_filter(e: np.ndarray, prm: Params = Params()):
    """b_i: the union of the 8-connected regions of the event mask e that are
    kept by area, solidity and eccentricity. Returns (b, regions) where
    regions lists each region's stats, keep flag and threshold margins."""
    lab, n = label8(e)
    b = np.zeros_like(e, dtype=bool)
    regions = []
    if n == 0:
        return b, regions
    flat = lab.ravel()
    order = np.argsort(flat, kind="stable")
    bounds = np.searchsorted(flat[order], np.arange(1, n + 2))
    H, W = e.shape
    thr = 1.0 - prm.ecc_max * prm.ecc_max
    for r in range(n):
        idx = order[bounds[r]:bounds[r + 1]]
        ys, xs = np.divmod(idx, W)
        st = region_stats(ys, xs)
        keep_area = prm.area_min <= st["area"] <= prm.area_max
        keep_sol = st["solidity"] >= prm.solidity_min
        keep_ecc = st["ratio"] >= thr
        st.update(label=r + 1, keep=bool(keep_area and keep_sol and keep_ecc),
                  keep_area=keep_area, keep_sol=keep_sol, keep_ecc=keep_ecc,
                  margin_sol=abs(st["solidity"] - prm.solidity_min),
                  margin_ecc=abs(st["ratio"] - thr))
        regions.append(st)
        if st["keep"]:
            b.ravel()[idx] = True
    return b, regions


def aggregate(b: np.ndarray, prm: Params = Params()):
    """n_b(x) = sum_i b_i(x), b(x) = [n_b >= c_min], components of b."""
    nb = b.sum(axis=0)
    bb = nb >= prm.min_event_segs
    lab, n = label8(bb)
    return nb, bb, lab, n


# ----------------------------------------------------------------------------
# Footprint reconstruction: NMF of Eq. 3 per component (Sec. III-D)
# ----------------------------------------------------------------------------

def spa(P: np.ndarray, delta: float, max_rank: int) -> list:
    """Successive projection on the columns of P (Gillis and Vavasis, 2014).

    R starts as P. Each step picks j* = argmax_j ||R[:, j]||_2 (lowest j on
    ties), stops when that norm falls below delta times the first pick's norm
    or at max_rank, else projects R onto the orthogonal complement of the
    picked residual column."""
    R = P.astype(np.float64).copy()
    picks = []
    ref = None
    while len(picks) < max_rank:
        norms = np.sqrt((R * R).sum(axis=0))
        j = int(np.argmax(norms))
        if ref is None:
            ref = norms[j]
        elif norms[j] < delta * ref:
            break
        picks.append(j)
        u = R[:, j] / norms[j]
        R = R - np.outer(u, u @ R)
    return picks


def _hals_update_A(P, F, A):
    FtP = F.T @ P
    FtF = F.T @ F
    for n in range(A.shape[0]):
        if FtF[n, n] > 0:
            A[n] = np.maximum(0.0, A[n] + (FtP[n] - FtF[n] @ A) / FtF[n, n])
    return A


def _hals_update_F(P, F, A):
    PAt = P @ A.T
    AAt = A @ A.T
    for n in range(F.shape[1]):
        if AAt[n, n] > 0:
            F[:, n] = np.maximum(0.0, F[:, n] + (PAt[:, n] - F @ AAt[:, n]) / AAt[n, n])
    return F


def hals(P: np.ndarray, F0: np.ndarray, sweeps: int):
    """HALS for P ~ F A with F, A >= 0 (Eq. 3): A starts at 0 and gets one
    row-wise update; then each sweep updates the rows of A in order and the
    columns of F in order, clipping at 0. Rows/columns with zero Gram diagonal
    are left unchanged."""
    F = F0.copy()
    A = np.zeros((F.shape[1], P.shape[1]))
    A = _hals_update_A(P, F, A)
    for _ in range(sweeps):
        A = _hals_update_A(P, F, A)
        F = _hals_update_F(P, F, A)
    return F, A


def nmf_component(P: np.ndarray, prm: Params = Params()):
    """NMF of one component's probability matrix P [M_c, K].

    Returns (F [M_c, N] scaled to max 1 per column, A [N, K], picks) with N
    the SPA rank over the nonzero columns; N = 0 when P is all zero."""
    nz = np.flatnonzero(np.abs(P).sum(axis=0) > 0)
    if len(nz) == 0:
        return np.zeros((P.shape[0], 0)), np.zeros((0, P.shape[1])), []
    picks = [int(nz[j]) for j in spa(P[:, nz], prm.spa_delta, prm.nmf_max_rank)]
    F0 = P[:, picks].copy()
    F0 /= F0.max(axis=0, keepdims=True)
    F, A = hals(P, F0, prm.nmf_sweeps)
    for n in range(F.shape[1]):
        m = F[:, n].max()
        if m > 0:
            F[:, n] /= m
            A[n] *= m
    return F, A, picks


def footprints(p: np.ndarray, labels: np.ndarray, n_comp: int, prm: Params = Params()):
    """Per-component NMF of the stacked maps p [K, H, W] (Eq. 3).

    Returns a list of dicts (component, weights [H, W], mask [H, W],
    activity [K], peak raster index), ordered by component then peak index,
    with footprints whose mask has fewer than area_min pixels dropped."""
    K, H, W = p.shape
    out = []
    flat_lab = labels.ravel()
    pf = p.reshape(K, -1)
    for c in range(1, n_comp + 1):
        pix = np.flatnonzero(flat_lab == c)          # raster order
        P = pf[:, pix].T                             # [M_c, K]
        F, A, _ = nmf_component(P, prm)
        items = []
        for n in range(F.shape[1]):
            f = F[:, n]
            if f.max() <= 0:
                continue
            mask = f >= prm.footprint_level
            if mask.sum() < prm.area_min:
                continue
            wimg = np.zeros(H * W)
            wimg[pix] = f
            items.append(dict(component=c, weights=wimg.reshape(H, W),
                              mask=(wimg >= prm.footprint_level).reshape(H, W) & (labels == c),
                              activity=A[n].copy(), peak=int(pix[int(np.argmax(f))])))
        items.sort(key=lambda d: d["peak"])
        out += items
    return out


# ----------------------------------------------------------------------------
# Whole stage
# ----------------------------------------------------------------------------

@dataclass
class Result:
    S: np.ndarray          # [K, H, W]
    T: np.ndarray          # [K, H, W]
    D: np.ndarray          # [K, H, W]
    sigma: np.ndarray      # [H, W]
    mean: np.ndarray       # [H, W]
    corr: np.ndarray       # [H, W]
    moments: np.ndarray    # [5, H, W] pooled co-moments
    z: np.ndarray
    e: np.ndarray
    p: np.ndarray
    count: np.ndarray      # [H, W] events per pixel
    b: np.ndarray          # [K, H, W] kept-region masks
    nb: np.ndarray         # [H, W]
    labels: np.ndarray     # [H, W] components of the aggregate mask
    n_comp: int
    footprints: list
    regions: list = field(default_factory=list)   # per segment
    event_margin: np.ndarray = None


def segment(video: np.ndarray, prm: Params = Params(), with_corr: bool = True) -> Result:
    """Run every step on a uint16 video [T, H, W]."""
    L = prm.seg_len
    K = video.shape[0] // L
    if K == 0:
        raise ValueError("video shorter than one segment")
    H, W = video.shape[1:]
    S = np.zeros((K, H, W))
    Tm = np.zeros((K, H, W))
    D = np.zeros((K, H, W))
    C = np.zeros((5, H, W))
    for i in range(K):
        seg = video[i * L:(i + 1) * L]
        r = summarize_segment(seg, prm)
        S[i], Tm[i], D[i] = r["S"], r["T"], r["D"]
        if with_corr:
            C += segment_moments(seg)
    sigma = np.sqrt(2.0 * np.pi) * D.sum(axis=0) / K
    ev = event_maps(Tm, sigma, prm)
    b = np.zeros((K, H, W), bool)
    regions = []
    for i in range(K):
        b[i], reg = shape_filter(ev["e"][i], prm)
        regions.append(reg)
    nb, bb, lab, n = aggregate(b, prm)
    fps = footprints(ev["p"], lab, n, prm)
    return Result(S=S, T=Tm, D=D, sigma=sigma, mean=S.mean(axis=0),
                  corr=correlation_image(C) if with_corr else None, moments=C,
                  z=ev["z"], e=ev["e"], p=ev["p"], count=ev["count"], b=b,
                  nb=nb, labels=lab, n_comp=n, footprints=fps, regions=regions,
                  event_margin=ev["margin"])
