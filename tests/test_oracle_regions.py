"""Pins of the oracle's event maps, connected components and region-shape
filter (Sec. III-D: threshold, then drop regions by area, concaveness and
eccentricity, then OR over segments and take connected components)."""
import numpy as np
import pytest
import scipy.ndimage as ndi
from scipy.spatial import ConvexHull

import oracle


def test_event_maps_definition_and_floor():
    T = np.array([[[10.0, 15.0, 0.0], [20.0, 4.0, 7.0]]])
    sig = np.array([[2.0, 3.0, 1e-4], [4.0, 1.0, 1.4]])
    ev = oracle.event_maps(T, sig, oracle.Params(event_z=5.0))
    np.testing.assert_array_equal(ev["e"][0], [[True, True, False], [True, False, True]])
    np.testing.assert_allclose(ev["p"][0], [[0.0, 0.0, 0.0], [0.0, 0.0, 0.0]], atol=1e-15)
    assert ev["z"][0, 0, 2] == 0.0        # sigma below the floor: no event
    assert ev["count"].tolist() == [[1, 1, 0], [1, 0, 1]]


def test_event_commutes_with_prior_normalisation():
    # max - median is positively homogeneous: normalising the smoothed video by
    # a per-pixel constant first gives exactly T / sigma
    rng = np.random.default_rng(3)
    seg = rng.poisson(1000, size=(50, 9, 8)).astype(np.uint16)
    vbar = oracle.smooth_frames(seg)
    s = rng.uniform(1, 5, size=(9, 8))
    n = np.sort(vbar / s, axis=0)
    T_after = n[-1] - 0.5 * (n[24] + n[25])
    T = oracle.summarize_segment(seg)["T"]
    np.testing.assert_allclose(T / s, T_after, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("seed", range(6))
def test_label8_matches_scipy(seed):
    rng = np.random.default_rng(seed)
    m = rng.random((23, 31)) < (0.2 + 0.1 * seed)
    lab, n = oracle.label8(m)
    ref, nref = ndi.label(m, structure=np.ones((3, 3)))
    assert n == nref
    # same partition, numbered by minimum raster index
    firsts = [np.flatnonzero(lab.ravel() == c)[0] for c in range(1, n + 1)]
    assert firsts == sorted(firsts)
    for c in range(1, n + 1):
        ids = np.unique(ref[lab == c])
        assert len(ids) == 1 and np.array_equal(ref == ids[0], lab == c)


@pytest.mark.parametrize("seed", range(5))
def test_hull_matches_scipy(seed):
    rng = np.random.default_rng(seed)
    pts = rng.integers(0, 30, size=(40, 2))
    assert oracle.hull_area2(pts.tolist()) == round(2 * ConvexHull(pts).volume)


def test_hull_degenerate():
    assert oracle.hull_area2([(0, 0), (1, 1), (2, 2)]) == 0
    assert oracle.hull_area2([(0, 0), (0, 1)]) == 0


def _stats(pix):
    ys = np.array([p[0] for p in pix])
    xs = np.array([p[1] for p in pix])
    return oracle.region_stats(ys, xs)


def test_region_single_pixel():
    s = _stats([(4, 4)])
    assert s["area"] == 1 and s["hull2"] == 2 and s["solidity"] == 1.0 and s["ecc"] == 0.0


def test_region_square():
    s = _stats([(y, x) for y in range(3) for x in range(3)])
    assert s["area"] == 9 and s["hull2"] == 18 and s["solidity"] == 1.0
    assert s["ecc"] == 0.0


def test_region_line_is_fully_eccentric():
    s = _stats([(2, x) for x in range(5)])
    assert s["ratio"] == 0.0 and s["ecc"] == 1.0


def test_region_L_tromino():
    s = _stats([(0, 0), (0, 1), (1, 0)])
    assert s["hull2"] == 7                      # hull area 3.5
    assert abs(s["solidity"] - 6.0 / 7.0) < 1e-15


def test_region_rectangle_eccentricity():
    # a x b pixel rectangle: var_x = (a^2-1)/12, var_y = (b^2-1)/12
    s = _stats([(y, x) for y in range(3) for x in range(5)])
    assert abs(s["ratio"] - 8.0 / 24.0) < 1e-15
    assert abs(s["ecc"] - np.sqrt(2.0 / 3.0)) < 1e-15


def test_region_rotated_rectangle_eccentricity_invariant():
    pix = [(y, x) for y in range(3) for x in range(7)]
    a = _stats(pix)
    b = _stats([(x, y) for y, x in pix])          # transpose
    assert abs(a["ratio"] - b["ratio"]) < 1e-15 and a["hull2"] == b["hull2"]


def test_shape_filter_bounds():
    prm = oracle.Params()
    e = np.zeros((40, 40), bool)
    e[2:6, 2:6] = True            # 16 px square: kept (area_min is inclusive)
    e[10:13, 10:15] = True        # 15 px rectangle: too small
    e[20:22, 0:30] = True         # 60 px bar: too eccentric
    # a U shape: low solidity
    e[28:38, 28] = True
    e[28:38, 36] = True
    e[37, 28:37] = True
    b, regs = oracle.shape_filter(e, prm)
    keep = {r["label"]: r["keep"] for r in regs}
    assert keep == {1: True, 2: False, 3: False, 4: False}
    assert regs[2]["keep_ecc"] is False and regs[3]["keep_sol"] is False
    assert b[2:6, 2:6].all() and b.sum() == 16


def test_shape_filter_area_max():
    prm = oracle.Params(area_max=100)
    e = np.zeros((30, 30), bool)
    e[0:10, 0:10] = True
    e[15:26, 15:26] = True
    b, regs = oracle.shape_filter(e, prm)
    assert [r["keep"] for r in regs] == [True, False]


def test_aggregate_min_count_and_labels():
    b = np.zeros((3, 10, 10), bool)
    b[0, 1:4, 1:4] = True
    b[1, 2:5, 2:5] = True
    b[2, 7:9, 7:9] = True
    nb, bb, lab, n = oracle.aggregate(b, oracle.Params(min_event_segs=2))
    assert nb.max() == 2 and n == 1 and bb.sum() == 4
    nb, bb, lab, n = oracle.aggregate(b, oracle.Params(min_event_segs=1))
    assert n == 2 and lab[1, 1] == 1 and lab[7, 7] == 2
