"""Helpers shared by the GPU parity tests: oracle parameters matching a
seg_config, the summary-image tolerance, and an oracle run of the footprint
reconstruction from given (float32) segment summaries."""
import numpy as np

import oracle

REL = 1e-4          # FP32 summary images vs the FP64 oracle
EVENT_WINDOW = 1e-6  # decisions with |z - theta| <= 1e-6 theta are not compared


def params_from_config(cfg) -> oracle.Params:
    """oracle.Params holding exactly the (float32) values the library uses."""
    f = lambda v: float(np.float32(v))
    return oracle.Params(seg_len=cfg.seg_len, sigma=f(cfg.gauss_sigma), radius=cfg.gauss_radius,
                         event_z=f(cfg.event_z), min_event_segs=cfg.min_event_segs,
                         area_min=cfg.area_min, area_max=cfg.area_max,
                         solidity_min=f(cfg.solidity_min), ecc_max=f(cfg.ecc_max),
                         nmf_max_rank=cfg.nmf_max_rank, nmf_sweeps=cfg.nmf_sweeps,
                         spa_delta=f(cfg.spa_delta), footprint_level=f(cfg.footprint_level),
                         sigma_floor=f(cfg.sigma_floor))


def assert_image_close(gpu, ref, rel=REL, what=""):
    """||gpu - ref||_inf <= rel ||ref||_inf, and per pixel <= rel |ref| where
    |ref| >= 1e-2 ||ref||_inf (the absolute term covers values near zero)."""
    gpu = np.asarray(gpu, np.float64)
    ref = np.asarray(ref, np.float64)
    scale = np.abs(ref).max()
    err = np.abs(gpu - ref)
    assert err.max() <= rel * scale + 1e-30, f"{what}: max err {err.max():.3e} vs {rel * scale:.3e}"
    big = np.abs(ref) >= 1e-2 * scale
    if big.any():
        r = (err[big] / np.abs(ref[big])).max()
        assert r <= rel, f"{what}: max relative err {r:.3e} on large pixels"


def oracle_from_summaries(T, D, prm: oracle.Params):
    """The footprint reconstruction of the oracle fed with given summaries
    (stage isolation): noise scale, events, shape filter, aggregation,
    components and NMF, all in FP64 from the given arrays."""
    T = np.asarray(T, np.float64)
    D = np.asarray(D, np.float64)
    K = T.shape[0]
    sigma = np.sqrt(2.0 * np.pi) * D.sum(axis=0) / K
    ev = oracle.event_maps(T, sigma, prm)
    b = np.zeros(T.shape, bool)
    regions = []
    for i in range(K):
        b[i], reg = oracle.shape_filter(ev["e"][i], prm)
        regions.append(reg)
    nb, bb, lab, n = oracle.aggregate(b, prm)
    fps = oracle.footprints(ev["p"], lab, n, prm)
    return dict(sigma=sigma, z=ev["z"], e=ev["e"], p=ev["p"], count=ev["count"],
                margin=ev["margin"], b=b, nb=nb, labels=lab, n_comp=n, footprints=fps,
                regions=regions)


def region_margin_ok(regions, prm_window=EVENT_WINDOW):
    """True when no region decision lies within the comparison window."""
    for reg in regions:
        for r in reg:
            if r["keep_area"] and r["margin_ecc"] <= prm_window:
                return False
            if r["keep_area"] and r["keep_ecc"] and r["margin_sol"] <= prm_window:
                return False
    return True


def compare_footprints(gpu: dict, ref_list: list, min_iou=0.99):
    """Same components with the same number of footprints each, and every
    footprint's mask (matched in order within a component) at IoU >= min_iou."""
    ref_comp = np.array([f["component"] for f in ref_list], np.int32)
    assert np.array_equal(np.asarray(gpu["component"]), ref_comp), (gpu["component"], ref_comp)
    ious = []
    for j, f in enumerate(ref_list):
        a = gpu["masks"][j]
        b = f["mask"]
        inter = np.logical_and(a, b).sum()
        union = np.logical_or(a, b).sum()
        ious.append(inter / union if union else 1.0)
    if ious:
        assert min(ious) >= min_iou, ious
    return ious
