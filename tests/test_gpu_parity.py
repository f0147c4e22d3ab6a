"""GPU path vs the FP64 oracle, through the C ABI.

Bars: FP32 summary images within 1e-4 of the oracle (relative to the image
maximum; per pixel where |ref| >= 1e-2 max); event counts, kept masks and
component labels bit-exact when no event decision lies within 1e-6 theta of
the threshold (otherwise the downstream stages are compared on the oracle's
own summaries, see test_stage_isolation); footprints: the same number per
component and mask IoU >= 0.99.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2403_16438_amd import abi, segment_video, Session, to_device_frames
from synth import preset, simulate

from parity import (EVENT_WINDOW, assert_image_close, check_against_full_oracle,
                    check_finalize_stage_isolation, compare_footprints, oracle_from_summaries,
                    params_from_config, region_margin_ok, session_outputs)

pytestmark = pytest.mark.gpu


def _maps(sess, kind):
    return sess.segment_maps(kind).cpu().numpy()


def _gpu_all(sess):
    return dict(S=_maps(sess, abi.SEG_MAP_S), T=_maps(sess, abi.SEG_MAP_T), P=_maps(sess, abi.SEG_MAP_P),
                B=_maps(sess, abi.SEG_MAP_B) > 0.5, sigma=sess.image(abi.SEG_IMG_NOISE),
                mean=sess.image(abi.SEG_IMG_MEAN), corr=sess.image(abi.SEG_IMG_CORR),
                count=sess.image(abi.SEG_IMG_EVENT_COUNT), nb=sess.image(abi.SEG_IMG_MASK_COUNT),
                labels=sess.image(abi.SEG_IMG_LABELS), fp=sess.footprints())


@pytest.fixture(scope="module")
def c1():
    video, truth = simulate(preset(1), 0)
    sess = segment_video(video)
    prm = params_from_config(sess.cfg)
    ref = oracle.segment(video, prm)
    return video, truth, sess, prm, ref, _gpu_all(sess)


def test_summary_images(c1):
    video, truth, sess, prm, ref, g = c1
    assert sess.num_segments == 20
    for i in range(ref.S.shape[0]):
        assert_image_close(g["S"][i], ref.S[i], what=f"S[{i}]")
        assert_image_close(g["T"][i], ref.T[i], what=f"T[{i}]")
    assert_image_close(g["sigma"], ref.sigma, what="sigma")
    assert_image_close(g["mean"], ref.mean, what="mean")
    assert_image_close(g["corr"], ref.corr, what="corr")
    # S is one FP64 division of an exact integer sum on both sides
    assert np.array_equal(g["S"], ref.S.astype(np.float32))


def test_events_masks_labels(c1):
    video, truth, sess, prm, ref, g = c1
    out = session_outputs(sess)
    in_window = check_against_full_oracle(out, ref, prm)
    assert in_window == 0          # this video has no decision near theta
    assert_image_close(g["P"], ref.p, what="p")
    check_finalize_stage_isolation(out, prm)


def test_paper_or_aggregation():
    """c_min = 1, the paper's OR of the kept masks (Sec. III-D), against the
    whole oracle and by stage isolation."""
    video, truth = simulate(preset(1), 0)
    sess = segment_video(video, min_event_segs=1)
    prm = params_from_config(sess.cfg)
    assert prm.min_event_segs == 1
    ref = oracle.segment(video, prm)
    out = session_outputs(sess)
    assert check_against_full_oracle(out, ref, prm) == 0
    r = check_finalize_stage_isolation(out, prm)
    assert (r["nb"] == 1).any()            # the OR keeps pixels c_min = 2 drops
    assert len(r["footprints"]) >= 4


def test_footprints(c1):
    video, truth, sess, prm, ref, g = c1
    assert len(ref.footprints) == 4
    ious = compare_footprints(g["fp"], ref.footprints)
    assert len(ious) == 4
    f1 = oracle.match_f1(g["fp"]["masks"], truth.masks(), 0.3)
    assert f1["f1"] == 1.0


def test_stage_isolation(c1):
    """Footprint reconstruction fed the oracle's own summaries (as float32)."""
    video, truth, sess, prm, ref, g = c1
    T32 = ref.T.astype(np.float32)
    S32 = ref.S.astype(np.float32)
    D32 = ref.D.astype(np.float32)
    s2 = Session(64, 64, 1000)
    s2.load_summaries(T32, S32, D32)
    s2.finalize()
    torch.cuda.synchronize()
    r = oracle_from_summaries(T32, D32, prm)
    assert not (r["margin"] <= EVENT_WINDOW * prm.event_z).any()
    assert region_margin_ok(r["regions"])
    assert np.array_equal(s2.image(abi.SEG_IMG_EVENT_COUNT), r["count"])
    assert np.array_equal(_maps(s2, abi.SEG_MAP_B) > 0.5, r["b"])
    assert np.array_equal(s2.image(abi.SEG_IMG_MASK_COUNT), r["nb"])
    assert np.array_equal(s2.image(abi.SEG_IMG_LABELS), r["labels"])
    np.testing.assert_allclose(_maps(s2, abi.SEG_MAP_P), r["p"], rtol=1e-6, atol=1e-6)
    compare_footprints(s2.footprints(), r["footprints"])


def _tall_scene(K=3, H=160, W=128):
    """Event regions of both row classes of the shape filter: a tall ellipse
    (69 rows, kept), a tall arch (70 rows, rejected by solidity alone), a tall
    line (80 rows, rejected by eccentricity), a small disk (kept) and a short
    bar (rejected by eccentricity); every segment the same."""
    yy, xx = np.mgrid[0:H, 0:W]
    m = np.zeros((H, W), bool)
    m |= ((yy - 40) / 34.0) ** 2 + ((xx - 30) / 14.0) ** 2 <= 1.0
    m[85:155, 50:56] = True
    m[85:155, 68:74] = True
    m[85:91, 56:68] = True
    m |= (yy - 20) ** 2 + (xx - 100) ** 2 <= 25
    m[40:42, 88:126] = True
    m[60:140, 110:113] = True
    D = np.ones((K, H, W), np.float32)            # sigma = sqrt(2 pi)
    T = np.where(m, 10.0 * np.sqrt(2.0 * np.pi), 0.0).astype(np.float32)[None].repeat(K, 0)
    return T, np.zeros_like(T), D


def test_tall_regions_shape_filter():
    """Regions taller than 64 rows take the shape filter's wide-table kernel,
    shorter ones the compact one; both against the oracle (Sec. III-D)."""
    T, S, D = _tall_scene()
    s = Session(160, 128, 150)
    s.load_summaries(T, S, D)
    s.finalize()
    torch.cuda.synchronize()
    prm = params_from_config(s.cfg)
    r = oracle_from_summaries(T, D, prm)
    assert region_margin_ok(r["regions"])
    reg = {st["area"]: st for st in r["regions"][0]}
    assert reg[1485]["keep"] and reg[81]["keep"]
    assert reg[912]["keep_area"] and reg[912]["keep_ecc"] and not reg[912]["keep_sol"]
    assert not reg[240]["keep_ecc"] and not reg[76]["keep_ecc"]
    assert np.array_equal(s.image(abi.SEG_IMG_EVENT_COUNT), r["count"])
    assert np.array_equal(_maps(s, abi.SEG_MAP_B) > 0.5, r["b"])
    assert np.array_equal(s.image(abi.SEG_IMG_MASK_COUNT), r["nb"])
    assert np.array_equal(s.image(abi.SEG_IMG_LABELS), r["labels"])
    assert r["labels"].max() == 2


@pytest.mark.parametrize("block", [1, 7, 50, 333])
def test_blocking_invariance(c1, block):
    video, truth, sess, prm, ref, g = c1
    s2 = segment_video(video, block=block)
    h = _gpu_all(s2)
    for k in ("S", "T", "P", "B", "sigma", "corr", "count", "nb", "labels"):
        assert np.array_equal(h[k], g[k]), k
    assert np.array_equal(h["fp"]["weights"], g["fp"]["weights"])
    assert np.array_equal(h["fp"]["activity"], g["fp"]["activity"])


def test_trailing_partial_segment(c1):
    video, truth, sess, prm, ref, g = c1
    extra = np.concatenate([video, video[:25]], axis=0)
    s2 = segment_video(extra)
    assert s2.num_segments == 20
    assert np.array_equal(_maps(s2, abi.SEG_MAP_T), g["T"])
    assert np.array_equal(s2.image(abi.SEG_IMG_LABELS), g["labels"])


@pytest.mark.parametrize("shape", [(37, 53), (5, 4), (1, 1), (130, 70), (16, 200)])
def test_ragged_and_tiny_frames(shape):
    H, W = shape
    rng = np.random.default_rng(H * 1000 + W)
    video = rng.poisson(1000, size=(150, H, W)).astype(np.uint16)
    video[60:62, H // 2, W // 2] += 400
    sess = segment_video(video)
    prm = params_from_config(sess.cfg)
    S = _maps(sess, abi.SEG_MAP_S)
    T = _maps(sess, abi.SEG_MAP_T)
    for i in range(3):
        r = oracle.summarize_segment(video[i * 50:(i + 1) * 50], prm)
        assert_image_close(S[i], r["S"], what=f"S{shape}[{i}]")
        assert_image_close(T[i], r["T"], what=f"T{shape}[{i}]")


def test_zero_activity_no_footprints():
    video, _ = simulate(preset(1, n_neurons=0), 11)
    sess = segment_video(video)
    assert sess.footprints()["masks"].shape[0] == 0
    assert sess.image(abi.SEG_IMG_LABELS).max() == 0


def test_constant_video_has_no_events():
    video = np.full((100, 20, 24), 1234, np.uint16)
    sess = segment_video(video)
    assert np.all(_maps(sess, abi.SEG_MAP_T) == 0)
    assert np.all(sess.image(abi.SEG_IMG_NOISE) == 0)
    assert sess.image(abi.SEG_IMG_EVENT_COUNT).max() == 0
    assert sess.footprints()["masks"].shape[0] == 0


def test_error_conventions():
    s = Session(32, 32, 100)
    frames = to_device_frames(np.zeros((60, 32, 32), np.uint16))
    with pytest.raises(abi.SegError) as e:
        s.finalize()                      # no complete segment yet
    assert e.value.code == abi.SEG_E_STATE
    with pytest.raises(abi.SegError) as e:
        s.footprints()
    assert e.value.code == abi.SEG_E_STATE
    s.push(frames)
    with pytest.raises(abi.SegError) as e:
        s.push(frames)                    # 120 > max_frames
    assert e.value.code == abi.SEG_E_CAPACITY
    with pytest.raises(abi.SegError) as e:
        s.load_summaries(np.zeros((1, 32, 32)), np.zeros((1, 32, 32)), np.zeros((1, 32, 32)))
    assert e.value.code == abi.SEG_E_STATE
    s.finalize()
    with pytest.raises(abi.SegError) as e:
        s.push(frames[:10])
    assert e.value.code == abi.SEG_E_STATE
    with pytest.raises(abi.SegError) as e:
        s.finalize()
    assert e.value.code == abi.SEG_E_STATE
    assert abi.seg_last_error(s.handle) == abi.SEG_OK
    torch.cuda.synchronize()
