"""Parity at the workload sizes, in the launch configuration bench.py times.

256 x 256 x 10,000 (the benchmark video, seed 2000, pushed in one call as
bench.py does): the whole FP64 oracle against the GPU path. The bars are
those of the small parity tests: summary images within 1e-4, counts and
labels bit-exact outside the threshold window, footprints with IoU >= 0.99.

Both sizes also check the footprint reconstruction by stage isolation: the
oracle fed the session's own FP32 summaries, with counts, kept masks, n_b and
labels bit-exact and footprints at IoU >= 0.99, so a decision inside the
threshold window never leaves the later stages unchecked.

512 x 512 x 20,000 streamed in 500-frame blocks: the oracle on sampled
segments (their summaries), the finalize by stage isolation on the split NMF
(several cooperative launches) and on one workgroup per component, the block
push against a single push of the whole video (bit-exact, all outputs), and
footprints against the planted truth.
"""
import numpy as np
import pytest
import torch

import oracle
import oracle.traces as otr
from paper_2403_16438_amd import abi, Session, to_device_frames
from synth import preset, simulate
from synth.gpu import GpuScene

from parity import (EVENT_WINDOW, assert_image_close, check_against_full_oracle, check_finalize_stage_isolation,
                    compare_footprints, params_from_config, session_outputs)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bench_video():
    video, truth = simulate(preset(2), 2000)
    T, H, W = video.shape
    sess = Session(H, W, T)
    sess.push(to_device_frames(video, torch.device("cuda:0")))
    sess.finalize()
    torch.cuda.synchronize()
    prm = params_from_config(sess.cfg)
    ref = oracle.segment(video, prm)
    return video, truth, sess, prm, ref


def test_benchmark_video_summaries(bench_video):
    video, truth, sess, prm, ref = bench_video
    assert sess.num_segments == 200
    S = sess.segment_maps(abi.SEG_MAP_S).cpu().numpy()
    T = sess.segment_maps(abi.SEG_MAP_T).cpu().numpy()
    assert np.array_equal(S, ref.S.astype(np.float32))
    for i in range(0, 200, 7):
        assert_image_close(T[i], ref.T[i], what=f"T[{i}]")
    assert_image_close(T, ref.T, what="T (all segments)")
    assert_image_close(sess.image(abi.SEG_IMG_NOISE), ref.sigma, what="sigma")
    assert_image_close(sess.image(abi.SEG_IMG_MEAN), ref.mean, what="mean")
    assert_image_close(sess.image(abi.SEG_IMG_CORR), ref.corr, what="corr")


def test_benchmark_video_events_and_labels(bench_video, record_property):
    """Counts against the whole oracle outside the threshold window; the
    downstream stages on the session's own summaries (stage isolation), so a
    decision in the window never leaves them unchecked."""
    video, truth, sess, prm, ref = bench_video
    out = session_outputs(sess)
    in_window = check_against_full_oracle(out, ref, prm)
    record_property("pixels_with_window_decision", in_window)
    print("pixels with a decision within 1e-6 theta:", in_window)
    check_finalize_stage_isolation(out, prm)


def test_benchmark_video_paper_or(bench_video):
    """c_min = 1 (the paper's OR, Sec. III-D) on the same video, by stage
    isolation on its own summaries."""
    video, truth, sess, prm, ref = bench_video
    T, H, W = video.shape
    s1 = Session(H, W, T, min_event_segs=1)
    s1.push(to_device_frames(video, torch.device("cuda:0")))
    s1.finalize()
    torch.cuda.synchronize()
    prm1 = params_from_config(s1.cfg)
    assert prm1.min_event_segs == 1
    r = check_finalize_stage_isolation(session_outputs(s1), prm1)
    assert len(r["footprints"]) >= len(ref.footprints)
    s1.close()


def test_benchmark_video_footprints(bench_video):
    video, truth, sess, prm, ref = bench_video
    fp = sess.footprints()
    assert len(ref.footprints) >= 20
    compare_footprints(fp, ref.footprints)
    assert oracle.match_f1(fp["masks"], truth.masks())["f1"] >= 0.9


def test_benchmark_video_after_motion_correction(bench_video):
    """The paper's order of stages: the video with planted drift (up to
    6 px), corrected on the GPU, then segmented; the footprints match those
    of the still video."""
    from paper_2403_16438_amd import MotionCorrector
    from synth import plant_motion
    video, truth, sess, prm, ref = bench_video
    moved, planted = plant_motion(video, 6, 2001)
    d = to_device_frames(moved, torch.device("cuda:0"))
    mc = MotionCorrector(256, 256, torch.device("cuda:0"), radius=8)
    mc.set_template(d[:50])
    corrected, motion = mc.correct(d)
    del d
    s2 = Session(256, 256, 10000)
    s2.push(corrected)
    s2.finalize()
    torch.cuda.synchronize()
    assert np.array_equal(motion.cpu().numpy(), planted)
    a, b = s2.footprints()["masks"], sess.footprints()["masks"]
    m = oracle.match_f1(a, b)
    print("footprints after correction", a.shape[0], "still", b.shape[0], m)
    assert m["f1"] >= 0.95


def test_benchmark_video_traces(bench_video):
    """Traces of every footprint over all 10,000 frames, bit-exact (exact
    integer sums, one FP64 division on both sides)."""
    video, truth, sess, prm, ref = bench_video
    masks = sess.footprints()["masks"]
    got = sess.traces(to_device_frames(video, torch.device("cuda:0")))
    torch.cuda.synchronize()
    assert np.array_equal(got.cpu().numpy(), otr.extract_traces(video, masks).astype(np.float32))


@pytest.fixture(scope="module")
def large_field():
    cfg = preset(3)
    scene = GpuScene(cfg, 3000)
    T, H, W = cfg.frames, cfg.height, cfg.width
    video = scene.render(0, T)                                  # device, 10.5 GB
    blocks = Session(H, W, T)
    for t0 in range(0, T, 500):
        blocks.push(video[t0:t0 + 500])
    blocks.finalize()
    whole = Session(H, W, T)
    whole.push(video)
    whole.finalize()
    torch.cuda.synchronize()
    return cfg, scene, video, blocks, whole


def test_large_field_finalize_against_oracle(large_field, record_property):
    """The footprint reconstruction at 512 x 512 x 20,000 (400 segments,
    about 90 components: the split NMF in several cooperative launches)
    against the oracle fed the session's own summaries: counts, kept masks,
    n_b and labels bit-exact, footprints at IoU >= 0.99."""
    cfg, scene, video, blocks, whole = large_field
    prof = blocks.profile()
    record_property("nmf_workgroups", prof["nmf_workgroups"])
    assert prof["nmf_path"] == abi.SEG_NMF_SPLIT and prof["nmf_workgroups"] > 256
    r = check_finalize_stage_isolation(session_outputs(blocks), params_from_config(blocks.cfg))
    print("512x512x20000: components", r["n_comp"], "footprints", len(r["footprints"]),
          "NMF workgroups", prof["nmf_workgroups"])
    assert r["n_comp"] >= 60


def test_large_field_single_workgroup_nmf_against_oracle(large_field):
    """The same recording with one NMF workgroup per component."""
    cfg, scene, video, blocks, whole = large_field
    T, H, W = cfg.frames, cfg.height, cfg.width
    s = Session(H, W, T, nmf_path=abi.SEG_NMF_SINGLE)
    s.push(video)
    s.finalize()
    torch.cuda.synchronize()
    assert s.profile()["nmf_path"] == abi.SEG_NMF_SINGLE
    check_finalize_stage_isolation(session_outputs(s), params_from_config(s.cfg))
    s.close()


def test_large_field_sampled_segments(large_field):
    cfg, scene, video, blocks, whole = large_field
    prm = params_from_config(blocks.cfg)
    for i in (0, 173, 399):
        seg = video[50 * i:50 * (i + 1)].cpu().numpy().view(np.uint16)
        ref = oracle.summarize_segment(seg, prm)
        S = blocks.segment_maps(abi.SEG_MAP_S, i, 1).cpu().numpy()[0]
        T = blocks.segment_maps(abi.SEG_MAP_T, i, 1).cpu().numpy()[0]
        D = blocks.segment_maps(abi.SEG_MAP_D, i, 1).cpu().numpy()[0]
        assert np.array_equal(S, ref["S"].astype(np.float32)), i
        assert_image_close(T, ref["T"], what=f"T[{i}]")
        assert_image_close(D, ref["D"], what=f"D[{i}]")


def test_large_field_blocks_equal_whole(large_field):
    cfg, scene, video, blocks, whole = large_field
    for kind in (abi.SEG_MAP_S, abi.SEG_MAP_T, abi.SEG_MAP_P):
        assert torch.equal(blocks.segment_maps(kind), whole.segment_maps(kind)), kind
    for kind in (abi.SEG_IMG_NOISE, abi.SEG_IMG_CORR, abi.SEG_IMG_LABELS):
        assert np.array_equal(blocks.image(kind), whole.image(kind)), kind
    a, b = blocks.footprints(), whole.footprints()
    assert np.array_equal(a["weights"], b["weights"])
    assert np.array_equal(a["activity"], b["activity"])


def test_large_field_traces_sampled_frames(large_field):
    """All 20,000 frames in one call; the oracle on sampled frames."""
    cfg, scene, video, blocks, whole = large_field
    masks = blocks.footprints()["masks"]
    got = blocks.traces(video)
    torch.cuda.synchronize()
    assert got.shape == (masks.shape[0], cfg.frames)
    for t in (0, 1, 4999, 12345, 19984, 19999):
        frame = video[t:t + 1].cpu().numpy().view(np.uint16)
        ref = otr.extract_traces(frame, masks).astype(np.float32)[:, 0]
        assert np.array_equal(got[:, t].cpu().numpy(), ref), t


def test_large_field_truth(large_field, record_property):
    cfg, scene, video, blocks, whole = large_field
    fp = blocks.footprints()
    f1 = oracle.match_f1(fp["masks"], scene.truth.masks())
    record_property("f1_512", f1["f1"])
    print("512x512x20000: footprints", fp["masks"].shape[0], "truth", len(scene.truth.masks()), "F1", f1)
    assert f1["f1"] >= 0.7
