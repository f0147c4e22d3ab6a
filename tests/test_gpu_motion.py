"""Motion correction on the GPU (include/seg_mc.h) against the FP64 oracle.

Bars: templates bit-exact (integer arithmetic on both sides); vector scores
within 1e-10 of the oracle (both evaluate ZNCC in FP64: the GPU from exact
integer moments, the oracle from centred values, so they differ by rounding
only); motion equal to the oracle's wherever the oracle's best score leads
the runner-up by more than 1e-9, and otherwise a vector whose oracle score is
within 1e-9 of the best; corrected frames bit-exact against the oracle's
shift of the same frames (template values where the shift leaves the frame).
"""
import numpy as np
import pytest
import torch

import oracle.motion as om
from paper_2403_16438_amd import MotionCorrector, abi, to_device_frames
from synth import move_frames, plant_motion, preset, simulate

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
SCORE_TOL = 1e-10
GAP = 1e-9


def _texture(H, W, seed):
    rng = np.random.default_rng(seed)
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    img = np.full((H, W), 1000.0)
    for _ in range(max(20, H * W // 150)):
        cy, cx, s, a = rng.uniform(0, H), rng.uniform(0, W), rng.uniform(2, 6), rng.uniform(-300, 300)
        img += a * np.exp(-((yy - cy) ** 2 + (xx - cx) ** 2) / (2 * s * s))
    return np.clip(np.rint(img), 0, 65535).astype(np.uint16)


def _noisy(tmpl, n, seed, noise=20.0):
    rng = np.random.default_rng(seed)
    v = tmpl[None].astype(np.float64) + rng.normal(0.0, noise, (n,) + tmpl.shape)
    return np.clip(np.rint(v), 0, 65535).astype(np.uint16)


def _gpu(frames, R, tmpl_frames=None):
    T, H, W = frames.shape
    mc = MotionCorrector(H, W, DEV, radius=R)
    d = to_device_frames(frames, DEV)
    mc.set_template(d[:50] if tmpl_frames is None else to_device_frames(tmpl_frames, DEV))
    motion, sc = mc.estimate(d, scores=True)
    out = mc.apply(d, motion)
    torch.cuda.synchronize()
    return mc, motion.cpu().numpy(), sc.cpu().numpy(), out.cpu().numpy().view(np.uint16)


def _check_against_oracle(frames, R, motion, sc, corrected, tmpl, frames_idx=None):
    idx = range(frames.shape[0]) if frames_idx is None else frames_idx
    vec = om.vectors(R)
    for t in idx:
        ref = om.scores(frames[t], tmpl, R)
        err = np.abs(sc[t] - ref).max()
        assert err <= SCORE_TOL, (t, err)
        order = np.argsort(-ref, kind="stable")
        best = ref[order[0]]
        dy, dx = -int(motion[t, 0]), -int(motion[t, 1])
        assert abs(dy) <= R and abs(dx) <= R
        pick = vec.index((dy, dx))
        if best - ref[order[1]] > GAP:
            assert pick == order[0], (t, pick, order[0])
        else:
            assert ref[pick] >= best - GAP, t
        assert np.array_equal(corrected[t], om.apply_shifts(frames[t:t + 1], motion[t:t + 1], tmpl)[0]), t


def test_small_recording_against_oracle():
    video, _ = simulate(preset(1, frames=300), 3)
    moved, planted = plant_motion(video, 3, 11)
    mc, motion, sc, out = _gpu(moved, 4)
    tmpl = om.make_template(moved[:50])
    assert np.array_equal(mc.template(), tmpl)
    assert (mc.n_patches, mc.n_vectors) == (4, 81)
    _check_against_oracle(moved, 4, motion, sc, out, tmpl)


@pytest.mark.parametrize("R", [1, 2, 3, 5, 6, 7, 9, 10])
def test_every_radius_recovers_planted_shifts(R):
    """All candidate vectors of each radius (kernel instances 1..7 tiles per
    wave), on a textured scene with noise: exact recovery and oracle scores."""
    H, W = 21 * 3 + 2 * R + 5, 21 * 4 + 2 * R + 2
    tmpl = _texture(H, W, R)
    shifts = np.array(om.vectors(R), np.int32)
    frames = move_frames(_noisy(tmpl, len(shifts), 100 + R), shifts)
    mc, motion, sc, out = _gpu(frames, R, tmpl_frames=tmpl[None])
    assert np.array_equal(mc.template(), tmpl)
    assert np.array_equal(motion, shifts)
    _check_against_oracle(frames, R, motion, sc, out, tmpl, frames_idx=range(0, len(shifts), max(1, len(shifts) // 25)))


def test_benchmark_shaped_frames_against_oracle():
    """256 x 256, R = 8: 121 tiles over 8 slices, 289 vectors."""
    video, _ = simulate(preset(2, frames=150), 5)
    moved, planted = plant_motion(video, 6, 2)
    mc, motion, sc, out = _gpu(moved, 8)
    assert (mc.n_patches, mc.n_vectors) == (121, 289)
    tmpl = om.make_template(moved[:50])
    assert np.array_equal(mc.template(), tmpl)
    assert np.array_equal(motion, planted)
    _check_against_oracle(moved, 8, motion, sc, out, tmpl, frames_idx=range(0, 150, 5))
    assert np.array_equal(out[:, 8:-8, 8:-8], video[:, 8:-8, 8:-8])


def test_split_calls_equal_one_call():
    """Frame counts that leave partial workgroups and cross the 2,048-frame
    launch: the scores of every frame do not depend on the call split."""
    tmpl = _texture(70, 90, 7)
    shifts = np.array(om.vectors(3), np.int32)
    shifts = np.tile(shifts, (2100 // len(shifts) + 1, 1))[:2100]
    frames = move_frames(_noisy(tmpl, 2100, 8), shifts)
    mc = MotionCorrector(70, 90, DEV, radius=3)
    d = to_device_frames(frames, DEV)
    mc.set_template(to_device_frames(tmpl[None], DEV))
    whole_m, whole_s = mc.estimate(d, scores=True)
    parts_m, parts_s, t0 = [], [], 0
    for n in (1, 15, 17, 2049, 18):
        m, s = mc.estimate(d[t0:t0 + n], scores=True)
        parts_m.append(m)
        parts_s.append(s)
        t0 += n
    torch.cuda.synchronize()
    assert t0 == 2100
    assert torch.equal(torch.cat(parts_m), whole_m)
    assert torch.equal(torch.cat(parts_s), whole_s)
    assert np.array_equal(whole_m.cpu().numpy(), shifts)


def test_flat_frames_and_template():
    """Zero variance everywhere: every ZNCC is 0, every score 0, and the
    first vector wins (motion (R, R)) on both sides."""
    frames = np.full((20, 50, 50), 1234, np.uint16)
    mc, motion, sc, out = _gpu(frames, 2, tmpl_frames=frames[:1])
    assert np.array_equal(sc, np.zeros_like(sc))
    ref_m, _ = om.estimate(frames, om.make_template(frames[:1]), 2)
    assert np.array_equal(motion, ref_m) and np.array_equal(ref_m[0], [2, 2])
    assert np.array_equal(out, frames)


def test_full_range_values():
    """Pixels up to 65535: integer moments near their largest values."""
    rng = np.random.default_rng(9)
    tmpl = rng.integers(0, 65536, size=(60, 60), dtype=np.uint16)
    shifts = np.array([(0, 0), (2, -1), (-2, 2), (1, 1)], np.int32)
    frames = move_frames(np.repeat(tmpl[None], 4, 0), shifts)
    mc, motion, sc, out = _gpu(frames, 2, tmpl_frames=tmpl[None])
    assert np.array_equal(motion, shifts)
    _check_against_oracle(frames, 2, motion, sc, out, tmpl)


def test_errors_and_empty():
    mc = MotionCorrector(64, 64, DEV, radius=4)
    d = torch.zeros((3, 64, 64), dtype=torch.int16, device=DEV)
    motion = torch.zeros((3, 2), dtype=torch.int32, device=DEV)
    st = torch.cuda.current_stream().cuda_stream
    with pytest.raises(abi.SegError) as e:
        mc.estimate(d)
    assert e.value.code == abi.SEG_E_STATE
    mc.set_template(d)
    abi.seg_mc_estimate(mc.handle, d.data_ptr(), 0, motion.data_ptr(), None, st)     # nothing to do
    with pytest.raises(abi.SegError) as e:
        abi.seg_mc_apply(mc.handle, d.data_ptr(), 3, motion.data_ptr(), d[1:].data_ptr(), st)
    assert e.value.code == abi.SEG_E_INVAL
    with pytest.raises(abi.SegError) as e:
        abi.seg_mc_set_template(mc.handle, d.data_ptr(), 0, st)
    assert e.value.code == abi.SEG_E_INVAL
    m = mc.estimate(d)
    torch.cuda.synchronize()
    assert m.shape == (3, 2)


def test_benchmark_recording_full_size():
    """256 x 256 x 10,000 with drift up to 6 px, in the launch configuration
    bench.py times: every planted displacement recovered; the oracle on
    sampled frames; corrected frames equal the still video inside the
    R-pixel border."""
    video, _ = simulate(preset(2), 2000)
    moved, planted = plant_motion(video, 6, 2001)
    mc = MotionCorrector(256, 256, DEV, radius=8)
    d = to_device_frames(moved, DEV)
    mc.set_template(d[:50])
    motion, sc = mc.estimate(d, scores=True)
    out = mc.apply(d, motion)
    torch.cuda.synchronize()
    got = motion.cpu().numpy()
    assert np.array_equal(got, planted)
    tmpl = om.make_template(moved[:50])
    sample = [0, 49, 50, 2047, 2048, 5000, 7777, 9999]
    sc_s = sc[sample].cpu().numpy()
    out_s = out[sample].cpu().numpy().view(np.uint16)
    _check_against_oracle(moved[sample], 8, got[sample], sc_s, out_s, tmpl)
    still = to_device_frames(video, DEV)
    assert torch.equal(out[:, 8:-8, 8:-8], still[:, 8:-8, 8:-8])
