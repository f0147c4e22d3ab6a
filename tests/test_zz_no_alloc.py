"""The allocation-free motion estimate (seg_mc_estimate_static) against the
workspace one (seg_mc_estimate), through the C ABI.

Both run the same kernels in the same order of sums, so motion and scores
must be identical. Two calls in a row share the library's fixed array: the
second has fewer frames and another corrector with more candidate vectors, so
anything the first call left behind would show up in its results.
"""
import numpy as np
import pytest
import torch

from paper_2403_16438_amd import MotionCorrector, abi, to_device_frames
from synth import plant_motion, preset, simulate

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _corrector(H, W, R, seed, frames):
    video, _ = simulate(preset(1, height=H, width=W, frames=frames), seed)
    moved, _ = plant_motion(video, R - 1, seed + 1)
    d = to_device_frames(moved, DEV)
    mc = MotionCorrector(H, W, DEV, radius=R)
    mc.set_template(d[:50])
    return mc, d


def _static(mc, frames, with_scores=True):
    n = frames.shape[0]
    m = torch.full((n, 2), -99, dtype=torch.int32, device=DEV)
    s = (torch.full((n, mc.n_vectors), float("nan"), dtype=torch.float64, device=DEV)
         if with_scores else None)
    mc.estimate_static(frames, m, s)
    torch.cuda.synchronize()
    return m, s


def test_static_estimate_equals_workspace_estimate():
    assert abi.SEG_MC_STATIC_MAX_FRAMES == 256
    a, da = _corrector(96, 112, 6, 5, 300)
    ref_m, ref_s = a.estimate(da, scores=True)
    m, s = _static(a, da[:256])                      # a full call
    assert torch.equal(m, ref_m[:256])
    assert torch.equal(s, ref_s[:256])
    b, db = _corrector(128, 128, 10, 9, 120)         # then fewer frames, more vectors
    ref_m2, ref_s2 = b.estimate(db[13:90], scores=True)
    m2, s2 = _static(b, db[13:90])
    assert torch.equal(m2, ref_m2)
    assert torch.equal(s2, ref_s2)
    m3, _ = _static(a, da[200:223], with_scores=False)   # motion only
    assert torch.equal(m3, ref_m[200:223])
    torch.cuda.synchronize()


def test_static_estimate_limits():
    a, da = _corrector(64, 64, 4, 3, 300)
    with pytest.raises(abi.SegError) as e:
        _static(a, da[:257])
    assert e.value.code == abi.SEG_E_CAPACITY
    fresh = MotionCorrector(64, 64, DEV, radius=4)   # no template yet
    with pytest.raises(abi.SegError) as e:
        _static(fresh, da[:10])
    assert e.value.code == abi.SEG_E_STATE
    m, _ = _static(a, da[:0])                        # nothing to do
    assert m.shape == (0, 2)
    # the corrector is still usable after the rejected calls
    ref = a.estimate(da[:40])
    m, _ = _static(a, da[:40], with_scores=False)
    assert torch.equal(m, ref)
