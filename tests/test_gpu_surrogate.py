"""The learned surrogate inside a segmentation session, and what training
gains: a short training run on simulated 64x64 segments, then the plain and
the surrogate detectors on held-out 128x128 videos against ground truth."""
import numpy as np
import pytest
import torch

import oracle
from paper_2403_16438_amd import abi, segment_video, Session
from paper_2403_16438_amd.surrogate import Surrogate, he_init
from paper_2403_16438_amd.train import SceneBank, for_frames, train
from synth import preset
from synth.gpu import GpuScene

pytestmark = pytest.mark.gpu


def _video(h, w, frames, seed, **kw):
    cfg = preset(2, height=h, width=w, frames=frames, n_neurons=8, n_overlap=2, **kw)
    sc = GpuScene(cfg, seed)
    return sc.render(0, frames).cpu().numpy().view(np.uint16), sc.truth


def test_session_maps_equal_network_output():
    """The session's detection maps are the network's probabilities per segment."""
    v, _ = _video(64, 64, 250, 31)
    net = Surrogate(1, 64, 64, he_init(5))
    sess = segment_video(v, block=70, net=net)
    P = sess.segment_maps(abi.SEG_MAP_P).cpu().numpy()
    assert P.shape == (5, 64, 64)
    for i in range(5):
        p = net.forward(torch.from_numpy(v[i * 50:(i + 1) * 50][None].view(np.int16)).cuda())
        assert np.array_equal(P[i], p[0].cpu().numpy())
    # the events are the thresholded probabilities
    count = sess.image(abi.SEG_IMG_EVENT_COUNT)
    assert np.array_equal(count, (P >= 0.5).sum(0))


def test_surrogate_needs_a_model_and_shape():
    s = Session(64, 64, 100, detector=abi.SEG_DET_SURROGATE, event_z=0.5, min_event_segs=1)
    with pytest.raises(abi.SegError) as e:
        s.push(torch.zeros((50, 64, 64), dtype=torch.int16, device="cuda"))
    assert e.value.code == abi.SEG_E_NOMODEL
    with pytest.raises(abi.SegError) as e:
        s.set_model(Surrogate(1, 32, 32))
    assert e.value.code == abi.SEG_E_SHAPE


@pytest.fixture(scope="module")
def trained():
    bank = SceneBank(120, device="cuda")
    net, losses = train(steps=250, batch=16, lr=1e-3, bank=bank)
    return net, losses


def test_training_converges(trained):
    net, losses = trained
    first, last = np.mean(losses[:20]), np.mean(losses[-20:])
    assert last < 0.6 * first, (first, last)


def test_gain_over_plain(trained, record_property):
    """Footprint F1 (IoU 0.3) of both detectors against ground truth on two
    held-out videos: dF/F relative to the local total baseline, and the hard
    mode where it is relative to the neuron's own fluorescence (dimmer)."""
    net, _ = trained
    out = {}
    for mode in ("total", "neuron"):
        v, truth = _video(128, 128, 2000, 2000, dff_reference=mode)
        plain = segment_video(v).footprints()["masks"]
        sur = segment_video(v, net=for_frames(net, 128, 128)).footprints()["masks"]
        out[mode] = (oracle.match_f1(plain, truth.masks())["f1"], oracle.match_f1(sur, truth.masks())["f1"])
        record_property(f"f1_{mode}", out[mode])
    print("F1 plain / surrogate:", out)
    assert out["total"][0] >= 0.8          # the plain detector on its own terms
    assert out["total"][1] > 0.0           # the surrogate finds neurons after a short training
