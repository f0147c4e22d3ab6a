"""Checkpoint and resume through the C ABI (seg_export_state /
seg_import_state): a recording interrupted mid-segment and resumed in a new
session gives bit-identical results to an uninterrupted one; states are
checked against the configuration and the session's progress."""
import numpy as np
import pytest
import torch

from paper_2403_16438_amd import Session, abi, to_device_frames
from synth import preset, simulate

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def video():
    v, _ = simulate(preset(1), 0)
    return to_device_frames(v, torch.device("cuda:0"))


def _outputs(s):
    return dict(T=s.segment_maps(abi.SEG_MAP_T).cpu().numpy(), S=s.segment_maps(abi.SEG_MAP_S).cpu().numpy(),
                corr=s.image(abi.SEG_IMG_CORR), labels=s.image(abi.SEG_IMG_LABELS), fp=s.footprints())


@pytest.mark.parametrize("cut", [437, 500, 49])
def test_resume_is_bit_identical(video, cut):
    whole = Session(64, 64, 1000)
    whole.push(video)
    whole.finalize()
    a = Session(64, 64, 1000)
    a.push(video[:cut])
    state = a.export_state()
    b = Session(64, 64, 1000)
    b.import_state(state)
    b.push(video[cut:])
    b.finalize()
    x, y = _outputs(whole), _outputs(b)
    for k in ("T", "S", "corr", "labels"):
        assert np.array_equal(x[k], y[k]), k
    assert np.array_equal(x["fp"]["weights"], y["fp"]["weights"])
    assert np.array_equal(x["fp"]["activity"], y["fp"]["activity"])


def test_state_checks(video):
    a = Session(64, 64, 1000)
    a.push(video[:120])
    state = a.export_state()
    other = Session(64, 64, 1000, event_z=4.0)
    with pytest.raises(abi.SegError) as e:
        other.import_state(state)
    assert e.value.code == abi.SEG_E_INVAL
    used = Session(64, 64, 1000)
    used.push(video[:10])
    with pytest.raises(abi.SegError) as e:
        used.import_state(state)
    assert e.value.code == abi.SEG_E_STATE
    fresh = Session(64, 64, 1000)
    with pytest.raises(abi.SegError) as e:
        fresh.import_state(state[:-1])
    assert e.value.code == abi.SEG_E_CAPACITY
    bad = state.copy()
    bad[0] ^= 0xFF
    with pytest.raises(abi.SegError) as e:
        fresh.import_state(bad)
    assert e.value.code == abi.SEG_E_INVAL
    a.finalize()
    with pytest.raises(abi.SegError) as e:
        a.export_state()
    assert e.value.code == abi.SEG_E_STATE
