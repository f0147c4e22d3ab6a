"""Streaming server: continuous batching across sessions of different frame
sizes, admission by HBM budget, and each session's result identical alone
and in the mix (bit for bit: every work item runs the same code on the same
data)."""
import numpy as np
import pytest
import torch

from paper_2403_16438_amd import abi, Session
from paper_2403_16438_amd.serve import Batch, Server, SessionSpec
from synth import preset
from synth.gpu import GpuScene

pytestmark = pytest.mark.gpu

BLOCK = 100


def _specs(keep=True):
    mk = lambda name, h, w, seed, fps, arr: SessionSpec(
        name, preset(2, height=h, width=w, frames=4 * BLOCK, n_neurons=3, n_overlap=1, n_blobs=1,
                     n_vessels=(0, 1), min_sep=20.0, edge_margin=10.0),
        seed, fps, arr, blocks=4, block_frames=BLOCK, keep_maps=keep)
    return [mk("a", 64, 64, 7001, 800.0, 0.0), mk("b", 96, 128, 7002, 600.0, 0.05),
            mk("c", 70, 50, 7003, 1000.0, 0.1)]


def _same(r1, r2):
    assert r1["segments"] == r2["segments"] == 8
    assert np.array_equal(r1["S"], r2["S"])
    assert np.array_equal(r1["T"], r2["T"])
    f1, f2 = r1["footprints"], r2["footprints"]
    assert np.array_equal(f1["weights"], f2["weights"])
    assert np.array_equal(f1["activity"], f2["activity"])


@pytest.fixture(scope="module")
def mix():
    srv = Server(hbm_budget=8 << 30, time_scale=20.0)
    out = srv.run(_specs())
    srv.close()
    return out


def test_mix_runs_all_blocks(mix):
    assert mix["sessions"] == 3 and mix["blocks"] == 12
    assert set(mix["results"]) == {"a", "b", "c"}
    assert mix["p50_ms"] is not None and mix["p99_ms"] >= mix["p50_ms"]


@pytest.mark.parametrize("name", ["a", "b", "c"])
def test_alone_equals_mix(mix, name):
    spec = [s for s in _specs() if s.name == name][0]
    spec.arrival = 0.0
    srv = Server(hbm_budget=8 << 30, time_scale=20.0)
    alone = srv.run([spec])
    srv.close()
    _same(alone["results"][name], mix["results"][name])


@pytest.mark.parametrize("name", ["b", "c"])
def test_batched_equals_single_session_push(mix, name):
    spec = [s for s in _specs() if s.name == name][0]
    scene = GpuScene(spec.cfg, spec.seed)
    s = Session(spec.cfg.height, spec.cfg.width, spec.blocks * BLOCK)
    for j in range(spec.blocks):
        s.push(scene.render(j * BLOCK, (j + 1) * BLOCK))
    s.finalize()
    torch.cuda.synchronize()
    ref = dict(segments=s.num_segments, S=s.segment_maps(abi.SEG_MAP_S).cpu().numpy(),
               T=s.segment_maps(abi.SEG_MAP_T).cpu().numpy(), footprints=s.footprints())
    _same(ref, mix["results"][name])


def test_budget_queues_sessions(mix):
    specs = _specs()
    one = max(Server.session_bytes(s) for s in specs)
    srv = Server(hbm_budget=one + 1024, time_scale=20.0)
    out = srv.run(specs)
    srv.close()
    assert out["peak_bytes"] <= one + 1024
    assert max(out["admit_wait_s"].values()) > 0.0      # someone had to wait
    for n in "abc":
        _same(out["results"][n], mix["results"][n])


def test_push_batch_errors_push_nothing():
    b = Batch(4, "cuda")
    s1 = Session(32, 32, 200)
    s2 = Session(32, 32, 100)
    fr = torch.zeros((60, 32, 32), dtype=torch.int16, device="cuda")
    with pytest.raises(abi.SegError) as e:
        b.push([s1, s1], [fr, fr])
    assert e.value.code == abi.SEG_E_INVAL
    b.push([s1, s2], [fr, fr])
    assert s1.num_segments == 1 and s2.num_segments == 1
    with pytest.raises(abi.SegError) as e:
        b.push([s1, s2], [fr, fr])                     # s2 over capacity (120 > 100)
    assert e.value.code == abi.SEG_E_CAPACITY
    assert s1.num_segments == 1                          # nothing pushed for s1 either
    s2.finalize()
    with pytest.raises(abi.SegError) as e:
        b.push([s1, s2], [fr[:10], fr[:10]])
    assert e.value.code == abi.SEG_E_STATE
    torch.cuda.synchronize()
    b.close()
