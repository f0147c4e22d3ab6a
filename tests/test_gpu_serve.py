"""Streaming server: continuous batching across sessions of different frame
sizes, admission by HBM budget, each session's result identical alone and in
the mix (bit for bit: every work item runs the same code on the same data),
and every served session against the FP64 oracle run on its video: S
bit-exact, T, D and the noise scale within 1e-4, event counts bit-exact
outside the threshold window, and the footprint reconstruction by stage
isolation (counts, kept masks, n_b and labels bit-exact, footprints at
IoU >= 0.99). The last check uses the four frame sizes of the 16-session
workload (128 x 128, 256 x 256, 512 x 128, 512 x 512)."""
import numpy as np
import pytest
import torch

from paper_2403_16438_amd import abi, Session
from paper_2403_16438_amd.serve import Batch, Server, SessionSpec
import oracle
from synth import preset
from synth.gpu import GpuScene

from parity import check_against_full_oracle, check_finalize_stage_isolation, params_from_config

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


def _served_against_oracle(spec, res):
    """One served session (results with keep_maps) against the oracle run on
    the frames its camera rendered."""
    frames = spec.blocks * spec.block_frames
    video = GpuScene(spec.cfg, spec.seed).render(0, frames).cpu().numpy().view(np.uint16)
    cfg = abi.seg_default_config(spec.cfg.height, spec.cfg.width, frames)
    prm = params_from_config(cfg)
    ref = oracle.segment(video, prm)
    g = dict(res, fp=res["footprints"])
    in_window = check_against_full_oracle(g, ref, prm)
    check_finalize_stage_isolation(g, prm)
    return ref, in_window


@pytest.mark.parametrize("name", ["a", "b", "c"])
def test_served_session_against_oracle(mix, name):
    spec = [s for s in _specs() if s.name == name][0]
    _served_against_oracle(spec, mix["results"][name])


def test_workload_frame_sizes_against_oracle():
    """One served session of each frame size of the 16-session workload, two
    500-frame blocks each, admitted and batched together."""
    sizes = [(128, 128), (256, 256), (512, 128), (512, 512)]
    specs = []
    for k, (h, w) in enumerate(sizes):
        scale = h * w / 65536.0                   # the workload's density scaling
        n = max(2, int(round(30 * scale)))
        cfg = preset(5, height=h, width=w, frames=1000, n_neurons=n, n_overlap=int(round(0.2 * n)),
                     n_blobs=max(1, int(round(5 * scale))))
        specs.append(SessionSpec(f"s{h}x{w}", cfg, 5100 + k, 1000.0, 0.0, blocks=2, block_frames=500,
                                 keep_maps=True))
    srv = Server(hbm_budget=24 << 30, time_scale=25.0)
    out = srv.run(specs)
    srv.close()
    assert out["blocks"] == 8 and set(out["results"]) == {s.name for s in specs}
    assert out["mean_batch"] > 1.0          # blocks of different sessions shared launches
    for sp in specs:
        ref, in_window = _served_against_oracle(sp, out["results"][sp.name])
        print(sp.name, "footprints", len(ref.footprints), "pixels with a window decision", in_window)


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
