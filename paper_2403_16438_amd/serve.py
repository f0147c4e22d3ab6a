"""Streaming server: concurrent recording sessions with continuous batching.

* Admission by HBM budget: the budget is one device allocation made when the
  server starts (an arena), carved first-fit into session workspaces and
  frame-block staging buffers, so that nothing calls the device allocator
  while sessions stream. A session is admitted when its workspace plus its
  two staging buffers fit in the arena; otherwise it waits in a FIFO queue
  and is admitted when a finishing session returns its memory.
* Each admitted session keeps its running state on the device (the library
  workspace). Its camera releases one block of frames every
  block_frames / fps seconds; the block is rendered into a staging buffer on
  a camera stream (standing in for the frame grabber's DMA).
* Continuous batching: every tick gathers the blocks that are ready across
  all sessions and pushes them with one graph replay of the batched streaming
  kernel on the compute stream (`seg_push_batch`); blocks that become ready
  while a batch runs join the next one.
* A session whose last block has been pushed is finalized on a worker thread
  and its own stream, overlapping the other sessions' streaming work; its
  memory returns to the budget afterwards.
* Latency of a block = completion of the batch that carried it minus the
  block's release time; p50 / p99 are reported with the aggregate frames/s.
"""
from __future__ import annotations

import time
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np
import torch

from . import abi, lifetime
from .session import Session


class Arena:
    """One device allocation carved into 256-byte aligned pieces (first fit,
    neighbouring free pieces merged on release)."""

    def __init__(self, nbytes: int, device):
        self.nbytes = (int(nbytes) + 255) & ~255
        self.buf = torch.empty(self.nbytes, dtype=torch.uint8, device=device)
        self.free = [(0, self.nbytes)]          # sorted (offset, size)

    def alloc(self, n: int):
        n = (int(n) + 255) & ~255
        for k, (o, sz) in enumerate(self.free):
            if sz >= n:
                if sz == n:
                    self.free.pop(k)
                else:
                    self.free[k] = (o + n, sz - n)
                return o, n
        return None

    def release(self, o: int, n: int) -> None:
        self.free.append((o, n))
        self.free.sort()
        merged = []
        for fo, fs in self.free:
            if merged and merged[-1][0] + merged[-1][1] == fo:
                merged[-1] = (merged[-1][0], merged[-1][1] + fs)
            else:
                merged.append((fo, fs))
        self.free = merged

    def view(self, o: int, n: int) -> torch.Tensor:
        return self.buf[o:o + n]


class Batch:
    """A seg_batch object with its device slot table in torch memory."""

    def __init__(self, max_slots: int, device):
        self.device = torch.device(device)
        nbytes = abi.seg_batch_bytes(max_slots)
        with torch.cuda.device(self.device):
            self.table = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            self.handle = abi.seg_batch_create(max_slots, (self.table.data_ptr() + 255) & ~255, nbytes)
        lifetime.track(self)
        self.max_slots = max_slots

    def push(self, sessions, frames, stream=None) -> None:
        st = (stream or torch.cuda.current_stream(self.device)).cuda_stream
        abi.seg_push_batch(self.handle, [s.handle for s in sessions], [f.data_ptr() for f in frames],
                           [f.shape[0] for f in frames], st)

    def close(self) -> None:
        if getattr(self, "handle", None) is not None:
            abi.seg_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:   # at interpreter exit the lifetime module may already be torn down
            if lifetime.released_by_finalizer():
                self.close()
        except Exception:
            pass


@dataclass
class SessionSpec:
    name: str
    cfg: object            # synth.SimConfig (frame size, frames, scene)
    seed: int
    fps: float
    arrival: float         # seconds after the server starts
    blocks: int
    block_frames: int = 500
    keep_maps: bool = False


@dataclass
class _Live:
    spec: SessionSpec
    sess: Session
    scene: object
    staging: list
    piece: tuple               # (offset, bytes) in the arena
    admitted: float
    rendered: int = 0          # blocks rendered into staging
    pushed: int = 0            # blocks pushed
    completed: int = 0
    cam_events: dict = field(default_factory=dict)
    last_event: object = None
    finalizing: object = None


class Server:
    def __init__(self, hbm_budget: int, device="cuda", max_batch: int = 16, time_scale: float = 1.0):
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.budget = int(hbm_budget)
        self.time_scale = float(time_scale)
        self.batch = Batch(max_batch, self.device)
        self.max_batch = max_batch
        self.compute = torch.cuda.Stream(self.device)
        self.camera = torch.cuda.Stream(self.device)
        self.finals = torch.cuda.Stream(self.device)
        self.arena = Arena(self.budget, self.device)

    @staticmethod
    def workspace_bytes(spec: SessionSpec) -> int:
        c = spec.cfg
        cfg = abi.seg_default_config(c.height, c.width, spec.blocks * spec.block_frames)
        return (abi.seg_workspace_bytes(cfg) + 256 + 255) & ~255

    @staticmethod
    def staging_bytes(spec: SessionSpec) -> int:
        return (spec.block_frames * spec.cfg.height * spec.cfg.width * 2 + 255) & ~255

    @classmethod
    def session_bytes(cls, spec: SessionSpec) -> int:
        return cls.workspace_bytes(spec) + 2 * cls.staging_bytes(spec)

    def run(self, specs, on_block=None) -> dict:
        from synth.gpu import GpuScene
        specs = sorted(specs, key=lambda s: s.arrival)
        for s in specs:
            if self.session_bytes(s) > self.arena.nbytes:
                raise ValueError(f"session {s.name} alone exceeds the HBM budget")
        # the cameras (synthetic scenes rendering frames on the GPU) exist
        # before the server starts, as the recording hardware would
        scenes = {sp.name: GpuScene(sp.cfg, sp.seed, self.device) for sp in specs}
        torch.cuda.synchronize(self.device)
        t0 = time.perf_counter()
        now = lambda: (time.perf_counter() - t0) * self.time_scale   # recording time (s)
        pending = list(specs)
        queue: list = []
        live: dict = {}
        used = 0
        inflight = []       # (event, [(live, block index)])
        lat = []            # seconds of wall time
        results = {}
        admit_wait = {}
        peak_used = 0
        nbatches = 0
        nblocks = 0
        frames_done = 0
        pool = ThreadPoolExecutor(1)
        admit_s = []        # wall seconds spent admitting each session
        gaps = []           # (gap seconds, recording time) of the longest loop iterations
        t_prev = time.perf_counter()

        def release_time(lv, j):
            return lv.spec.arrival + (j + 1) * lv.spec.block_frames / lv.spec.fps

        fin_log = []        # (recording time at start, wall seconds) of each finalize

        def finalize(lv):
            tf = time.perf_counter()
            tstart = now()
            try:
                return _finalize(lv)
            finally:
                fin_log.append((tstart, time.perf_counter() - tf))

        def _finalize(lv):
            with torch.cuda.stream(self.finals):
                self.finals.wait_event(lv.last_event)
                lv.sess.finalize(self.finals)
                out = dict(footprints=lv.sess.footprints(), segments=lv.sess.num_segments)
                if lv.spec.keep_maps:
                    maps = lambda k: lv.sess.segment_maps(k).cpu().numpy()
                    out.update(S=maps(abi.SEG_MAP_S), T=maps(abi.SEG_MAP_T), D=maps(abi.SEG_MAP_D),
                               P=maps(abi.SEG_MAP_P), B=maps(abi.SEG_MAP_B) > 0.5,
                               sigma=lv.sess.image(abi.SEG_IMG_NOISE),
                               count=lv.sess.image(abi.SEG_IMG_EVENT_COUNT),
                               nb=lv.sess.image(abi.SEG_IMG_MASK_COUNT),
                               labels=lv.sess.image(abi.SEG_IMG_LABELS))
                torch.cuda.current_stream(self.device).synchronize()
            return out

        while pending or queue or live:
            t_it = time.perf_counter()
            if t_it - t_prev > 0.02:
                gaps.append((t_it - t_prev, now()))
            t_prev = t_it
            tnow = now()
            while pending and pending[0].arrival <= tnow:
                queue.append(pending.pop(0))
            # admission (FIFO, by HBM budget)
            while queue:
                sp = queue[0]
                piece = self.arena.alloc(self.session_bytes(sp))
                if piece is None:
                    break
                queue.pop(0)
                ta = time.perf_counter()
                o, n = piece
                wsb, sb = self.workspace_bytes(sp), self.staging_bytes(sp)
                shape = (sp.block_frames, sp.cfg.height, sp.cfg.width)
                staging = [self.arena.view(o + wsb + k * sb, sb)[:2 * shape[0] * shape[1] * shape[2]]
                           .view(torch.int16).view(shape) for k in range(2)]
                sess = Session(sp.cfg.height, sp.cfg.width, sp.blocks * sp.block_frames, self.device,
                               workspace=self.arena.view(o, wsb))
                live[sp.name] = _Live(sp, sess, scenes[sp.name], staging, piece, tnow)
                admit_s.append(time.perf_counter() - ta)
                admit_wait[sp.name] = tnow - sp.arrival
                used += n
                peak_used = max(peak_used, used)
            # camera: render released blocks (two staging buffers per session)
            for lv in live.values():
                while (lv.rendered < lv.spec.blocks and lv.rendered - lv.completed < 2
                       and release_time(lv, lv.rendered) <= tnow):
                    j = lv.rendered
                    buf = lv.staging[j % 2]
                    with torch.cuda.stream(self.camera):
                        lv.scene.render(j * lv.spec.block_frames, (j + 1) * lv.spec.block_frames, out=buf,
                                        stream=self.camera)
                        ev = torch.cuda.Event()
                        ev.record(self.camera)
                    lv.cam_events[j] = ev
                    lv.rendered += 1
            # continuous batching: one push for every ready block (one per session)
            ready = [lv for lv in live.values() if lv.pushed < lv.rendered and lv.finalizing is None]
            if ready:
                ready = ready[: self.max_batch]
                for lv in ready:
                    self.compute.wait_event(lv.cam_events.pop(lv.pushed))
                with torch.cuda.stream(self.compute):
                    self.batch.push([lv.sess for lv in ready], [lv.staging[lv.pushed % 2] for lv in ready],
                                    self.compute)
                    ev = torch.cuda.Event()
                    ev.record(self.compute)
                inflight.append((ev, [(lv, lv.pushed) for lv in ready]))
                for lv in ready:
                    lv.pushed += 1
                    lv.last_event = ev
                nbatches += 1
            # completions
            still = []
            for ev, items in inflight:
                if ev.query():
                    tdone = time.perf_counter()
                    for lv, j in items:
                        rel_wall = t0 + release_time(lv, j) / self.time_scale
                        lat.append(tdone - rel_wall)
                        lv.completed += 1
                        nblocks += 1
                        frames_done += lv.spec.block_frames
                        if on_block:
                            on_block(lv.spec.name, j)
                else:
                    still.append((ev, items))
            inflight = still
            # finished sessions: finalize on the worker, then release memory
            for name, lv in list(live.items()):
                if lv.finalizing is None and lv.completed == lv.spec.blocks:
                    lv.finalizing = pool.submit(finalize, lv)
                elif lv.finalizing is not None and lv.finalizing.done():
                    results[name] = lv.finalizing.result()
                    lv.sess.close()
                    self.arena.release(*lv.piece)
                    used -= lv.piece[1]
                    del live[name]
            if not ready:
                time.sleep(0.0005)
        pool.shutdown()
        torch.cuda.synchronize(self.device)
        wall = time.perf_counter() - t0
        lat_ms = np.array(lat) * 1e3
        return dict(results=results, sessions=len(specs), blocks=nblocks, batches=nbatches,
                    mean_batch=nblocks / max(nbatches, 1), frames=frames_done, wall_s=wall,
                    frames_per_s=frames_done / wall,
                    p50_ms=float(np.percentile(lat_ms, 50)) if len(lat) else None,
                    p99_ms=float(np.percentile(lat_ms, 99)) if len(lat) else None,
                    max_ms=float(lat_ms.max()) if len(lat) else None,
                    admit_wait_s=admit_wait, peak_bytes=peak_used, budget=self.budget,
                    admit_s=admit_s, loop_gaps=sorted(gaps, reverse=True)[:10], finalizes=fin_log)

    def close(self):
        self.batch.close()
