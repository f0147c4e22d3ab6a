"""Session: a recording being segmented on one GPU.

PyTorch provides the device memory (the workspace and frame buffers) and the
stream; every step of the segmentation runs in libseg.so through `abi`.
"""
from __future__ import annotations

import numpy as np
import torch

from . import abi, lifetime


def to_device_frames(video: np.ndarray, device="cuda") -> torch.Tensor:
    """uint16 [n, H, W] host array -> contiguous device tensor holding the
    same bytes (int16 view: torch has no full uint16 support)."""
    v = np.ascontiguousarray(video, dtype=np.uint16)
    return torch.from_numpy(v.view(np.int16)).to(device)


class Session:
    def __init__(self, height: int, width: int, max_frames: int, device=None,
                 workspace: torch.Tensor | None = None, **overrides):
        dev = torch.device(device or "cuda")
        if dev.type != "cuda":
            raise ValueError("Session needs a GPU device")
        if dev.index is None:
            dev = torch.device("cuda", torch.cuda.current_device())
        self.device = dev
        self.cfg = abi.seg_default_config(height, width, max_frames)
        for k, v in overrides.items():
            if not hasattr(self.cfg, k):
                raise KeyError(k)
            setattr(self.cfg, k, v)
        self.nbytes = abi.seg_workspace_bytes(self.cfg)
        with torch.cuda.device(self.device):
            if workspace is not None and workspace.numel() >= self.nbytes + 256:
                self.workspace = workspace
            else:
                self.workspace = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=self.device)
            base = self.workspace.data_ptr()
            aligned = (base + 255) & ~255
            self.handle = abi.seg_create(self.cfg, aligned, self.nbytes)
        lifetime.track(self)
        self.H, self.W = height, width

    def set_model(self, net) -> None:
        """Attach a Surrogate (SEG_DET_SURROGATE) or a SummaryUNet of 64 x 64
        patches (SEG_DET_UNET), before the first push."""
        abi.check(abi.lib.seg_set_model(self.handle, net.handle), "seg_set_model")
        self.net = net   # keep it alive while the session pushes

    # -- streaming
    def push(self, frames: torch.Tensor, stream: torch.cuda.Stream | None = None) -> None:
        if frames.device != self.device or not frames.is_contiguous():
            raise ValueError("frames must be a contiguous tensor on the session's device")
        if frames.dtype not in (torch.int16, torch.uint16) or tuple(frames.shape[1:]) != (self.H, self.W):
            raise ValueError("frames must be 16-bit [n, H, W]")
        st = (stream or torch.cuda.current_stream(self.device)).cuda_stream
        abi.seg_push_frames(self.handle, frames.data_ptr(), frames.shape[0], st)

    def finalize(self, stream: torch.cuda.Stream | None = None) -> None:
        st = (stream or torch.cuda.current_stream(self.device)).cuda_stream
        abi.seg_finalize(self.handle, st)

    @property
    def num_segments(self) -> int:
        return abi.seg_num_segments(self.handle)

    # -- results
    def footprints(self) -> dict:
        n = abi.seg_get_footprints(self.handle, 0, None, None, None, None)
        K = self.num_segments
        w = np.zeros((n, self.H, self.W), np.float32)
        m = np.zeros((n, self.H, self.W), np.uint8)
        a = np.zeros((n, K), np.float32)
        c = np.zeros(n, np.int32)
        abi.seg_get_footprints(self.handle, n, w, m, a, c)
        return dict(weights=w, masks=m.astype(bool), activity=a, component=c)

    def traces(self, frames: torch.Tensor, out: torch.Tensor | None = None,
               stream: torch.cuda.Stream | None = None) -> torch.Tensor:
        """Mean intensity of every footprint's mask in each frame (seg_extract_traces).

        frames: contiguous 16-bit [n, H, W] on the session's device. `out`, if
        given, is a float32 [N, n] view whose rows may be strided (a column
        slice of a [N, T] array); else a new [N, n] tensor is returned."""
        if frames.device != self.device or not frames.is_contiguous():
            raise ValueError("frames must be a contiguous tensor on the session's device")
        if frames.dtype not in (torch.int16, torch.uint16) or tuple(frames.shape[1:]) != (self.H, self.W):
            raise ValueError("frames must be 16-bit [n, H, W]")
        n = abi.seg_get_footprints(self.handle, 0, None, None, None, None)
        if out is None:
            out = torch.empty((n, frames.shape[0]), dtype=torch.float32, device=self.device)
        if (out.dtype != torch.float32 or out.device != self.device or tuple(out.shape) != (n, frames.shape[0])
                or (out.numel() and out.stride(1) != 1)):
            raise ValueError("out must be float32 [N, n] on the session's device, unit column stride")
        st = (stream or torch.cuda.current_stream(self.device)).cuda_stream
        ld = out.stride(0) if n > 1 else frames.shape[0]
        abi.seg_extract_traces(self.handle, frames.data_ptr(), frames.shape[0], out.data_ptr(), ld, st)
        return out

    def export_state(self, stream: torch.cuda.Stream | None = None) -> np.ndarray:
        """Checkpoint of an open session (host bytes, seg_export_state)."""
        st = (stream or torch.cuda.current_stream(self.device)).cuda_stream
        return abi.seg_export_state(self.handle, st)

    def import_state(self, state: np.ndarray, stream: torch.cuda.Stream | None = None) -> None:
        """Resume from a checkpoint (fresh session, same configuration)."""
        st = (stream or torch.cuda.current_stream(self.device)).cuda_stream
        abi.seg_import_state(self.handle, np.ascontiguousarray(state, np.uint8), st)

    def profile(self) -> dict:
        """Device times (HIP events) and NMF work of the last finalize."""
        return abi.seg_get_profile(self.handle)

    def image(self, kind: int) -> np.ndarray:
        dt = np.float32 if kind in (abi.SEG_IMG_MEAN, abi.SEG_IMG_CORR, abi.SEG_IMG_NOISE) else np.int32
        out = np.zeros((self.H, self.W), dt)
        abi.seg_get_image(self.handle, kind, out)
        return out

    def segment_maps(self, kind: int, first: int = 0, count: int | None = None) -> torch.Tensor:
        count = self.num_segments - first if count is None else count
        out = torch.empty((count, self.H, self.W), dtype=torch.float32, device=self.device)
        st = torch.cuda.current_stream(self.device).cuda_stream
        abi.seg_get_segment_maps(self.handle, kind, first, count, out.data_ptr(), st)
        return out

    def load_summaries(self, T, S, D, U=None, P=None) -> None:
        f = lambda a: None if a is None else np.ascontiguousarray(a, np.float32)
        T = f(T)
        abi.seg_load_summaries(self.handle, T.shape[0], T, f(S), f(D), f(U), f(P))

    def close(self) -> None:
        if getattr(self, "handle", None) is not None:
            abi.seg_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:   # at interpreter exit the lifetime module may already be torn down
            if lifetime.released_by_finalizer():
                self.close()
        except Exception:
            pass


def segment_video(video: np.ndarray, block: int | None = None, net=None, **overrides) -> Session:
    """Push a host uint16 video [T, H, W] (in blocks of `block` frames) and
    finalize. Returns the finalized session. With `net` the learned detector
    is used: a Surrogate reads the frames (events at probability >= 0.5,
    c_min = 2), a SummaryUNet the summary patches (events at probability
    >= 0.7, c_min = 3, the setting with the best F1 on validation recordings
    of the training kind). Keyword overrides replace these."""
    T, H, W = video.shape
    if net is not None:
        from .unet import SummaryUNet
        if isinstance(net, SummaryUNet):
            learned = dict(detector=abi.SEG_DET_UNET, event_z=0.7, min_event_segs=3)
        else:
            learned = dict(detector=abi.SEG_DET_SURROGATE, event_z=0.5, min_event_segs=2)
        overrides = dict(learned, **overrides)
    s = Session(H, W, max(T, 50), **overrides)
    if net is not None:
        s.set_model(net)
    block = block or T
    for t0 in range(0, T, block):
        s.push(to_device_frames(video[t0:t0 + block], s.device))
    s.finalize()
    torch.cuda.synchronize(s.device)
    return s
