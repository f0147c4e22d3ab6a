"""Motion correction (include/seg_mc.h) over torch device tensors.

Argument marshalling only: the template, scores, motion and corrected frames
are computed by libseg.so.
"""
from __future__ import annotations

import numpy as np
import torch

from . import abi, lifetime


class MotionCorrector:
    def __init__(self, height: int, width: int, device=None, **overrides):
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.cfg = abi.seg_mc_default_config(height, width)
        for k, v in overrides.items():
            setattr(self.cfg, k, v)
        with torch.cuda.device(self.device):
            self.nbytes = abi.seg_mc_workspace_bytes(self.cfg)
            self.workspace = torch.empty(self.nbytes + 256, dtype=torch.uint8, device=self.device)
            aligned = (self.workspace.data_ptr() + 255) & ~255
            self.handle = abi.seg_mc_create(self.cfg, aligned, self.nbytes)
        lifetime.track(self)
        self.H, self.W = height, width
        self.n_patches, self.n_vectors = abi.seg_mc_layout(self.handle)

    def _check(self, frames: torch.Tensor) -> None:
        if frames.device != self.device or not frames.is_contiguous():
            raise ValueError("frames must be a contiguous tensor on the corrector's device")
        if frames.dtype not in (torch.int16, torch.uint16) or tuple(frames.shape[1:]) != (self.H, self.W):
            raise ValueError("frames must be 16-bit [n, H, W]")

    def _stream(self, stream):
        return (stream or torch.cuda.current_stream(self.device)).cuda_stream

    def set_template(self, frames: torch.Tensor, stream=None) -> None:
        """Template = rounded mean of `frames` (normally the first 50)."""
        self._check(frames)
        abi.seg_mc_set_template(self.handle, frames.data_ptr(), frames.shape[0], self._stream(stream))

    def template(self) -> np.ndarray:
        out = np.zeros((self.H, self.W), np.uint16)
        abi.seg_mc_get_template(self.handle, out)
        return out

    def estimate(self, frames: torch.Tensor, scores: bool = False, stream=None):
        """Motion (my, mx) per frame as int32 [n, 2]; with scores=True also
        the per-vector scores [n, V] (float64)."""
        self._check(frames)
        n = frames.shape[0]
        motion = torch.empty((n, 2), dtype=torch.int32, device=self.device)
        sc = torch.empty((n, self.n_vectors), dtype=torch.float64, device=self.device) if scores else None
        abi.seg_mc_estimate(self.handle, frames.data_ptr(), n, motion.data_ptr(),
                            sc.data_ptr() if sc is not None else None, self._stream(stream))
        return (motion, sc) if scores else motion

    def estimate_static(self, frames: torch.Tensor, motion: torch.Tensor, scores: torch.Tensor | None = None,
                        stream=None) -> None:
        """seg_mc_estimate_static: as estimate(), into caller-given outputs
        (int32 [n, 2] and optionally float64 [n, V]), with the partial sums in
        the library's fixed device array; n <= SEG_MC_STATIC_MAX_FRAMES."""
        self._check(frames)
        n = frames.shape[0]
        if (motion.dtype != torch.int32 or tuple(motion.shape) != (n, 2) or not motion.is_contiguous()
                or motion.device != self.device):
            raise ValueError("motion must be contiguous int32 [n, 2] on the corrector's device")
        if scores is not None and (scores.dtype != torch.float64 or tuple(scores.shape) != (n, self.n_vectors)
                                   or not scores.is_contiguous() or scores.device != self.device):
            raise ValueError("scores must be contiguous float64 [n, V] on the corrector's device")
        abi.seg_mc_estimate_static(self.handle, frames.data_ptr(), n, motion.data_ptr(),
                                   scores.data_ptr() if scores is not None else None, self._stream(stream))

    def apply(self, frames: torch.Tensor, motion: torch.Tensor, out: torch.Tensor | None = None,
              stream=None) -> torch.Tensor:
        self._check(frames)
        if motion.dtype != torch.int32 or tuple(motion.shape) != (frames.shape[0], 2) or not motion.is_contiguous():
            raise ValueError("motion must be contiguous int32 [n, 2]")
        if out is None:
            out = torch.empty_like(frames)
        self._check(out)
        abi.seg_mc_apply(self.handle, frames.data_ptr(), frames.shape[0], motion.data_ptr(), out.data_ptr(),
                         self._stream(stream))
        return out

    def correct(self, frames: torch.Tensor, stream=None):
        """Estimate and apply: (corrected frames, motion)."""
        motion = self.estimate(frames, stream=stream)
        return self.apply(frames, motion, stream=stream), motion

    def close(self) -> None:
        if getattr(self, "handle", None):
            abi.lib.seg_mc_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:   # at interpreter exit the lifetime module may already be torn down
            if lifetime.released_by_finalizer():
                self.close()
        except Exception:
            pass
