"""GPU rendering of the simulator's videos (input generator only).

The scene (background, footprints, activity traces, flicker) is drawn by
`synth.simulate.draw` exactly as for the CPU simulator, so the ground truth is
the same; the shot and read noise come from a counter-based Philox4x32-10
generator on the GPU (see synth/csrc/render.hip). Frames are rendered straight
into device memory, which is what feeds the training set and the streaming
sessions at recording rate.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libsynth.so")
SRC = os.path.join(HERE, "csrc", "render.hip")


def build() -> str:
    tmp = LIB + ".tmp"
    cmd = ["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O3", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", SRC, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode:
        raise RuntimeError(r.stderr)
    os.replace(tmp, LIB)
    return LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (one HIP runtime per process: torch's)
        if not os.path.exists(LIB):
            raise ImportError(f"{LIB} is missing: build it with synth.gpu.build()")
        _lib = C.CDLL(LIB)
        P = C.c_void_p
        _lib.synth_render.argtypes = [P, P, P, P, C.c_float, C.c_int, C.c_int, C.c_int, C.c_int,
                                      C.c_int, C.c_int, C.c_ulonglong, C.c_float, P, P]
        _lib.synth_render.restype = C.c_int
    return _lib


class GpuScene:
    """A drawn scene resident on the GPU; renders frame ranges on demand."""

    def __init__(self, cfg, seed: int, device="cuda"):
        import torch
        from .simulate import draw
        truth, act, flick, _ = draw(cfg, seed)
        self.cfg, self.seed, self.truth = cfg, seed, truth
        self.device = torch.device(device)
        f = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.float32), device=self.device)
        self.B = f(truth.background)
        fp = truth.footprints.reshape(len(truth.footprints), -1)
        fp = np.where(fp >= 1e-6, fp, 0.0)   # far tails: each pixel visits nearby neurons only
        self.G = f(fp) if len(truth.footprints) else None
        self.act = f(act) if len(truth.footprints) else None
        self.flick = f(flick)

    def render(self, t0: int, t1: int, out=None, stream=None):
        """Frames [t0, t1) as a device int16 tensor [t1 - t0, H, W] (uint16 bytes)."""
        import torch
        lib = _load()
        cfg = self.cfg
        n = t1 - t0
        if out is None:
            out = torch.empty((n, cfg.height, cfg.width), dtype=torch.int16, device=self.device)
        st = (stream or torch.cuda.current_stream(self.device)).cuda_stream
        ptr = lambda t: None if t is None else C.c_void_p(t.data_ptr())
        rc = lib.synth_render(ptr(self.B), ptr(self.G), ptr(self.act), ptr(self.flick),
                              cfg.drift, len(self.truth.footprints), cfg.height, cfg.width, t0, n,
                              cfg.frames, self.seed * 0x9E3779B1 + 0x5EED, cfg.read_noise,
                              C.c_void_p(out.data_ptr()), C.c_void_p(st))
        if rc:
            raise RuntimeError(f"synth_render failed ({rc})")
        return out
