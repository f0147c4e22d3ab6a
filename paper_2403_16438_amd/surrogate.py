"""Learned surrogate detector (include/seg_nn.h): binding and trainer.

PyTorch provides the parameter and workspace memory and the stream; the
network's forward, loss, backward and RMSProp update run in libseg.so.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import abi, lifetime

LAYERS = ["t1", "t2", "t3", "e1a", "e1b", "e2a", "e2b", "e3a", "e3b", "u2", "d2a", "d2b", "u1",
          "d1a", "d1b", "out"]


def param_count() -> int:
    n = C.c_size_t()
    abi.check(abi.lib.seg_nn_param_count(C.byref(n)), "seg_nn_param_count")
    return n.value


def param_layout():
    out = []
    for i, name in enumerate(LAYERS):
        r, c = C.c_uint32(), C.c_uint32()
        wo, bo = C.c_size_t(), C.c_size_t()
        abi.check(abi.lib.seg_nn_param_layout(i, C.byref(r), C.byref(c), C.byref(wo), C.byref(bo)),
                  "seg_nn_param_layout")
        out.append((name, r.value, c.value, wo.value, bo.value))
    return out


def he_init(seed: int) -> np.ndarray:
    """He-normal weights (fan-in = weight columns), zero biases; FP32."""
    rng = np.random.default_rng(seed)
    theta = np.zeros(param_count(), np.float32)
    for name, r, c, wo, bo in param_layout():
        theta[wo:wo + r * c] = rng.standard_normal(r * c) * np.sqrt(2.0 / c)
    return theta


class Surrogate:
    def __init__(self, batch: int, height: int, width: int, theta=None, device="cuda"):
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.B, self.H, self.W = batch, height, width
        nb = C.c_size_t()
        abi.check(abi.lib.seg_nn_workspace_bytes(batch, height, width, C.byref(nb)), "seg_nn_workspace_bytes")
        self.params = torch.zeros(param_count(), dtype=torch.float32, device=self.device)
        self.ws = torch.empty(nb.value + 256, dtype=torch.uint8, device=self.device)
        h = C.c_void_p()
        abi.check(abi.lib.seg_nn_create(batch, height, width, C.c_void_p(self.params.data_ptr()),
                                        C.c_void_p((self.ws.data_ptr() + 255) & ~255), nb.value, C.byref(h)),
                  "seg_nn_create")
        self.handle = h
        lifetime.track(self)
        self.load(he_init(0) if theta is None else theta)

    def _st(self):
        return C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def load(self, theta) -> None:
        self.params.copy_(torch.as_tensor(np.asarray(theta, np.float32)))
        abi.check(abi.lib.seg_nn_sync_weights(self.handle, self._st()), "seg_nn_sync_weights")

    def theta(self) -> np.ndarray:
        return self.params.cpu().numpy()

    def forward(self, frames: torch.Tensor) -> torch.Tensor:
        """frames: 16-bit [b, 50, H, W] device tensor -> probabilities [b, H, W]."""
        b = frames.shape[0]
        out = torch.empty((b, self.H, self.W), dtype=torch.float32, device=self.device)
        abi.check(abi.lib.seg_nn_forward(self.handle, C.c_void_p(frames.data_ptr()), b,
                                         C.c_void_p(out.data_ptr()), self._st()), "seg_nn_forward")
        return out

    def logits(self) -> torch.Tensor:
        out = torch.empty((self.B, self.H, self.W), dtype=torch.float32, device=self.device)
        abi.check(abi.lib.seg_nn_logits(self.handle, C.c_void_p(out.data_ptr()), self._st()), "seg_nn_logits")
        return out

    def backward(self, frames: torch.Tensor, labels: torch.Tensor, want_grad=False):
        b = frames.shape[0]
        loss = C.c_float()
        g = torch.empty_like(self.params) if want_grad else None
        abi.check(abi.lib.seg_nn_backward(self.handle, C.c_void_p(frames.data_ptr()),
                                          C.c_void_p(labels.data_ptr()), b,
                                          C.c_void_p(g.data_ptr()) if g is not None else None,
                                          C.byref(loss), self._st()), "seg_nn_backward")
        return loss.value, g

    def step(self, lr=1e-3, rho=0.9, eps=1e-7) -> None:
        abi.check(abi.lib.seg_nn_step(self.handle, lr, rho, eps, self._st()), "seg_nn_step")

    def close(self):
        if getattr(self, "handle", None) is not None:
            abi.lib.seg_nn_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:   # at interpreter exit the lifetime module may already be torn down
            if lifetime.released_by_finalizer():
                self.close()
        except Exception:
            pass


def gemm_test(A: torch.Tensor, B: torch.Tensor, a_trans=False, b_trans=False, splits=1) -> torch.Tensor:
    M = A.shape[1] if a_trans else A.shape[0]
    K = A.shape[0] if a_trans else A.shape[1]
    N = B.shape[0] if b_trans else B.shape[1]
    Cm = torch.empty((M, N), dtype=torch.float32, device=A.device)
    scratch = torch.empty(max(1, splits) * M * N, dtype=torch.float32, device=A.device)
    st = torch.cuda.current_stream(A.device).cuda_stream
    abi.check(abi.lib.seg_nn_gemm_test(C.c_void_p(A.data_ptr()), int(a_trans), C.c_void_p(B.data_ptr()),
                                       int(b_trans), C.c_void_p(Cm.data_ptr()), M, N, K, splits,
                                       C.c_void_p(scratch.data_ptr()), C.c_void_p(st)), "seg_nn_gemm_test")
    return Cm
