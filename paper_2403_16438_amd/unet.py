"""The paper's detector input (include/seg_nn.h, seg_nn_st_*): a U-Net on
64 x 64 patches of a segment's summary images (S_i, T_i), merged over the
frame by weighted averaging. Binding only: the patches, normalisation,
network, loss, gradients, update and merge run in libseg.so.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import abi, lifetime
from .surrogate import LAYERS


def param_count() -> int:
    n = C.c_size_t()
    abi.check(abi.lib.seg_nn_st_param_count(C.byref(n)), "seg_nn_st_param_count")
    return n.value


def param_layout():
    """(name, rows, cols, w_offset, b_offset) of the non-empty layers."""
    out = []
    for i, name in enumerate(LAYERS):
        r, c = C.c_uint32(), C.c_uint32()
        wo, bo = C.c_size_t(), C.c_size_t()
        abi.check(abi.lib.seg_nn_st_param_layout(i, C.byref(r), C.byref(c), C.byref(wo), C.byref(bo)),
                  "seg_nn_st_param_layout")
        if r.value:
            out.append((name, r.value, c.value, wo.value, bo.value))
    return out


def he_init(seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    theta = np.zeros(param_count(), np.float32)
    for name, r, c, wo, bo in param_layout():
        theta[wo:wo + r * c] = rng.standard_normal(r * c) * np.sqrt(2.0 / c)
    return theta


def patch_count(height: int, width: int) -> int:
    n = C.c_uint32()
    abi.check(abi.lib.seg_nn_st_patch_count(height, width, C.byref(n)), "seg_nn_st_patch_count")
    return n.value


def _st(device):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def patches(S: torch.Tensor, T: torch.Tensor) -> torch.Tensor:
    """[n_patch, 2, 64, 64] patches of device maps S, T [H, W] (float32)."""
    H, W = S.shape
    out = torch.empty((patch_count(H, W), 2, 64, 64), dtype=torch.float32, device=S.device)
    abi.check(abi.lib.seg_nn_st_patches(C.c_void_p(S.data_ptr()), C.c_void_p(T.data_ptr()), H, W,
                                        C.c_void_p(out.data_ptr()), _st(S.device)), "seg_nn_st_patches")
    return out


def merge(prob: torch.Tensor, height: int, width: int) -> torch.Tensor:
    """[H, W] weighted mean of patch probabilities [n_patch, 64, 64]."""
    out = torch.empty((height, width), dtype=torch.float32, device=prob.device)
    abi.check(abi.lib.seg_nn_st_merge(C.c_void_p(prob.data_ptr()), height, width, C.c_void_p(out.data_ptr()),
                                      _st(prob.device)), "seg_nn_st_merge")
    return out


class SummaryUNet:
    def __init__(self, batch: int, height: int = 64, width: int = 64, theta=None, device="cuda"):
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.B, self.H, self.W = batch, height, width
        nb = C.c_size_t()
        abi.check(abi.lib.seg_nn_st_workspace_bytes(batch, height, width, C.byref(nb)),
                  "seg_nn_st_workspace_bytes")
        self.params = torch.zeros(param_count(), dtype=torch.float32, device=self.device)
        self.ws = torch.empty(nb.value + 256, dtype=torch.uint8, device=self.device)
        h = C.c_void_p()
        abi.check(abi.lib.seg_nn_st_create(batch, height, width, C.c_void_p(self.params.data_ptr()),
                                           C.c_void_p((self.ws.data_ptr() + 255) & ~255), nb.value, C.byref(h)),
                  "seg_nn_st_create")
        self.handle = h
        lifetime.track(self)
        self.load(he_init(0) if theta is None else theta)

    def load(self, theta) -> None:
        self.params.copy_(torch.as_tensor(np.asarray(theta, np.float32)))
        abi.check(abi.lib.seg_nn_sync_weights(self.handle, _st(self.device)), "seg_nn_sync_weights")

    def theta(self) -> np.ndarray:
        return self.params.cpu().numpy()

    def forward(self, st: torch.Tensor) -> torch.Tensor:
        """Raw patches [b, 2, H, W] (S, T) -> probabilities [b, H, W]."""
        b = st.shape[0]
        out = torch.empty((b, self.H, self.W), dtype=torch.float32, device=self.device)
        abi.check(abi.lib.seg_nn_st_forward(self.handle, C.c_void_p(st.data_ptr()), b, C.c_void_p(out.data_ptr()),
                                            _st(self.device)), "seg_nn_st_forward")
        return out

    def logits(self) -> torch.Tensor:
        """Logits [B, H, W] of the last forward or backward call."""
        out = torch.empty((self.B, self.H, self.W), dtype=torch.float32, device=self.device)
        abi.check(abi.lib.seg_nn_logits(self.handle, C.c_void_p(out.data_ptr()), _st(self.device)), "seg_nn_logits")
        return out

    def backward(self, st: torch.Tensor, labels: torch.Tensor, want_grad=False):
        b = st.shape[0]
        loss = C.c_float()
        g = torch.empty_like(self.params) if want_grad else None
        abi.check(abi.lib.seg_nn_st_backward(self.handle, C.c_void_p(st.data_ptr()), C.c_void_p(labels.data_ptr()),
                                             b, C.c_void_p(g.data_ptr()) if g is not None else None,
                                             C.byref(loss), _st(self.device)), "seg_nn_st_backward")
        return loss.value, g

    def step(self, lr=1e-3, rho=0.9, eps=1e-7) -> None:
        abi.check(abi.lib.seg_nn_step(self.handle, lr, rho, eps, _st(self.device)), "seg_nn_step")

    def segment_map(self, S: torch.Tensor, T: torch.Tensor) -> torch.Tensor:
        """Probability map [H, W] of one segment from its device S and T."""
        H, W = S.shape
        pt = patches(S, T)
        prob = torch.empty((pt.shape[0], 64, 64), dtype=torch.float32, device=self.device)
        for a in range(0, pt.shape[0], self.B):
            prob[a:a + self.B] = self.forward(pt[a:a + self.B])
        return merge(prob, H, W)

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
