"""ctypes binding of include/seg.h (argument marshalling only).

Every computation runs in libseg.so; importing this module without the built
library raises immediately (build it with `python -m paper_2403_16438_amd.build`).
"""
from __future__ import annotations

import ctypes as C
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
# SEG_LIBRARY selects another build of the same library, e.g. the one whose
# host code is instrumented with address and undefined-behaviour sanitizers
# (build.build_sanitized)
LIB_PATH = os.environ.get("SEG_LIBRARY") or os.path.join(HERE, "libseg.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "seg.h")

SEG_OK = 0
SEG_E_INVAL = -1
SEG_E_SHAPE = -2
SEG_E_STATE = -3
SEG_E_CAPACITY = -4
SEG_E_DEVICE = -5
SEG_E_NOMODEL = -6

SEG_DET_PLAIN = 0
SEG_DET_SURROGATE = 1
SEG_DET_UNET = 2
SEG_NN_INPUT_FRAMES, SEG_NN_INPUT_SUMMARIES = 0, 1
SEG_NMF_AUTO, SEG_NMF_SINGLE, SEG_NMF_SPLIT = 0, 1, 2

SEG_IMG_MEAN, SEG_IMG_CORR, SEG_IMG_NOISE = 0, 1, 2
SEG_IMG_EVENT_COUNT, SEG_IMG_MASK_COUNT, SEG_IMG_LABELS = 3, 4, 5
SEG_MAP_S, SEG_MAP_T, SEG_MAP_P, SEG_MAP_B, SEG_MAP_D = 0, 1, 2, 3, 4


class seg_config(C.Structure):
    _fields_ = [("height", C.c_uint32), ("width", C.c_uint32),
                ("seg_len", C.c_uint32), ("max_frames", C.c_uint32),
                ("gauss_sigma", C.c_float), ("gauss_radius", C.c_uint32),
                ("event_z", C.c_float), ("min_event_segs", C.c_uint32),
                ("area_min", C.c_uint32), ("area_max", C.c_uint32),
                ("solidity_min", C.c_float), ("ecc_max", C.c_float),
                ("nmf_max_rank", C.c_uint32), ("nmf_sweeps", C.c_uint32),
                ("spa_delta", C.c_float), ("footprint_level", C.c_float),
                ("sigma_floor", C.c_float), ("detector", C.c_uint32),
                ("nmf_path", C.c_uint32)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class seg_mc_config(C.Structure):
    _fields_ = [("height", C.c_uint32), ("width", C.c_uint32), ("radius", C.c_uint32)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class seg_profile(C.Structure):
    _fields_ = [("maps_ms", C.c_float), ("nmf_ms", C.c_float), ("nmf_flops", C.c_double),
                ("nmf_path", C.c_uint32), ("nmf_workgroups", C.c_uint32),
                ("components", C.c_uint32), ("max_rank", C.c_uint32)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class SegError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {strerror(code)} ({code})")


def _load():
    # PyTorch ships its own HIP runtime (same soname as /opt/rocm's). Loading
    # torch first makes libseg.so bind to that runtime, so the process holds a
    # single HIP runtime and torch's device memory and streams are valid here.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2403_16438_amd.build`")
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    u32 = C.c_uint32
    sig = {
        "seg_default_config": (C.c_int, [u32, u32, u32, C.POINTER(seg_config)]),
        "seg_workspace_bytes": (C.c_int, [C.POINTER(seg_config), C.POINTER(C.c_size_t)]),
        "seg_create": (C.c_int, [C.POINTER(seg_config), P, C.c_size_t, C.POINTER(P)]),
        "seg_push_frames": (C.c_int, [P, P, u32, P]),
        "seg_finalize": (C.c_int, [P, P]),
        "seg_num_segments": (C.c_int, [P, C.POINTER(u32)]),
        "seg_get_footprints": (C.c_int, [P, u32, C.POINTER(u32), P, P, P, P]),
        "seg_get_image": (C.c_int, [P, C.c_int, P]),
        "seg_extract_traces": (C.c_int, [P, P, C.c_uint64, P, C.c_uint64, P]),
        "seg_get_profile": (C.c_int, [P, C.POINTER(seg_profile)]),
        "seg_state_bytes": (C.c_int, [P, C.POINTER(C.c_size_t)]),
        "seg_export_state": (C.c_int, [P, P, C.c_size_t, P]),
        "seg_import_state": (C.c_int, [P, P, C.c_size_t, P]),
        "seg_get_segment_maps": (C.c_int, [P, C.c_int, u32, u32, P, P]),
        "seg_load_summaries": (C.c_int, [P, u32, P, P, P, P, P]),
        "seg_destroy": (C.c_int, [P]),
        "seg_batch_bytes": (C.c_int, [u32, C.POINTER(C.c_size_t)]),
        "seg_batch_create": (C.c_int, [u32, P, C.c_size_t, C.POINTER(P)]),
        "seg_push_batch": (C.c_int, [P, C.POINTER(P), C.POINTER(P), C.POINTER(u32), u32, P]),
        "seg_batch_destroy": (C.c_int, [P]),
        "seg_nn_param_count": (C.c_int, [C.POINTER(C.c_size_t)]),
        "seg_nn_param_layout": (C.c_int, [u32, C.POINTER(u32), C.POINTER(u32), C.POINTER(C.c_size_t),
                                          C.POINTER(C.c_size_t)]),
        "seg_nn_workspace_bytes": (C.c_int, [u32, u32, u32, C.POINTER(C.c_size_t)]),
        "seg_nn_create": (C.c_int, [u32, u32, u32, P, P, C.c_size_t, C.POINTER(P)]),
        "seg_nn_sync_weights": (C.c_int, [P, P]),
        "seg_nn_forward": (C.c_int, [P, P, u32, P, P]),
        "seg_nn_backward": (C.c_int, [P, P, P, u32, P, C.POINTER(C.c_float), P]),
        "seg_nn_step": (C.c_int, [P, C.c_float, C.c_float, C.c_float, P]),
        "seg_nn_logits": (C.c_int, [P, P, P]),
        "seg_nn_gemm_test": (C.c_int, [P, C.c_int, P, C.c_int, P, C.c_int, C.c_int, C.c_int, C.c_int, P, P]),
        "seg_nn_destroy": (C.c_int, [P]),
        "seg_nn_shape": (C.c_int, [P, C.POINTER(u32), C.POINTER(u32), C.POINTER(u32)]),
        "seg_nn_st_param_count": (C.c_int, [C.POINTER(C.c_size_t)]),
        "seg_nn_st_param_layout": (C.c_int, [u32, C.POINTER(u32), C.POINTER(u32), C.POINTER(C.c_size_t),
                                             C.POINTER(C.c_size_t)]),
        "seg_nn_st_workspace_bytes": (C.c_int, [u32, u32, u32, C.POINTER(C.c_size_t)]),
        "seg_nn_st_create": (C.c_int, [u32, u32, u32, P, P, C.c_size_t, C.POINTER(P)]),
        "seg_nn_st_forward": (C.c_int, [P, P, u32, P, P]),
        "seg_nn_st_backward": (C.c_int, [P, P, P, u32, P, C.POINTER(C.c_float), P]),
        "seg_nn_input": (C.c_int, [P, C.POINTER(u32)]),
        "seg_nn_st_patch_count": (C.c_int, [u32, u32, C.POINTER(u32)]),
        "seg_nn_st_patches": (C.c_int, [P, P, u32, u32, P, P]),
        "seg_nn_st_merge": (C.c_int, [P, u32, u32, P, P]),
        "seg_set_model": (C.c_int, [P, P]),
        "seg_mc_default_config": (C.c_int, [u32, u32, C.POINTER(seg_mc_config)]),
        "seg_mc_workspace_bytes": (C.c_int, [C.POINTER(seg_mc_config), C.POINTER(C.c_size_t)]),
        "seg_mc_create": (C.c_int, [C.POINTER(seg_mc_config), P, C.c_size_t, C.POINTER(P)]),
        "seg_mc_layout": (C.c_int, [P, C.POINTER(u32), C.POINTER(u32)]),
        "seg_mc_set_template": (C.c_int, [P, P, u32, P]),
        "seg_mc_get_template": (C.c_int, [P, P]),
        "seg_mc_estimate": (C.c_int, [P, P, C.c_uint64, P, P, P]),
        "seg_mc_estimate_static": (C.c_int, [P, P, C.c_uint64, P, P, P]),
        "seg_mc_apply": (C.c_int, [P, P, C.c_uint64, P, P, P]),
        "seg_mc_destroy": (C.c_int, [P]),
        "seg_strerror": (C.c_char_p, [C.c_int]),
        "seg_last_error": (C.c_int, [P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


def header_functions() -> list:
    """Names of the functions declared in include/seg.h, seg_nn.h and seg_mc.h."""
    inc = os.path.dirname(HEADER)
    text = "".join(open(os.path.join(inc, f)).read() for f in ("seg.h", "seg_nn.h", "seg_mc.h"))
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(seg_\w+)\s*\(", text, re.M)))


def strerror(code: int) -> str:
    return lib.seg_strerror(code).decode()


def check(code: int, where: str) -> None:
    if code != SEG_OK:
        raise SegError(code, where)


def seg_default_config(height: int, width: int, max_frames: int) -> seg_config:
    c = seg_config()
    check(lib.seg_default_config(height, width, max_frames, C.byref(c)), "seg_default_config")
    return c


def seg_workspace_bytes(cfg: seg_config) -> int:
    n = C.c_size_t()
    check(lib.seg_workspace_bytes(C.byref(cfg), C.byref(n)), "seg_workspace_bytes")
    return n.value


def seg_create(cfg: seg_config, dev_workspace: int, nbytes: int):
    h = C.c_void_p()
    check(lib.seg_create(C.byref(cfg), C.c_void_p(dev_workspace), nbytes, C.byref(h)), "seg_create")
    return h


def seg_push_frames(h, dev_frames: int, n: int, stream: int) -> None:
    check(lib.seg_push_frames(h, C.c_void_p(dev_frames), n, C.c_void_p(stream)), "seg_push_frames")


def seg_finalize(h, stream: int) -> None:
    check(lib.seg_finalize(h, C.c_void_p(stream)), "seg_finalize")


def seg_num_segments(h) -> int:
    k = C.c_uint32()
    check(lib.seg_num_segments(h, C.byref(k)), "seg_num_segments")
    return k.value


def seg_get_footprints(h, capacity: int, weights, masks, activity, component) -> int:
    n = C.c_uint32()
    ptr = lambda a: None if a is None else a.ctypes.data_as(C.c_void_p)
    check(lib.seg_get_footprints(h, capacity, C.byref(n), ptr(weights), ptr(masks),
                                 ptr(activity), ptr(component)), "seg_get_footprints")
    return n.value


def seg_get_image(h, kind: int, out) -> None:
    check(lib.seg_get_image(h, kind, out.ctypes.data_as(C.c_void_p)), "seg_get_image")


def seg_extract_traces(h, dev_frames: int, n_frames: int, dev_out: int, ld: int, stream: int) -> None:
    check(lib.seg_extract_traces(h, C.c_void_p(dev_frames), n_frames, C.c_void_p(dev_out), ld,
                                 C.c_void_p(stream)), "seg_extract_traces")


def seg_get_segment_maps(h, kind: int, first: int, count: int, dev_out: int, stream: int) -> None:
    check(lib.seg_get_segment_maps(h, kind, first, count, C.c_void_p(dev_out), C.c_void_p(stream)),
          "seg_get_segment_maps")


def seg_load_summaries(h, k: int, T, S, D, U=None, P=None) -> None:
    ptr = lambda a: None if a is None else a.ctypes.data_as(C.c_void_p)
    check(lib.seg_load_summaries(h, k, ptr(T), ptr(S), ptr(D), ptr(U), ptr(P)), "seg_load_summaries")


def seg_destroy(h) -> None:
    lib.seg_destroy(h)


def seg_last_error(h) -> int:
    return lib.seg_last_error(h)


def seg_batch_bytes(max_slots: int) -> int:
    n = C.c_size_t()
    check(lib.seg_batch_bytes(max_slots, C.byref(n)), "seg_batch_bytes")
    return n.value


def seg_batch_create(max_slots: int, dev_table: int, nbytes: int):
    h = C.c_void_p()
    check(lib.seg_batch_create(max_slots, C.c_void_p(dev_table), nbytes, C.byref(h)), "seg_batch_create")
    return h


def seg_push_batch(b, sessions, dev_frames, n_frames, stream: int) -> None:
    k = len(sessions)
    S = (C.c_void_p * k)(*[s.value for s in sessions])
    F = (C.c_void_p * k)(*dev_frames)
    N = (C.c_uint32 * k)(*n_frames)
    check(lib.seg_push_batch(b, S, F, N, k, C.c_void_p(stream)), "seg_push_batch")


def seg_batch_destroy(b) -> None:
    lib.seg_batch_destroy(b)


def seg_get_profile(h) -> dict:
    out = seg_profile()
    check(lib.seg_get_profile(h, C.byref(out)), "seg_get_profile")
    return out.as_dict()


def seg_export_state(h, stream: int):
    import numpy as np
    n = C.c_size_t()
    check(lib.seg_state_bytes(h, C.byref(n)), "seg_state_bytes")
    buf = np.empty(n.value, np.uint8)
    check(lib.seg_export_state(h, buf.ctypes.data_as(C.c_void_p), n.value, C.c_void_p(stream)),
          "seg_export_state")
    return buf


def seg_import_state(h, buf, stream: int) -> None:
    check(lib.seg_import_state(h, buf.ctypes.data_as(C.c_void_p), buf.nbytes, C.c_void_p(stream)),
          "seg_import_state")


# ---- motion correction (include/seg_mc.h) ----

def seg_mc_default_config(height: int, width: int) -> seg_mc_config:
    c = seg_mc_config()
    check(lib.seg_mc_default_config(height, width, C.byref(c)), "seg_mc_default_config")
    return c


def seg_mc_workspace_bytes(cfg: seg_mc_config) -> int:
    n = C.c_size_t()
    check(lib.seg_mc_workspace_bytes(C.byref(cfg), C.byref(n)), "seg_mc_workspace_bytes")
    return n.value


def seg_mc_create(cfg: seg_mc_config, dev_workspace: int, nbytes: int):
    h = C.c_void_p()
    check(lib.seg_mc_create(C.byref(cfg), C.c_void_p(dev_workspace), nbytes, C.byref(h)), "seg_mc_create")
    return h


def seg_mc_layout(h) -> tuple:
    p, v = C.c_uint32(), C.c_uint32()
    check(lib.seg_mc_layout(h, C.byref(p), C.byref(v)), "seg_mc_layout")
    return p.value, v.value


def seg_mc_set_template(h, dev_frames: int, n: int, stream: int) -> None:
    check(lib.seg_mc_set_template(h, C.c_void_p(dev_frames), n, C.c_void_p(stream)), "seg_mc_set_template")


def seg_mc_get_template(h, out) -> None:
    check(lib.seg_mc_get_template(h, out.ctypes.data_as(C.c_void_p)), "seg_mc_get_template")


def seg_mc_estimate(h, dev_frames: int, n: int, dev_motion: int, dev_scores: int | None, stream: int) -> None:
    check(lib.seg_mc_estimate(h, C.c_void_p(dev_frames), n, C.c_void_p(dev_motion),
                              C.c_void_p(dev_scores) if dev_scores else None, C.c_void_p(stream)),
          "seg_mc_estimate")


SEG_MC_STATIC_MAX_FRAMES = 256


def seg_mc_estimate_static(h, dev_frames: int, n: int, dev_motion: int, dev_scores: int | None,
                           stream: int) -> None:
    check(lib.seg_mc_estimate_static(h, C.c_void_p(dev_frames), n, C.c_void_p(dev_motion),
                                     C.c_void_p(dev_scores) if dev_scores else None, C.c_void_p(stream)),
          "seg_mc_estimate_static")


def seg_mc_apply(h, dev_frames: int, n: int, dev_motion: int, dev_out: int, stream: int) -> None:
    check(lib.seg_mc_apply(h, C.c_void_p(dev_frames), n, C.c_void_p(dev_motion), C.c_void_p(dev_out),
                           C.c_void_p(stream)), "seg_mc_apply")
