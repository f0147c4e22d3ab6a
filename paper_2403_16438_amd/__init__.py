"""MI355X-native neuron segmentation for voltage imaging (Bando et al., 2023,
Sec. III), with the motion correction before it and the voltage traces after
it (Sec. II): HIP kernels behind the C ABI of include/seg.h and
include/seg_mc.h, with a thin Python binding. PyTorch supplies device memory and streams only."""
from . import abi, lifetime
from .motion import MotionCorrector
from .session import Session, segment_video, to_device_frames
from .lifetime import shutdown

__all__ = ["abi", "MotionCorrector", "Session", "segment_video", "shutdown", "to_device_frames"]
