"""MI355X-native neuron segmentation for voltage imaging (Bando et al., 2023,
Sec. III): HIP kernels behind the C ABI of include/seg.h, with a thin Python
binding. PyTorch supplies device memory and streams only."""
from . import abi
from .session import Session, segment_video, to_device_frames

__all__ = ["abi", "Session", "segment_video", "to_device_frames"]
