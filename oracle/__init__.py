"""Plain FP64 CPU oracle of the neuron-segmentation stage.

TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import this package. The GPU library neither imports
nor links anything here, and this package shares no code with it.

Functions without an independent pin say so in their docstring
("parity unpinned"); every other function is checked by tests against closed
forms, hand-worked examples, brute force or a library special case.
"""
from .segment import (Params, Result, gaussian_weights, reflect_index,
                      smoothing_matrix, smooth_frames, summarize_segment,
                      segment_moments, correlation_image, event_maps,
                      label8, region_stats, hull_area2, shape_filter,
                      aggregate, spa, hals, nmf_component, footprints, segment)
from .metrics import iou_matrix, match_f1

__all__ = ["Params", "Result", "gaussian_weights", "reflect_index",
           "smoothing_matrix", "smooth_frames", "summarize_segment",
           "segment_moments", "correlation_image", "event_maps", "label8",
           "region_stats", "hull_area2", "shape_filter", "aggregate", "spa",
           "hals", "nmf_component", "footprints", "segment", "iou_matrix",
           "match_f1"]
