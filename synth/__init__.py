"""Seeded synthetic voltage-imaging videos.

This package only draws inputs: a background field, neurons with Gaussian
footprints, Poisson spike trains, Poisson shot noise and Gaussian read noise.
It holds none of the segmentation method's arithmetic, so both the CPU oracle
and the GPU path can take their inputs from it without sharing any of the
method's code.
"""
from .simulate import (SimConfig, Truth, draw, preset, simulate, simulate_frames,
                       session_mix)
from .motion import draw_motion, move_frames, plant_motion

__all__ = ["SimConfig", "Truth", "draw", "preset", "simulate", "simulate_frames",
           "session_mix", "draw_motion", "move_frames", "plant_motion"]
