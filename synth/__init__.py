"""Seeded synthetic surveillance-video generator.

This module is the single source of inputs for both sides of every parity
check (the CPU oracle and the HIP library).  It holds none of the method's
arithmetic: it only draws frames and ground-truth masks.
"""
from .video import (  # noqa: F401
    StreamSpec,
    PRESETS,
    preset,
    make_stream,
    iter_frames,
    constant_stream,
    random_stream,
    alternating_stream,
    step_stream,
    latent_stream,
)
