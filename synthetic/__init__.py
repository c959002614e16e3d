"""Seeded synthetic scenes for the segment-embedding lift.

This package only draws inputs: Gaussians, cameras, per-view segment-id maps
and per-segment feature tables.  It contains none of the lift's arithmetic, so
both the CPU oracle and the GPU library can consume the very same bytes.
"""
from .scenes import (Scene, make_scene, CONFIGS, camera_dtype, f32_to_bf16_bits,
                     bf16_bits_to_f32, vocabulary_words)

__all__ = ["Scene", "make_scene", "CONFIGS", "camera_dtype", "f32_to_bf16_bits",
           "bf16_bits_to_f32", "vocabulary_words"]
