"""Seeded synthetic scenes and pulse sets.

This package only makes inputs: triangle meshes (vertices, triangle indices,
per-triangle reflectance) and pulses (origins, unit directions).  It holds none
of the simulation's arithmetic (no subrays, intersections, radiometry or
waveforms), so both the CPU oracle and the GPU path can consume the same arrays.

All randomness is counter-based (SplitMix64 of (seed, stream, index)), so a
given lattice point or object gets the same value whatever the grid size.
"""
from .rng import splitmix64, uniform01, stream_uniform
from .scenes import (Mesh, value_noise_field, dtm_mesh, add_boxes, merge_meshes,
                     ground_height, procedural_trees, flat_quad)
from .pulses import Pulses, tls_grid, als_lines, concat_pulses
from . import configs

__all__ = [
    "splitmix64", "uniform01", "stream_uniform", "Mesh", "value_noise_field",
    "dtm_mesh", "add_boxes", "merge_meshes", "ground_height", "procedural_trees",
    "flat_quad", "Pulses", "tls_grid", "als_lines", "concat_pulses", "configs",
]
