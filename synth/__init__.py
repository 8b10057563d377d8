"""Seeded synthetic shot generators.

This package draws the inputs of the X-ray tracing sum (detector geometry,
source spectrum, crystal cell and orientation, mosaic domain rotations,
structure-factor table, background scattering curves).  It holds none of the tracing arithmetic: everything
here is input construction, so both the oracle and the HIP path may consume it.
"""
from .shots import (  # noqa: F401
    Shot, SHAPE_SINCG, SHAPE_GAUSS, R_E,
    tiny_shot, full_shot, served_shot, micro_shot, roi_shot, direct_beam_shot,
    random_rotation, axis_angle_matrix, friedel_table, monoclinic_cell,
    orthorhombic_cell, pixel_sample,
    Background, water_background, air_background,
)
