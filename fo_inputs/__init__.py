"""Seeded synthetic inputs for the first-order (Blatter-Pattyn) Stokes assembly.

This package builds meshes, geometry fields and velocity fields only.  It holds
none of the discretised equations: both the CPU oracle and the HIP library take
its arrays as plain inputs.
"""
from .meshgen import (  # noqa: F401
    ExtrudedMesh,
    config0_slab,
    config1_icesheet,
    ensemble_member,
    learned_mesh,
    box_hex_single,
    right_wedge_single,
    structured_box,
    ellipse_mesh,
    smooth_velocity,
    perturbed,
    boundary_edges,
    floating_slab,
    marine_sheet,
)
