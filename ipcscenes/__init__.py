"""Seeded synthetic scene generators shared by the HIP library tests and the oracle.

This package only builds inputs: meshes, material parameters, body descriptions,
spring anchors, drive trajectories and coarse render meshes with their frames.  It contains none of the method's
arithmetic (no energies, no precompute, no contact, no solver).  Every scene is
a plain ``dict`` of numpy arrays; see ``scenes.SCENE_KEYS`` for the layout.
"""
from .scenes import (  # noqa: F401
    SCENE_KEYS,
    block_drop,
    gripper_squeeze,
    arm_squeeze,
    contact_rich,
    batched_squeeze,
    adjoint_squeeze,
    tiny_scene,
    hex_tets,
    validate_scene,
    tet_surface,
    dualmesh_frames,
)
