"""Seeded synthetic inputs shared by the FP64 oracle and the HIP path.

This package holds scene geometry, materials and job parameters only. It
contains none of the wave path tracer's arithmetic: no ray sampling, no
intersection, no BSDF, no phase. Both the oracle and the GPU library read
the arrays it produces.
"""
from .generators import (  # noqa: F401
    LAMBERT, GGX, MIRROR, DIELECTRIC, EMITTER, PRINCIPLED,
    make_scene, scene_tiny, scene_mid, scene_large, scene_arrays_ok,
    scene_patch, scene_mirror_patch, scene_slab, scene_furnace_sphere,
    scene_lambert_plane, scene_single_tri, scene_translate, empty_scene, scene_lit_plane,
    scene_slab_emitter, scene_ggx_plane, scene_depth_rescaled, scene_point_emitters,
    scene_emitter_box, scene_sheet_stack,
)
from .jobs import job_for_config, JOB_DEFAULTS  # noqa: F401
