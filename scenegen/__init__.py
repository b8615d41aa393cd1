"""Seeded synthetic scene generator shared by the oracle side and the GPU side.

It produces inputs only (cameras, features, groups, measurements,
associations); see ``scenegen.scene``.
"""
from .scene import (CONFIGS, DEFAULT_LOSS, OBS_POINT, OBS_LINE, ASSOC_PLANE_POINT,  # noqa: F401
                    ASSOC_PLANE_LINE, ASSOC_VP_LINE, ASSOC_JUNCTION, REL_VP_ORTHO, REL_VP_PARALLEL,
                    REL_PLANE_ORTHO, REL_PLANE_PARALLEL, RELATION_KINDS, LOSS_TRIVIAL,
                    LOSS_HUBER, LOSS_CAUCHY, make_scene, scene_counts, small_config, manhattan_config,
                    config_seed, quaternion_to_matrix, matrix_to_quaternion, ASSOC_PLANE_POINT_3D,
                    plane_3d_scene, SHAPE_SPHERE, SHAPE_CYLINDER, SHAPE_CONE, SHAPE_ELLIPSOID, SHAPE_CUBOID,
                    ASSOC_SHAPE_POINT, ASSOC_SHAPE_LINE)
from .shapes import add_shapes, shape_scene  # noqa: F401
