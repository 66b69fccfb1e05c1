"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package builds scenes (Gaussian parameter arrays, camera poses, upstream
gradients) from a seeded numpy PCG64 generator.  It contains none of the
renderer's or the merge's arithmetic: no projection, no compositing, no
Mahalanobis test.  The recipes stand in for the Replica and TUM RGB-D sequences
that the paper evaluates on (Sec. III-A); no dataset item is reproduced.
"""
from .scenes import (  # noqa: F401
    Camera,
    Scene,
    SH_DC_RANGE,
    cfg1_plain_forward,
    cfg2_keyframe,
    cfg3_room_window,
    cfg4_serving_maps,
    cfg5_large_sh3,
    KeyframeFeatures,
    gradcheck_crop,
    keyframe_features,
    random_pose_in_room,
    room_gaussians,
    tiny_scene,
    upstream_grads,
)
