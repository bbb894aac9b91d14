"""Seeded synthetic loop-closing scenes (inputs only).

This package builds the inputs that both the CPU oracle and the GPU library
consume: map points, keyframe keypoints, poses and Sim3s.  It draws every
random number the scenes need and nothing else; it contains no search,
matching, Hamming, decision, residual or Gauss-Newton arithmetic.
"""
from .scenes import (  # noqa: F401
    CAM_752, CAM_512, Event, Batch, LoopParams,
    gen_c1, gen_c2, gen_c3, gen_c4, gen_c5_event, gen_bidir, gen_inverse_pairs, gen_pose_graph, gen_event,
    concat_events,
    gen_tiny, verification_params, search_transforms, perturbed, ps2_passes, gen_c2_misplaced,
    ROBUST_ITERS, ROBUST_ROUNDS, ROBUST_OUTLIER_PX, ROBUST_LM_LAMBDA,
)
