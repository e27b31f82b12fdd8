"""Parameter sets.

Names follow the paper's parameter table (Table 8, "Parameter Tuning"
appendix) in snake_case, plus the few settings the paper leaves open.  The
values of the four paper presets are that table's; the c1..c5 sets are the
synthetic workloads this project measures (640x480 frames unless stated).

Readings where the paper gives no value:
* max_colour_linf = 30 (0..255 scale) for the colour check of hypothesis
  generation (the paper gives no threshold);
* the rigidity check uses max_translation_error_for_correct_pose as its
  tolerance on pairwise-distance differences;
* cov_regulariser = 1e-6 m^2 is added to each mode covariance before
  inversion;
* inlier_threshold = 0.05 m for the optional final refit over inliers;
* lm_iterations = 10 Levenberg-Marquardt iterations per survivor and round
  when pose_update is on;
* max_pose_candidates_after_cull >= max_pose_candidates disables the initial
  cull, giving pure halving rounds.
"""
from __future__ import annotations

import copy

FIELDS_INT = [
    "n_trees", "depth", "ref_width",
    "max_cluster_count", "min_cluster_size", "reservoir_capacity",
    "max_candidate_generation_iterations", "max_pose_candidates",
    "max_pose_candidates_after_cull", "ransac_inliers_per_iteration",
    "max_relocalisations_to_output", "use_prediction_covariance", "pose_update",
    "final_refine", "lm_iterations",
]
FIELDS_FLOAT = [
    "clusterer_sigma", "clusterer_tau",
    "min_squared_distance_between_sampled_modes",
    "max_translation_error_for_correct_pose", "max_colour_linf",
    "inlier_threshold", "cov_regulariser",
]
FIELDS_U64 = ["seed"]

_COMMON = dict(
    n_trees=5, depth=15, ref_width=640,
    max_colour_linf=30.0, inlier_threshold=0.05, cov_regulariser=1e-6,
    final_refine=0, seed=0, lm_iterations=10,
)

PAPER = {
    "default": dict(_COMMON, clusterer_sigma=0.1, clusterer_tau=0.05, max_cluster_count=50,
                    min_cluster_size=20, reservoir_capacity=1024,
                    max_candidate_generation_iterations=6000, max_pose_candidates=1024,
                    max_pose_candidates_after_cull=64, max_translation_error_for_correct_pose=0.05,
                    min_squared_distance_between_sampled_modes=0.09, pose_update=1,
                    ransac_inliers_per_iteration=512, use_prediction_covariance=1,
                    max_relocalisations_to_output=16),
    "fast": dict(_COMMON, clusterer_sigma=0.1, clusterer_tau=0.2, max_cluster_count=50,
                 min_cluster_size=5, reservoir_capacity=2048,
                 max_candidate_generation_iterations=500, max_pose_candidates=2048,
                 max_pose_candidates_after_cull=64, max_translation_error_for_correct_pose=0.05,
                 min_squared_distance_between_sampled_modes=0.0, pose_update=0,
                 ransac_inliers_per_iteration=256, use_prediction_covariance=0,
                 max_relocalisations_to_output=1),
    "intermediate": dict(_COMMON, clusterer_sigma=0.1, clusterer_tau=0.2, max_cluster_count=50,
                         min_cluster_size=5, reservoir_capacity=2048,
                         max_candidate_generation_iterations=1000, max_pose_candidates=2048,
                         max_pose_candidates_after_cull=64, max_translation_error_for_correct_pose=0.1,
                         min_squared_distance_between_sampled_modes=0.09, pose_update=1,
                         ransac_inliers_per_iteration=256, use_prediction_covariance=0,
                         max_relocalisations_to_output=1),
    "slow": dict(_COMMON, clusterer_sigma=0.1, clusterer_tau=0.2, max_cluster_count=50,
                 min_cluster_size=5, reservoir_capacity=2048,
                 max_candidate_generation_iterations=250, max_pose_candidates=2048,
                 max_pose_candidates_after_cull=64, max_translation_error_for_correct_pose=0.1,
                 min_squared_distance_between_sampled_modes=0.0225, pose_update=1,
                 ransac_inliers_per_iteration=256, use_prediction_covariance=0,
                 max_relocalisations_to_output=16),
}

_C2 = dict(_COMMON, clusterer_sigma=0.1, clusterer_tau=0.05, max_cluster_count=10,
           min_cluster_size=20, reservoir_capacity=1024,
           max_candidate_generation_iterations=6000, max_pose_candidates=1024,
           max_pose_candidates_after_cull=1024, max_translation_error_for_correct_pose=0.05,
           min_squared_distance_between_sampled_modes=0.09, pose_update=0,
           ransac_inliers_per_iteration=500, use_prediction_covariance=1,
           max_relocalisations_to_output=1, final_refine=1)

CONFIGS = {
    # 160x120, one depth-8 tree (forest reference width 160), small reservoirs
    "c1": dict(_C2, n_trees=1, depth=8, ref_width=160, clusterer_tau=0.2, min_cluster_size=5,
               max_cluster_count=5, reservoir_capacity=64, max_pose_candidates=64,
               max_pose_candidates_after_cull=64, ransac_inliers_per_iteration=100,
               final_refine=0),
    "c2": dict(_C2),
    # cascade stages share the c2 forest
    "c3a": dict(_C2, max_pose_candidates=256, max_pose_candidates_after_cull=256),
    "c3b": dict(_C2),
    "c3c": dict(_C2, max_pose_candidates=4096, max_pose_candidates_after_cull=4096,
                max_relocalisations_to_output=16, final_refine=0),
    "c4": dict(_C2),
    "c5": dict(_C2),
}
# the cascade workload's room: sized for its widest stage
CONFIGS["c3"] = dict(CONFIGS["c3c"])


def preset(name: str) -> dict:
    name = name.lower()
    if name in PAPER:
        return copy.deepcopy(PAPER[name])
    if name in CONFIGS:
        return copy.deepcopy(CONFIGS[name])
    raise KeyError(name)


# forest-generator settings per workload (random splits, see forest.py)
FOREST = {
    "c1": dict(n_trees=1, depth=8, p_depth=0.4, offset_range=130.0, tau_depth=0.2, tau_colour=64.0),
    "c2": dict(n_trees=5, depth=15, p_depth=0.4, offset_range=130.0, tau_depth=0.2, tau_colour=64.0),
}
