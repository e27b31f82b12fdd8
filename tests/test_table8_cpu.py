"""The parameter presets and the cascade's relocalisers against the values
the paper prints in Table 8 and its cascade thresholds (fixture
tests/golden/table8_parameters.json): the library's presets, the shared
Python presets and the cascade stages' per-call settings."""
import json
import os

import numpy as np
import pytest

import paper_1810_12163_amd as rl
from paper_1810_12163_amd.cascade import paper_stages
from rlsynth import presets

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table8_parameters.json")))


def _same(a, b):
    return np.float32(a) == np.float32(b)


@pytest.mark.parametrize("name", ["default", "fast", "intermediate", "slow"])
def test_presets_hold_the_table_values(name):
    col = GOLD["columns"][name]
    lib_p = rl.preset(name)
    py_p = presets.preset(name)
    for k, v in col.items():
        if v is None:                       # "N/A" in the table
            continue
        assert _same(lib_p[k], v), (name, k, lib_p[k], v)
        assert _same(py_p[k], v), (name, k, py_p[k], v)


def test_cascade_stages_hold_the_table_ransac_values_and_thresholds():
    stages = paper_stages()
    assert [s.name for s in stages] == ["fast", "intermediate", "slow"]
    th = GOLD["cascade_thresholds_m"]
    assert stages[0].threshold == th["fast_to_intermediate"]
    assert stages[1].threshold == th["intermediate_to_slow"]
    for st in stages:
        col = GOLD["columns"][st.name]
        cs = st.call_settings()
        assert cs["n_hypotheses"] == col["max_pose_candidates"]
        assert cs["n_cull"] == col["max_pose_candidates_after_cull"]
        assert cs["n_out"] == col["max_relocalisations_to_output"]
        assert cs["max_iterations"] == col["max_candidate_generation_iterations"]
        assert cs["eta"] == col["ransac_inliers_per_iteration"]
        assert cs["pose_update"] == col["pose_update"]
        assert _same(cs["min_squared_distance"], col["min_squared_distance_between_sampled_modes"])
        assert _same(cs["max_translation_error"], col["max_translation_error_for_correct_pose"])
        if col["use_prediction_covariance"] is not None:
            assert cs["use_covariance"] == col["use_prediction_covariance"]
