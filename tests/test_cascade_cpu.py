"""Cascade control without a GPU: stage order, fallback on the stage score,
and the threshold calibration (the q-th percentile of each stage's score over
the calibration frames it relocalises correctly), on a stand-in room whose
stage results are scripted."""
import numpy as np
import pytest

from paper_1810_12163_amd.cascade import Cascade, Stage, calibrate_thresholds


class ScriptedRoom:
    """relocalise returns a pose whose translation x is the request seed's
    scripted error for the stage, and whose score is scripted too; stages are
    told apart by request_seed % 8."""

    def __init__(self, table):
        self.table = table          # (frame seed, stage) -> (status, pose error, score)
        self.calls = []

    def relocalise(self, depth, rgb, K, request_seed=0, **kw):
        frame, si = request_seed // 8, request_seed % 8
        self.calls.append((frame, si))
        status, err, score = self.table[(frame, si)]
        H = np.eye(4, dtype=np.float32)
        H[0, 3] = err
        return dict(status=status, pose=H, mean_energy=score, n_out=1)


def cascade(room, thresholds=(1.0, 2.0)):
    stages = [Stage("a", 8, threshold=thresholds[0]), Stage("b", 8, threshold=thresholds[1]), Stage("c", 8)]
    return Cascade(room, stages, np.zeros((1, 16), np.float32), model="plane", fallback="energy")


def frame():
    return np.zeros((8, 8), np.float32), np.zeros((8, 8, 3), np.uint8), (1.0, 1.0, 4.0, 4.0)


def test_stages_run_in_order_until_a_score_is_at_most_its_threshold():
    table = {(0, 0): ("ok", 0.0, 0.5),                                   # accepted at a
             (1, 0): ("ok", 0.0, 1.5), (1, 1): ("ok", 0.0, 2.0),         # a falls back, b accepted (<=)
             (2, 0): ("no_pose", 0.0, 0.0), (2, 1): ("ok", 0.0, 9.0), (2, 2): ("ok", 0.0, 99.0)}
    room = ScriptedRoom(table)
    cas = cascade(room)
    d, c, K = frame()
    assert cas.relocalise(d, c, K, request_seed=0)["stage"] == "a"
    assert cas.relocalise(d, c, K, request_seed=1)["stage"] == "b"
    out = cas.relocalise(d, c, K, request_seed=2)
    assert out["stage"] == "c" and out["trail"][0][1] == float("inf")   # the last stage's pose is returned
    assert room.calls == [(0, 0), (1, 0), (1, 1), (2, 0), (2, 1), (2, 2)]


def test_calibration_takes_the_percentile_over_correct_frames_only():
    rng = np.random.default_rng(3)
    table, frames = {}, []
    scores_ok = {0: [], 1: []}
    for f in range(40):
        for si in range(3):
            wrong = rng.uniform() < 0.3
            score = float(rng.uniform(0, 10))
            table[(f, si)] = ("ok", 1.0 if wrong else 0.0, score)
            if si < 2 and not wrong:
                scores_ok[si].append(score)
        d, c, K = frame()
        frames.append((d, c, K, f, None))
    table[(40, 0)] = ("no_pose", 0.0, 0.0)                                 # never counted
    table[(40, 1)] = ("ok", 0.0, float("inf"))                             # unverifiable: not counted
    frames.append((*frame(), 40, None))
    room = ScriptedRoom(table)
    cas = cascade(room, thresholds=(-1.0, -1.0))
    th = calibrate_thresholds(cas, frames, lambda pose, truth: abs(float(pose[0, 3])) < 0.5, q=95.0)
    assert th == pytest.approx([np.percentile(scores_ok[0], 95), np.percentile(scores_ok[1], 95)])
    assert [st.threshold for st in cas.stages[:2]] == th
    # the last stage never runs during calibration
    assert all(si < 2 for _, si in room.calls)


def test_calibration_keeps_a_threshold_without_correct_frames():
    table = {(0, 0): ("ok", 1.0, 3.0), (0, 1): ("ok", 0.0, 4.0)}
    room = ScriptedRoom(table)
    cas = cascade(room, thresholds=(7.0, 8.0))
    th = calibrate_thresholds(cas, [(*frame(), 0, None)], lambda pose, truth: abs(float(pose[0, 3])) < 0.5)
    assert th == [7.0, 4.0]
