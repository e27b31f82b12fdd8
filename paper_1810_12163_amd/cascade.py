"""Relocalisation cascade (Sec. 3.2.5): differently-tuned relocalisers backed
by the same forest run one after another until one produces an acceptable
pose.

Stages run on one room (forest, reservoirs and modes are shared) with
per-call RANSAC settings.  A stage that keeps several hypotheses ranks them
with the model-based score and returns the best (Eq. 8).  Its pose is
accepted unless its score is above the stage's threshold, in which case the
next stage runs (the last stage's pose is always returned).

Model-based score (``model``): "depth", the depth-raycast comparison of
Eq. 6-7 on the analytic scene model (the paper's; raycast valid over
[min_depth, max_depth]), or "plane", the mean distance of the back-projected
live depth to the nearest surface.  Fallback score (``fallback``): "model",
the stage output's model score (the paper's), or "energy", the winner's mean
Eq. 5 energy over the final pixel set (E/|I|), which needs no scene model.
"""
from __future__ import annotations

import dataclasses
import time

import numpy as np


@dataclasses.dataclass
class Stage:
    """One relocaliser of the cascade: its hypothesis and RANSAC settings
    (Table 8's RANSAC rows; 0 or negative = the room's own value)."""
    name: str
    n_hypotheses: int
    n_out: int = 1
    decimate: bool = False        # run on the 2x decimated frame
    final_refine: int = -1
    threshold: float = float("inf")   # fall back when the stage score exceeds it
    n_cull: int = 0               # 0: no initial cull (N_cull = n_hypotheses)
    pose_update: int = -1
    max_iterations: int = 0
    eta: int = 0
    use_covariance: int = -1
    min_squared_distance: float = -1.0
    max_translation_error: float = -1.0

    def call_settings(self) -> dict:
        return dict(n_hypotheses=self.n_hypotheses, n_cull=self.n_cull or self.n_hypotheses, n_out=self.n_out,
                    final_refine=self.final_refine, pose_update=self.pose_update,
                    max_iterations=self.max_iterations, eta=self.eta, use_covariance=self.use_covariance,
                    min_squared_distance=self.min_squared_distance,
                    max_translation_error=self.max_translation_error)


def paper_stages(thresholds=(0.05, 0.075)) -> list:
    """The Fast -> Intermediate -> Slow cascade with Table 8's RANSAC settings
    and the tuned depth-difference thresholds (5 cm, then 7.5 cm).  The
    covariance is not used for Intermediate and Slow (Table 8); for Fast the
    table gives none, so the room's setting is kept."""
    return [
        Stage("fast", 2048, n_cull=64, n_out=1, max_iterations=500, eta=256, pose_update=0,
              min_squared_distance=0.0, max_translation_error=0.05, threshold=thresholds[0]),
        Stage("intermediate", 2048, n_cull=64, n_out=1, max_iterations=1000, eta=256, pose_update=1,
              use_covariance=0, min_squared_distance=0.09, max_translation_error=0.1, threshold=thresholds[1]),
        Stage("slow", 2048, n_cull=64, n_out=16, max_iterations=250, eta=256, pose_update=1, use_covariance=0,
              min_squared_distance=0.0225, max_translation_error=0.1),
    ]


def c3_stages(thresholds=(0.05, 0.075)) -> list:
    """The cascade of the 640x480 workload on one forest: (a) the 2x decimated
    frame with 256 hypotheses, (b) the full frame with 1024 hypotheses and the
    inlier refit, (c) 4096 hypotheses kept down to 16, which the cascade ranks
    by its model score.  Stage a falls back above thresholds[0], stage b above
    thresholds[1] (the paper's 5 cm and 7.5 cm by default)."""
    return [Stage("a", 256, decimate=True, threshold=thresholds[0]),
            Stage("b", 1024, final_refine=1, threshold=thresholds[1]),
            Stage("c", 4096, n_out=16)]


def decimate(depth, rgb, K):
    """The 2x decimated frame: pixel (x, y) <- (2x, 2y), intrinsics halved.
    Views of the full frame (no copy): the library reads every second pixel
    of every second row in place."""
    fx, fy, cx, cy = [float(v) for v in K]
    return depth[::2, ::2], rgb[::2, ::2], (fx / 2, fy / 2, cx / 2, cy / 2)


class Cascade:
    def __init__(self, room, stages, surfaces: np.ndarray, model: str = "depth", fallback: str = "model",
                 min_depth: float = 0.5, max_depth: float = 4.0):
        if model not in ("depth", "plane") or fallback not in ("model", "energy"):
            raise ValueError("model must be 'depth' or 'plane', fallback 'model' or 'energy'")
        self.room = room
        self.stages = list(stages)
        self.surfaces = np.ascontiguousarray(surfaces, dtype=np.float32)
        self.model = model
        self.fallback = fallback
        self.min_depth, self.max_depth = float(min_depth), float(max_depth)

    def scores(self, depth, rgb, K, poses12) -> np.ndarray:
        """Model-based score of each pose (lower is better; +inf: unverifiable)."""
        if self.model == "depth":
            return self.room.depth_scores(depth, rgb, K, self.surfaces, poses12, self.min_depth, self.max_depth)[0]
        return self.room.plane_scores(depth, rgb, K, self.surfaces, poses12)

    def _stage(self, si, depth, rgb, K, request_seed):
        """Stage si on the frame: (result, fallback score); the score is +inf
        when the stage returns no pose."""
        st = self.stages[si]
        d, c, Kk = decimate(depth, rgb, K) if st.decimate else (depth, rgb, K)
        res = self.room.relocalise(d, c, Kk, request_seed=request_seed * 8 + si, **st.call_settings())
        if res["status"] != "ok":
            return res, float("inf")
        if st.n_out > 1:
            k = res["n_out"]
            slots, poses = self.room.survivors(k)
            scores = self.scores(depth, rgb, K, poses)
            best = int(np.argmin(scores))          # ties -> the better-energy hypothesis
            H = np.eye(4, dtype=np.float32)
            H[:3, :3] = poses[best, :9].reshape(3, 3)
            H[:3, 3] = poses[best, 9:]
            res = dict(res, pose=H, winner=int(slots[best]), model_score=float(scores[best]), ranked=scores)
            return res, (float(scores[best]) if self.fallback == "model" else res["mean_energy"])
        if self.fallback == "model":
            p12 = np.concatenate([res["pose"][:3, :3].reshape(-1), res["pose"][:3, 3]])
            score = float(self.scores(depth, rgb, K, p12[None])[0])
            return dict(res, model_score=score), score
        return res, res["mean_energy"]

    def relocalise(self, depth, rgb, K, request_seed: int = 0) -> dict:
        t0 = time.perf_counter()
        trail = []
        res = None
        for si, st in enumerate(self.stages):
            res, score = self._stage(si, depth, rgb, K, request_seed)
            last = si == len(self.stages) - 1
            trail.append((st.name, score))
            if res["status"] != "ok":
                if last:
                    break
                continue
            if last or score <= st.threshold:
                break
        out = dict(res, stage=trail[-1][0], trail=trail, ms=(time.perf_counter() - t0) * 1e3)
        return out

    def stage_outputs(self, depth, rgb, K, request_seed: int = 0) -> list:
        """Every stage but the last on the frame, whatever the thresholds (the
        seeds relocalise uses): per stage (result, fallback score)."""
        return [self._stage(si, depth, rgb, K, request_seed) for si in range(len(self.stages) - 1)]


def calibrate_thresholds(cascade, frames, correct, q: float = 95.0) -> list:
    """Fallback thresholds from a calibration set: for each stage but the
    last, the q-th percentile of the stage's score over the frames whose
    stage pose is correct.  frames: (depth, rgb, K, request_seed, truth);
    correct(pose, truth) -> bool.  A stage with no correct frame keeps its
    threshold.  Returns the thresholds and sets them on the stages."""
    per_stage = [[] for _ in cascade.stages[:-1]]
    for depth, rgb, K, seed, truth in frames:
        for si, (res, score) in enumerate(cascade.stage_outputs(depth, rgb, K, request_seed=seed)):
            if res["status"] == "ok" and np.isfinite(score) and correct(res["pose"], truth):
                per_stage[si].append(score)
    out = []
    for st, v in zip(cascade.stages[:-1], per_stage):
        if v:
            st.threshold = float(np.percentile(v, q))
        out.append(st.threshold)
    return out
