"""Relocalisation cascade (Sec. 3.2.5): differently-tuned relocalisers backed
by the same forest run one after another until one produces an acceptable
pose.

Stages run on one room (forest, reservoirs and modes are shared) with
per-call RANSAC settings.  A stage's pose is accepted unless its score is
above the stage's threshold, in which case the next stage runs.  The last
stage keeps several hypotheses and ranks them with the model-based score
(the analytic-model stand-in for the paper's depth-raycast ranking,
Sec. 3.2.4); its best is returned.

Score used for the fallback decision: the winner's mean Eq. 5 energy over
the final pixel set (E/|I|).  The paper falls back on the ranking score of
the stage's output; that variant needs the model score of every stage, which
``fallback_on_model`` enables.
"""
from __future__ import annotations

import dataclasses
import time

import numpy as np


@dataclasses.dataclass
class Stage:
    name: str
    n_hypotheses: int
    n_out: int = 1
    decimate: bool = False        # run on the 2x decimated frame
    final_refine: int = -1
    threshold: float = float("inf")   # fall back when the stage score exceeds it


def decimate(depth, rgb, K):
    """2x decimation on the device: pixel (x, y) <- (2x, 2y), intrinsics halved."""
    d = depth[::2, ::2].contiguous()
    c = rgb[::2, ::2].contiguous()
    fx, fy, cx, cy = [float(v) for v in K]
    return d, c, (fx / 2, fy / 2, cx / 2, cy / 2)


class Cascade:
    def __init__(self, room, stages, surfaces: np.ndarray, fallback_on_model: bool = False):
        self.room = room
        self.stages = list(stages)
        self.surfaces = np.ascontiguousarray(surfaces, dtype=np.float32)
        self.fallback_on_model = fallback_on_model

    def relocalise(self, depth, rgb, K, request_seed: int = 0) -> dict:
        t0 = time.perf_counter()
        trail = []
        res = None
        for si, st in enumerate(self.stages):
            d, c, Kk = decimate(depth, rgb, K) if st.decimate else (depth, rgb, K)
            seed = request_seed * 8 + si
            res = self.room.relocalise(d, c, Kk, request_seed=seed, n_hypotheses=st.n_hypotheses,
                                       n_cull=st.n_hypotheses, n_out=st.n_out, final_refine=st.final_refine)
            last = si == len(self.stages) - 1
            if res["status"] != "ok":
                trail.append((st.name, float("inf")))
                if last:
                    break
                continue
            if st.n_out > 1:
                k = res["n_out"]
                slots, poses = self.room.survivors(k)
                scores = self.room.plane_scores(depth, rgb, K, self.surfaces, poses)
                best = int(np.argmin(scores))          # ties -> the better-energy hypothesis
                H = np.eye(4, dtype=np.float32)
                H[:3, :3] = poses[best, :9].reshape(3, 3)
                H[:3, 3] = poses[best, 9:]
                res = dict(res, pose=H, winner=int(slots[best]), model_score=float(scores[best]),
                           ranked=scores)
                score = float(scores[best])
            elif self.fallback_on_model:
                p12 = np.concatenate([res["pose"][:3, :3].reshape(-1), res["pose"][:3, 3]])
                score = float(self.room.plane_scores(depth, rgb, K, self.surfaces, p12[None])[0])
                res = dict(res, model_score=score)
            else:
                score = res["mean_energy"]
            trail.append((st.name, score))
            if last or score <= st.threshold:
                break
        out = dict(res, stage=trail[-1][0], trail=trail, ms=(time.perf_counter() - t0) * 1e3)
        return out
