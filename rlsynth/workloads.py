"""Concrete seeded workloads (frames + poses + forest + parameters).

Seeds: room r uses scene seed r, forest seed 1000 + r; frame noise seeds are
derived from (room, role, index).  Adaptation poses are independent random
poses in the room; each query pose lies within 20 cm / 20 degrees of a
randomly chosen adaptation pose (c1: 4 adaptation frames within 10 cm /
10 degrees of the query).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import forest as _forest
from . import presets as _presets
from . import scene as _scene


@dataclasses.dataclass
class Frame:
    depth: np.ndarray      # float32 (h, w)
    rgb: np.ndarray        # uint8 (h, w, 3)
    pose: np.ndarray       # float64 (4, 4) camera -> world (ground truth)
    K: tuple               # (fx, fy, cx, cy) float32

    @property
    def w(self):
        return self.depth.shape[1]

    @property
    def h(self):
        return self.depth.shape[0]


@dataclasses.dataclass
class Workload:
    name: str
    params: dict
    room: _scene.Room
    nodes: np.ndarray
    adapt: list
    queries: list


def _frame(room, pose, w, h, seed, **kw):
    d, rgb = _scene.render(room, pose, w, h, seed, **kw)
    return Frame(depth=d, rgb=rgb, pose=pose, K=_scene.intrinsics(w, h))


def frame_seed(room_id: int, role: int, index: int) -> int:
    return 1_000_000 * (room_id + 1) + 100_000 * role + index


def decimate(fr: Frame) -> Frame:
    """2x decimation: pixel (x, y) of the result is pixel (2x, 2y) of the
    input; fx, fy, cx, cy are halved."""
    fx, fy, cx, cy = fr.K
    return Frame(depth=np.ascontiguousarray(fr.depth[::2, ::2]),
                 rgb=np.ascontiguousarray(fr.rgb[::2, ::2]), pose=fr.pose,
                 K=(np.float32(fx / 2), np.float32(fy / 2), np.float32(cx / 2), np.float32(cy / 2)))


def c1(room_id: int = 0, n_queries: int = 1) -> Workload:
    """160x120 frames; 4 adaptation frames within 10 cm / 10 degrees of the
    first query; further queries within 10 cm / 10 degrees of an adaptation
    frame."""
    params = _presets.preset("c1")
    room = _scene.make_room(room_id)
    nodes = _forest.make_forest(1000 + room_id, **_presets.FOREST["c1"])
    rng = np.random.default_rng(frame_seed(room_id, 9, 0))
    w, h = 160, 120
    queries, adapt = [], []
    qpose = _scene.random_pose(room, rng)
    queries.append(_frame(room, qpose, w, h, frame_seed(room_id, 1, 0)))
    for i in range(4):
        ap = _scene.near_pose(room, qpose, rng, 0.10, 10.0)
        adapt.append(_frame(room, ap, w, h, frame_seed(room_id, 0, i)))
    for q in range(1, n_queries):
        base = adapt[int(rng.integers(len(adapt)))].pose
        queries.append(_frame(room, _scene.near_pose(room, base, rng, 0.10, 10.0), w, h,
                              frame_seed(room_id, 1, q)))
    return Workload("c1", params, room, nodes, adapt, queries)


def adapt_poses_for(room, room_id: int, n_adapt: int):
    rng = np.random.default_rng(frame_seed(room_id, 8, 0))
    return [_scene.random_pose(room, rng) for _ in range(n_adapt)]


def room_setup(room_id: int, n_adapt: int, w: int = 640, h: int = 480, forest_cfg: str = "c2"):
    room = _scene.make_room(room_id)
    nodes = _forest.make_forest(1000 + room_id, **_presets.FOREST[forest_cfg])
    poses = adapt_poses_for(room, room_id, n_adapt)
    adapt = [_frame(room, p, w, h, frame_seed(room_id, 0, i)) for i, p in enumerate(poses)]
    return room, nodes, adapt


def queries_for(room, adapt_poses, n, w=640, h=480, room_id=0, novel_fraction=0.0, start=0, processes=0):
    """Query frames near random adaptation poses; a ``novel_fraction`` of them
    are instead drawn >= 50 cm or >= 50 degrees away from every adaptation
    pose (the paper's hardest novelty bin).  ``room`` must be room ``room_id``
    of make_room; with processes > 1 the frames are rendered in worker
    processes (the same frames)."""
    poses = query_poses(room, adapt_poses, n, room_id, novel_fraction, start)
    if processes and processes > 1:
        return render_many([(room_id, p, w, h, frame_seed(room_id, 1, start + q)) for q, p in enumerate(poses)],
                           processes)
    return [_frame(room, p, w, h, frame_seed(room_id, 1, start + q)) for q, p in enumerate(poses)]


def query_poses(room, adapt_poses, n, room_id=0, novel_fraction=0.0, start=0):
    rng = np.random.default_rng(frame_seed(room_id, 7, start))
    out = []
    for q in range(n):
        if rng.uniform() < novel_fraction:
            while True:
                p = _scene.random_pose(room, rng)
                far = all((_scene.pose_error(p, a)[0] >= 0.5 or _scene.pose_error(p, a)[1] >= 50.0)
                          for a in adapt_poses)
                if far:
                    break
        else:
            base = adapt_poses[int(rng.integers(len(adapt_poses)))]
            p = _scene.near_pose(room, base, rng, 0.20, 20.0)
        out.append(p)
    return out


def c2(room_id: int = 0, n_adapt: int = 50, n_queries: int = 8) -> Workload:
    params = _presets.preset("c2")
    room, nodes, adapt = room_setup(room_id, n_adapt)
    queries = queries_for(room, [f.pose for f in adapt], n_queries, room_id=room_id)
    return Workload("c2", params, room, nodes, adapt, queries)


def c2_corrupted(room_id: int = 0, n_adapt: int = 50, n_queries: int = 16, dropout: float = 0.05,
                 depth_rel_sigma: float = 0.0, processes: int = 0, novel_fraction: float = 0.0) -> Workload:
    """The 640x480 workload (same room, forest, poses and noise seeds) with
    every adaptation and query frame rendered under the paper's robustness
    protocols: each pixel's depth zeroed iff r <= dropout, r ~ U[0, 1], and
    depth d replaced by d + n d, n ~ N(0, depth_rel_sigma^2).  A
    novel_fraction of the queries is drawn >= 50 cm or >= 50 degrees away
    from every adaptation pose."""
    room = _scene.make_room(room_id)
    nodes = _forest.make_forest(1000 + room_id, **_presets.FOREST["c2"])
    ap = adapt_poses_for(room, room_id, n_adapt)
    qp = query_poses(room, ap, n_queries, room_id, novel_fraction=novel_fraction)
    kw = dict(dropout=dropout, depth_rel_sigma=depth_rel_sigma)
    jobs = [(room_id, p, 640, 480, frame_seed(room_id, 0, i), kw) for i, p in enumerate(ap)]
    jobs += [(room_id, p, 640, 480, frame_seed(room_id, 1, q), kw) for q, p in enumerate(qp)]
    frames = render_many(jobs, processes)
    return Workload("c2", _presets.preset("c2"), room, nodes, frames[:n_adapt], frames[n_adapt:])


# --- parallel rendering (several rooms / many frames) ----------------------

def _render_job(job):
    room_id, pose, w, h, seed = job[:5]
    kw = job[5] if len(job) > 5 else {}
    room = _scene.make_room(room_id)
    return _frame(room, pose, w, h, seed, **kw)


def render_many(jobs, processes=None):
    """Renders (room_id, pose, w, h, seed[, render keywords]) jobs, in worker processes when
    processes > 1.  Results are identical to rendering them one by one.
    Workers are spawned (fresh interpreters), never forked: a forked copy of a
    process that has initialised the GPU runtime is not safe."""
    if not processes or processes <= 1 or len(jobs) < 4:
        return [_render_job(j) for j in jobs]
    import multiprocessing as mp
    ctx = mp.get_context("spawn")
    with ctx.Pool(processes) as pool:
        return pool.map(_render_job, jobs, chunksize=max(1, len(jobs) // (4 * processes)))


def _sweep_job(job):
    room_id, pose, w, h, seed, levels = job
    room = _scene.make_room(room_id)
    z, rgb, _ = _scene.raycast(room, pose, w, h)
    K = _scene.intrinsics(w, h)
    return [Frame(depth=_scene.corrupt(z, seed, **kw), rgb=rgb, pose=pose, K=K) for kw in levels]


def c2_sweep(levels, room_id: int = 0, n_adapt: int = 50, n_queries: int = 16, processes: int = 0,
             novel_fraction: float = 0.0):
    """c2_corrupted for several sensor settings at once (a list of render
    keywords: dropout, depth_rel_sigma): each pose is raycast once and every
    setting's noise is drawn from the frame's own seed, so the frames equal
    c2_corrupted's.  Returns one Workload per setting."""
    room = _scene.make_room(room_id)
    nodes = _forest.make_forest(1000 + room_id, **_presets.FOREST["c2"])
    ap = adapt_poses_for(room, room_id, n_adapt)
    qp = query_poses(room, ap, n_queries, room_id, novel_fraction=novel_fraction)
    levels = [dict(dict(dropout=0.05, depth_rel_sigma=0.0), **kw) for kw in levels]
    jobs = [(room_id, p, 640, 480, frame_seed(room_id, 0, i), levels) for i, p in enumerate(ap)]
    jobs += [(room_id, p, 640, 480, frame_seed(room_id, 1, q), levels) for q, p in enumerate(qp)]
    if processes and processes > 1 and len(jobs) >= 4:
        import multiprocessing as mp
        with mp.get_context("spawn").Pool(processes) as pool:
            per_pose = pool.map(_sweep_job, jobs, chunksize=max(1, len(jobs) // (4 * processes)))
    else:
        per_pose = [_sweep_job(j) for j in jobs]
    out = []
    for li in range(len(levels)):
        frames = [fr[li] for fr in per_pose]
        out.append(Workload("c2", _presets.preset("c2"), room, nodes, frames[:n_adapt], frames[n_adapt:]))
    return out


RESOLUTIONS = [(160, 120), (320, 240), (640, 480)]
HYPOTHESES = {160: 256, 320: 512, 640: 1024}


def serving_setup(n_rooms=16, n_adapt=20, n_cameras=32, frames_per_camera=4, processes=16, query_rooms=0,
                  queries_per_room=0):
    """Rooms for the serving workload: room r has the 640x480 forest of seed
    1000 + r, adapted from n_adapt frames.  Camera c watches room c % n_rooms at
    resolution RESOLUTIONS[c % 3]; its frames lie within 20 cm / 20 degrees of
    that room's adaptation poses (ground-truth poses kept for adaptation).
    Rooms below query_rooms also get queries_per_room distinct 640x480 query
    frames (rooms[r]["queries"]), drawn the same way."""
    rooms, adapt_jobs, cam_jobs = [], [], []
    for r in range(n_rooms):
        room = _scene.make_room(r)
        rng = np.random.default_rng(frame_seed(r, 8, 0))
        poses = [_scene.random_pose(room, rng) for _ in range(n_adapt)]
        nodes = _forest.make_forest(1000 + r, **_presets.FOREST["c2"])
        rooms.append(dict(room_id=r, nodes=nodes, poses=poses))
        adapt_jobs += [(r, p, 640, 480, frame_seed(r, 0, i)) for i, p in enumerate(poses)]
    for c in range(n_cameras):
        r = c % n_rooms
        w, h = RESOLUTIONS[c % 3]
        room = _scene.make_room(r)
        rng = np.random.default_rng(frame_seed(r, 6, c))
        for k in range(frames_per_camera):
            base = rooms[r]["poses"][int(rng.integers(n_adapt))]
            p = _scene.near_pose(room, base, rng, 0.20, 20.0)
            cam_jobs.append((r, p, w, h, frame_seed(r, 5, c * 100 + k)))
    q_jobs = []
    for r in range(min(n_rooms, query_rooms)):
        room = _scene.make_room(r)
        rng = np.random.default_rng(frame_seed(r, 4, 0))
        for k in range(queries_per_room):
            base = rooms[r]["poses"][int(rng.integers(n_adapt))]
            q_jobs.append((r, _scene.near_pose(room, base, rng, 0.20, 20.0), 640, 480, frame_seed(r, 4, k)))
    frames = render_many(adapt_jobs + cam_jobs + q_jobs, processes)
    na = len(adapt_jobs)
    for r in range(n_rooms):
        rooms[r]["adapt"] = frames[r * n_adapt:(r + 1) * n_adapt]
        rooms[r]["queries"] = []
    for j, fr in zip(q_jobs, frames[na + len(cam_jobs):]):
        rooms[j[0]]["queries"].append(fr)
    cams = []
    for c in range(n_cameras):
        cams.append(dict(room=c % n_rooms, frames=frames[na + c * frames_per_camera: na + (c + 1) * frames_per_camera]))
    return rooms, cams
