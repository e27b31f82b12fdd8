"""MI355X relocaliser: Python binding of librl.so (include/rl.h).

Argument marshalling only: every step of the relocaliser runs in the HIP
kernels of librl.so.  PyTorch provides the device memory (the room's
persistent and scratch buffers are torch uint8 tensors) and the stream.  If
the library has not been built, every entry point raises; there is no other
implementation to fall back to.

    room = Room(params, nodes, max_width=640, max_height=480)
    room.adapt(depth, rgb, K, pose)           # torch cuda tensors, 4x4 pose
    res = room.relocalise(depth, rgb, K, request_seed=0)
    res["pose"], res["energy"], res["status"]
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librl.so")

RL_OK, RL_NO_POSE, RL_EINVAL, RL_ENOMEM, RL_EDEVICE, RL_EBUSY = 0, 1, -1, -2, -3, -4

(BUF_NODES, BUF_RESERVOIR, BUF_SEEN, BUF_MODES, BUF_NMODES, BUF_LEAVES, BUF_NM, BUF_ELIGIBLE,
 BUF_HYPS, BUF_ILIST, BUF_TRACE_SLOTS, BUF_TRACE_ENERGY, BUF_SURVIVORS, BUF_ENERGY,
 BUF_DIRTY, BUF_CBOX, BUF_EREC, BUF_POSE64) = range(18)

HYP_DTYPE = np.dtype([("R", "<f4", (9,)), ("t", "<f4", (3,)), ("pix", "<i4", (3,)),
                      ("mode", "<i4", (3,)), ("iter", "<i4"), ("valid", "<i4")])
NODE_DTYPE = np.dtype([("dx", "<f4"), ("dy", "<f4"), ("tau", "<f4"), ("kind", "<u4")])


class RlError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"librl status {status}: {message}")
        self.status = status


class Intrinsics(ctypes.Structure):
    _fields_ = [("fx", ctypes.c_float), ("fy", ctypes.c_float), ("cx", ctypes.c_float),
                ("cy", ctypes.c_float)]


class Frame(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("depth", ctypes.c_void_p), ("rgb", ctypes.c_void_p), ("K", Intrinsics),
                ("rgb_channels", ctypes.c_int32), ("rgb_pitch_bytes", ctypes.c_int32),
                ("depth_pitch_bytes", ctypes.c_int32), ("step", ctypes.c_int32)]


class Params(ctypes.Structure):
    _fields_ = [
        ("n_trees", ctypes.c_int32), ("depth", ctypes.c_int32), ("ref_width", ctypes.c_int32),
        ("clusterer_sigma", ctypes.c_float), ("clusterer_tau", ctypes.c_float),
        ("max_cluster_count", ctypes.c_int32), ("min_cluster_size", ctypes.c_int32),
        ("reservoir_capacity", ctypes.c_int32),
        ("max_candidate_generation_iterations", ctypes.c_int32),
        ("max_pose_candidates", ctypes.c_int32), ("max_pose_candidates_after_cull", ctypes.c_int32),
        ("ransac_inliers_per_iteration", ctypes.c_int32),
        ("max_relocalisations_to_output", ctypes.c_int32),
        ("use_prediction_covariance", ctypes.c_int32), ("pose_update", ctypes.c_int32),
        ("final_refine", ctypes.c_int32), ("lm_iterations", ctypes.c_int32),
        ("min_squared_distance_between_sampled_modes", ctypes.c_float),
        ("max_translation_error_for_correct_pose", ctypes.c_float),
        ("max_colour_linf", ctypes.c_float), ("inlier_threshold", ctypes.c_float),
        ("cov_regulariser", ctypes.c_float), ("seed", ctypes.c_uint64),
    ]


class Result(ctypes.Structure):
    _fields_ = [("cam_to_world", ctypes.c_float * 16), ("energy", ctypes.c_float),
                ("mean_energy", ctypes.c_float), ("status", ctypes.c_int32),
                ("n_valid", ctypes.c_int32), ("n_inliers", ctypes.c_int32),
                ("winner", ctypes.c_int32), ("refitted", ctypes.c_int32),
                ("n_eligible", ctypes.c_int32), ("rounds", ctypes.c_int32),
                ("n_out", ctypes.c_int32), ("mode_version", ctypes.c_uint32), ("pad", ctypes.c_int32)]


# rl_result as a numpy record (decoding many results at once)
RESULT_DTYPE = np.dtype([("cam_to_world", "<f4", (16,)), ("energy", "<f4"), ("mean_energy", "<f4"),
                         ("status", "<i4"), ("n_valid", "<i4"), ("n_inliers", "<i4"), ("winner", "<i4"),
                         ("refitted", "<i4"), ("n_eligible", "<i4"), ("rounds", "<i4"), ("n_out", "<i4"),
                         ("mode_version", "<u4"), ("pad", "<i4")])


def decode_results(raw: np.ndarray, n: int) -> list:
    """Result dicts of the first n rl_result records in a byte buffer."""
    rec = np.frombuffer(np.ascontiguousarray(raw).data, dtype=RESULT_DTYPE, count=n)
    poses = rec["cam_to_world"].reshape(n, 4, 4)
    out = []
    for k in range(n):
        r = rec[k]
        out.append(dict(pose=poses[k].copy(), energy=float(r["energy"]), mean_energy=float(r["mean_energy"]),
                        status="ok" if r["status"] == RL_OK else "no_pose", n_valid=int(r["n_valid"]),
                        n_inliers=int(r["n_inliers"]), winner=int(r["winner"]), refitted=bool(r["refitted"]),
                        n_eligible=int(r["n_eligible"]), rounds=int(r["rounds"]), n_out=int(r["n_out"]),
                        mode_version=int(r["mode_version"])))
    return out


class RelocOpts(ctypes.Structure):
    _fields_ = [("n_hypotheses", ctypes.c_int32), ("n_cull", ctypes.c_int32), ("n_out", ctypes.c_int32),
                ("final_refine", ctypes.c_int32), ("pose_update", ctypes.c_int32),
                ("max_iterations", ctypes.c_int32), ("eta", ctypes.c_int32), ("use_covariance", ctypes.c_int32),
                ("min_squared_distance", ctypes.c_float), ("max_translation_error", ctypes.c_float)]


class Request(ctypes.Structure):
    _fields_ = [("room", ctypes.c_void_p), ("frame", Frame), ("request_seed", ctypes.c_uint64),
                ("n_hypotheses", ctypes.c_int32), ("pose_update", ctypes.c_int32), ("kind", ctypes.c_int32),
                ("cam_to_world", ctypes.c_float * 16)]


REQ_RELOCALISE, REQ_ADAPT = 0, 1


class AdaptRequest:
    """An adaptation request of a batch: room, frame (CUDA tensors, intrinsics)
    and the frame's camera->world pose."""
    __slots__ = ("room", "depth", "rgb", "K", "pose")

    def __init__(self, room, depth, rgb, K, pose):
        self.room, self.depth, self.rgb, self.K, self.pose = room, depth, rgb, K, pose


class ForestParams(ctypes.Structure):
    _fields_ = [("n_trees", ctypes.c_int32), ("depth", ctypes.c_int32), ("p_depth", ctypes.c_float),
                ("offset_range", ctypes.c_float), ("tau_depth", ctypes.c_float), ("tau_colour", ctypes.c_float),
                ("seed", ctypes.c_uint64)]


class BatchParams(ctypes.Structure):
    _fields_ = [("max_frames", ctypes.c_int32), ("max_width", ctypes.c_int32),
                ("max_height", ctypes.c_int32), ("max_hypotheses", ctypes.c_int32),
                ("max_eta", ctypes.c_int32), ("max_rounds", ctypes.c_int32),
                ("n_trees", ctypes.c_int32), ("max_modes_per_pixel", ctypes.c_int32)]


# every symbol include/rl.h declares
EXPORTS = [
    "rl_params_preset", "rl_params_validate", "relocaliser_state_bytes", "relocaliser_create",
    "relocaliser_destroy", "relocaliser_adapt", "relocaliser_update_modes",
    "relocaliser_relocalise", "relocaliser_relocalise_ex", "relocaliser_buffer",
    "relocaliser_set_trace", "rl_batch_workspace_bytes", "rl_batch_create", "rl_batch_destroy",
    "rl_batch_relocalise", "rl_batch_relocalise_async", "rl_last_error", "rl_version",
    "relocaliser_set_timer", "rl_batch_set_timer", "relocaliser_relocalise_opts", "rl_plane_scores",
    "relocaliser_set_mode_schedule", "relocaliser_set_schedule", "rl_batch_set_schedule",
    "relocaliser_set_degeneracy_screen", "rl_batch_set_degeneracy_screen",
    "rl_depth_scores", "rl_forest_generate", "relocaliser_save", "relocaliser_load",
    "rl_depth_scores_noalloc",
]

# launch schedules the library accepts (iterations per thread, fast waves,
# tree levels the traversal reads from LDS)
SCHEDULE_IPT = (2, 4, 8)
SCHEDULE_FAST_WAVES = (1, 2, 4)
SCHEDULE_LDS_LEVELS = (8, 6)
SCHEDULE_SCORE_WINDOWS = (0, 2)

TIMER_NONE, TIMER_TRAVERSE, TIMER_HYP_SEARCH, TIMER_RANSAC = 0, 1, 2, 3

_lib = None


def lib():
    """Loads librl.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1810_12163_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        P, I32, U64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64
        L.rl_params_preset.argtypes = [ctypes.c_char_p, ctypes.POINTER(Params)]
        L.rl_params_validate.argtypes = [ctypes.POINTER(Params)]
        L.relocaliser_state_bytes.argtypes = [ctypes.POINTER(Params), I32, I32,
                                              ctypes.POINTER(ctypes.c_size_t),
                                              ctypes.POINTER(ctypes.c_size_t)]
        L.relocaliser_create.argtypes = [ctypes.POINTER(Params), P, I32, I32, P, P, P,
                                         ctypes.POINTER(ctypes.c_void_p)]
        L.relocaliser_destroy.argtypes = [P]
        L.relocaliser_adapt.argtypes = [P, ctypes.POINTER(Frame), P, I32]
        L.relocaliser_update_modes.argtypes = [P]
        L.relocaliser_relocalise.argtypes = [P, ctypes.POINTER(Frame), U64, P, P, P]
        L.relocaliser_relocalise_ex.argtypes = [P, ctypes.POINTER(Frame), U64, ctypes.POINTER(Result)]
        L.relocaliser_buffer.argtypes = [P, I32, ctypes.POINTER(ctypes.c_size_t),
                                         ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(I32)]
        L.relocaliser_set_trace.argtypes = [P, I32]
        L.rl_batch_workspace_bytes.argtypes = [ctypes.POINTER(BatchParams), ctypes.POINTER(ctypes.c_size_t)]
        L.rl_batch_create.argtypes = [ctypes.POINTER(BatchParams), P, P, ctypes.POINTER(ctypes.c_void_p)]
        L.rl_batch_destroy.argtypes = [P]
        L.rl_batch_relocalise.argtypes = [P, P, I32, P, I32]
        L.rl_batch_relocalise_async.argtypes = [P, P, I32, P, I32]
        L.relocaliser_set_timer.argtypes = [P, I32, P, P]
        L.relocaliser_relocalise_opts.argtypes = [P, ctypes.POINTER(Frame), U64, ctypes.POINTER(RelocOpts),
                                                  ctypes.POINTER(Result)]
        L.rl_plane_scores.argtypes = [P, ctypes.POINTER(Frame), P, I32, P, I32, P]
        L.rl_batch_set_timer.argtypes = [P, I32, P, P]
        L.relocaliser_set_mode_schedule.argtypes = [P, I32]
        L.relocaliser_set_schedule.argtypes = [P, I32, I32, I32, I32]
        L.rl_forest_generate.argtypes = [ctypes.POINTER(ForestParams), P, ctypes.POINTER(ctypes.c_size_t)]
        L.relocaliser_save.argtypes = [P, ctypes.c_char_p]
        L.relocaliser_load.argtypes = [P, ctypes.c_char_p]
        L.rl_batch_set_schedule.argtypes = [P, I32, I32, I32, I32]
        L.relocaliser_set_degeneracy_screen.argtypes = [P, I32]
        L.rl_batch_set_degeneracy_screen.argtypes = [P, I32]
        L.rl_depth_scores.argtypes = [P, ctypes.POINTER(Frame), P, I32, P, I32, ctypes.c_float, ctypes.c_float,
                                      P, P, P]
        L.rl_depth_scores_noalloc.argtypes = [ctypes.POINTER(Frame), P, I32, P, I32, ctypes.c_float,
                                              ctypes.c_float, P, P, P, P]
        L.rl_last_error.restype = ctypes.c_char_p
        L.rl_version.restype = ctypes.c_char_p
        for name in EXPORTS:
            getattr(L, name)            # every declared entry point must resolve
        _lib = L
    return _lib


def _check(status, allow=(RL_OK,)):
    if status not in allow:
        raise RlError(status, lib().rl_last_error().decode())
    return status


def forest_generate(n_trees: int, depth: int, seed: int, p_depth: float = 0.4, offset_range: float = 130.0,
                    tau_depth: float = 0.2, tau_colour: float = 64.0) -> np.ndarray:
    """A random forest (rl_forest_generate): (n_trees, 2^depth - 1) node records."""
    fp = ForestParams(int(n_trees), int(depth), float(p_depth), float(offset_range), float(tau_depth),
                      float(tau_colour), int(seed))
    nb = ctypes.c_size_t()
    _check(lib().rl_forest_generate(ctypes.byref(fp), None, ctypes.byref(nb)))
    out = np.zeros((int(n_trees), (1 << int(depth)) - 1), dtype=NODE_DTYPE)
    assert out.nbytes == nb.value
    _check(lib().rl_forest_generate(ctypes.byref(fp), out.ctypes.data, ctypes.byref(nb)))
    return out


def params_struct(d: dict) -> Params:
    p = Params()
    for name, ctype in Params._fields_:
        if name not in d:
            raise KeyError(f"parameter {name} missing")
        setattr(p, name, d[name])
    return p


def room_state_bytes(params: dict, max_width: int, max_height: int):
    """(persistent, scratch) device bytes of a room (relocaliser_state_bytes)."""
    p = params_struct(params)
    pb, sb = ctypes.c_size_t(), ctypes.c_size_t()
    _check(lib().relocaliser_state_bytes(ctypes.byref(p), max_width, max_height, ctypes.byref(pb),
                                         ctypes.byref(sb)))
    return int(pb.value), int(sb.value)


def preset(name: str) -> dict:
    p = Params()
    _check(lib().rl_params_preset(name.encode(), ctypes.byref(p)))
    return {n: getattr(p, n) for n, _ in Params._fields_}


def _torch():
    import torch
    return torch


def _frame(depth, rgb, K) -> Frame:
    """The rl_frame of a (h, w) float32 depth tensor and an (h, w, 3) uint8
    colour tensor on the GPU, read in place: rows may be padded (any row
    stride), colour may be RGB or the first three channels of RGBA, and both
    may be views taking every second pixel of every second row (the 2x
    decimated frame, e.g. depth[::2, ::2]); K is the frame's own."""
    torch = _torch()
    if not (isinstance(depth, torch.Tensor) and isinstance(rgb, torch.Tensor)):
        raise TypeError("depth and rgb must be torch tensors on the GPU")
    if depth.dtype != torch.float32 or depth.dim() != 2 or not depth.is_cuda:
        raise TypeError("depth must be an (h, w) float32 CUDA tensor")
    h, w = depth.shape
    if rgb.dtype != torch.uint8 or rgb.dim() != 3 or tuple(rgb.shape[:2]) != (h, w) or rgb.shape[2] not in (3, 4) \
            or not rgb.is_cuda:
        raise TypeError("rgb must be an (h, w, 3) or (h, w, 4) uint8 CUDA tensor")
    sd0, sd1 = depth.stride()
    sr0, sr1, sr2 = rgb.stride()
    step = sd1
    ch = sr1 // step if step in (1, 2) else 0
    if step not in (1, 2) or sd0 % step or sr0 % step or sr2 != 1 or ch not in (3, 4) or sr1 != ch * step:
        raise TypeError("depth and rgb must take every pixel (or every second one, both alike) of rows with unit "
                        "element stride, colour with 3 or 4 bytes per pixel")
    f = Frame()
    f.width, f.height = int(w), int(h)
    f.depth, f.rgb = depth.data_ptr(), rgb.data_ptr()
    f.K = Intrinsics(*[float(v) for v in K])
    f.rgb_channels = ch
    f.step = step
    f.depth_pitch_bytes = sd0 * 4 // step
    f.rgb_pitch_bytes = sr0 // step
    return f


def _result(r: Result) -> dict:
    H = np.array(r.cam_to_world[:], dtype=np.float32).reshape(4, 4)
    return dict(pose=H, energy=float(r.energy), mean_energy=float(r.mean_energy),
                status="ok" if r.status == RL_OK else "no_pose", n_valid=int(r.n_valid),
                n_inliers=int(r.n_inliers), winner=int(r.winner), refitted=bool(r.refitted),
                n_eligible=int(r.n_eligible), rounds=int(r.rounds), n_out=int(r.n_out),
                mode_version=int(r.mode_version))


class Room:
    """One scene: forest, reservoirs and modes resident in device memory."""

    def __init__(self, params: dict, nodes: np.ndarray, max_width: int = 640, max_height: int = 480,
                 stream=None, device=None):
        torch = _torch()
        self.params = dict(params)
        self._p = params_struct(params)
        L = lib()
        pb, sb = ctypes.c_size_t(), ctypes.c_size_t()
        _check(L.relocaliser_state_bytes(ctypes.byref(self._p), max_width, max_height,
                                         ctypes.byref(pb), ctypes.byref(sb)))
        self.device = torch.device(device if device is not None else "cuda")
        self.persistent = torch.empty(pb.value, dtype=torch.uint8, device=self.device)
        self.scratch = torch.empty(sb.value, dtype=torch.uint8, device=self.device)
        # a stream of its own (default priority) so that relocalisation can replay a graph
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        nodes = np.ascontiguousarray(nodes)
        if nodes.dtype.itemsize != 16 or nodes.size != params["n_trees"] * ((1 << params["depth"]) - 1):
            raise ValueError("nodes must hold n_trees * (2^depth - 1) 16-byte records")
        self._nodes = nodes
        h = ctypes.c_void_p()
        _check(L.relocaliser_create(ctypes.byref(self._p), nodes.ctypes.data, max_width, max_height,
                                    self.persistent.data_ptr(), self.scratch.data_ptr(),
                                    self.stream.cuda_stream, ctypes.byref(h)))
        self.handle = h.value
        self.schedule = (4, 1, 8, 0)
        self.max_width, self.max_height = max_width, max_height

    def close(self):
        if getattr(self, "handle", None):
            self.stream.synchronize()          # nothing of this room may still be in flight
            lib().relocaliser_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _follow(self, *tensors):
        """Orders the room's stream after the caller's current stream (where
        the frame tensors were written), and keeps the caching allocator from
        reusing those tensors' memory before the room's stream has read them."""
        self.stream.wait_stream(_torch().cuda.current_stream(self.device))
        for t in tensors:
            t.record_stream(self.stream)

    def adapt(self, depth, rgb, K, pose, reliable: bool = True, record: bool = True):
        """record=False: the frame tensors' memory is kept by the caller until
        the adaptation has completed (no record_stream)."""
        f = _frame(depth, rgb, K)
        H = np.ascontiguousarray(np.asarray(pose, dtype=np.float32).reshape(16))
        if record:
            self._follow(depth, rgb)
        else:
            self._follow()
        _check(lib().relocaliser_adapt(self.handle, ctypes.byref(f), H.ctypes.data, 1 if reliable else 0))

    def update_modes(self):
        self._follow()
        _check(lib().relocaliser_update_modes(self.handle))

    def set_mode_schedule(self, leaves_per_frame: int):
        """0: exact mode update before each relocalisation; K > 0: RQS of the
        next K leaves (round robin) after each adapted frame."""
        _check(lib().relocaliser_set_mode_schedule(self.handle, int(leaves_per_frame)))

    def save(self, path: str):
        """Writes the room's persistent state to a file (relocaliser_save)."""
        _check(lib().relocaliser_save(self.handle, str(path).encode()))

    def load(self, path: str):
        """Reads a saved room of the same forest shape (relocaliser_load)."""
        _check(lib().relocaliser_load(self.handle, str(path).encode()))

    def set_schedule(self, ipt: int, fast_waves: int, lds_levels: int = 8, score_window: int = 0):
        """Result-invariant launch schedule: search iterations per thread
        (2, 4, 8), all-rounds scoring width in waves (1, 2, 4), the tree
        levels the traversal reads from LDS (6, 8) and the rounds of the
        first all-rounds scoring pass (0 = all in one pass, 1..3)."""
        _check(lib().relocaliser_set_schedule(self.handle, int(ipt), int(fast_waves), int(lds_levels), int(score_window)))
        self.schedule = (int(ipt), int(fast_waves), int(lds_levels), int(score_window))

    def set_degeneracy_screen(self, on: bool):
        """Result-invariant: with the screen off every triplet passing checks
        1-3 reaches the exact degeneracy test (relocaliser_set_degeneracy_screen)."""
        _check(lib().relocaliser_set_degeneracy_screen(self.handle, 1 if on else 0))

    def relocalise(self, depth, rgb, K, request_seed: int = 0, n_hypotheses: int = 0, n_cull: int = 0,
                   n_out: int = 0, final_refine: int = -1, pose_update: int = -1, max_iterations: int = 0,
                   eta: int = 0, use_covariance: int = -1, min_squared_distance: float = -1.0,
                   max_translation_error: float = -1.0) -> dict:
        """One frame; the optional hypothesis and RANSAC settings override the room's for this call."""
        f = _frame(depth, rgb, K)
        r = Result()
        self._follow(depth, rgb)
        opts = RelocOpts(int(n_hypotheses), int(n_cull), int(n_out), int(final_refine), int(pose_update),
                         int(max_iterations), int(eta), int(use_covariance), float(min_squared_distance),
                         float(max_translation_error))
        _check(lib().relocaliser_relocalise_opts(self.handle, ctypes.byref(f), int(request_seed),
                                                 ctypes.byref(opts), ctypes.byref(r)), allow=(RL_OK, RL_NO_POSE))
        return _result(r)

    def plane_scores(self, depth, rgb, K, surfaces: np.ndarray, poses12: np.ndarray) -> np.ndarray:
        """Model-based score (mean nearest-surface distance) of each pose."""
        f = _frame(depth, rgb, K)
        S = np.ascontiguousarray(surfaces, dtype=np.float32).reshape(-1, 16)
        P = np.ascontiguousarray(poses12, dtype=np.float32).reshape(-1, 12)
        out = np.zeros(P.shape[0], dtype=np.float64)
        self._follow(depth, rgb)
        _check(lib().rl_plane_scores(self.handle, ctypes.byref(f), S.ctypes.data, S.shape[0], P.ctypes.data,
                                     P.shape[0], out.ctypes.data))
        return out

    def depth_scores(self, depth, rgb, K, surfaces: np.ndarray, poses12: np.ndarray, min_depth: float = 0.5,
                     max_depth: float = 4.0):
        """Depth-raycast scores of Eq. 6-7 per pose: (s, mu, counts (n, 2))."""
        f = _frame(depth, rgb, K)
        S = np.ascontiguousarray(surfaces, dtype=np.float32).reshape(-1, 16)
        P = np.ascontiguousarray(poses12, dtype=np.float32).reshape(-1, 12)
        s = np.zeros(P.shape[0], dtype=np.float64)
        mu = np.zeros(P.shape[0], dtype=np.float64)
        cnt = np.zeros((P.shape[0], 2), dtype=np.int64)
        self._follow(depth, rgb)
        _check(lib().rl_depth_scores(self.handle, ctypes.byref(f), S.ctypes.data, S.shape[0], P.ctypes.data,
                                     P.shape[0], float(min_depth), float(max_depth), s.ctypes.data,
                                     mu.ctypes.data, cnt.ctypes.data))
        return s, mu, cnt

    def survivors(self, k: int):
        """(slots, poses (k, 12)) of the best k hypotheses of the last relocalisation."""
        slots = self.buffer_np(BUF_SURVIVORS, np.int32)[:k].copy()
        hy = self.buffer_np(BUF_HYPS, HYP_DTYPE)
        poses = np.concatenate([hy["R"][slots], hy["t"][slots]], axis=1).astype(np.float32)
        return slots, poses

    def set_trace(self, on: bool):
        _check(lib().relocaliser_set_trace(self.handle, 1 if on else 0))

    def set_timer(self, kernel: int, start=None, stop=None):
        """Record torch.cuda.Event pair (enable_timing=True) around a kernel."""
        _check(lib().relocaliser_set_timer(self.handle, kernel, start.cuda_event if start else None,
                                           stop.cuda_event if stop else None))

    def buffer(self, which: int):
        """torch uint8 view of an internal array (see RL_BUF_* in rl.h)."""
        off, nb, reg = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_int32()
        _check(lib().relocaliser_buffer(self.handle, which, ctypes.byref(off), ctypes.byref(nb),
                                        ctypes.byref(reg)))
        base = self.persistent if reg.value == 0 else self.scratch
        return base[off.value:off.value + nb.value]

    def buffer_np(self, which: int, dtype) -> np.ndarray:
        self.stream.synchronize()
        with _torch().cuda.stream(self.stream):
            out = self.buffer(which).cpu().numpy().view(dtype)
        return out


class Batch:
    """Many frames from several rooms in one launch sequence (optionally a HIP graph)."""

    def __init__(self, max_frames: int, max_width: int, max_height: int, max_hypotheses: int,
                 max_eta: int, max_rounds: int, n_trees: int, max_modes_per_pixel: int,
                 stream=None, device=None):
        torch = _torch()
        self._bp = BatchParams(max_frames, max_width, max_height, max_hypotheses, max_eta,
                               max_rounds, n_trees, max_modes_per_pixel)
        nb = ctypes.c_size_t()
        L = lib()
        _check(L.rl_batch_workspace_bytes(ctypes.byref(self._bp), ctypes.byref(nb)))
        self.device = torch.device(device if device is not None else "cuda")
        self.workspace = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        # a stream of its own (default priority): graph capture cannot use the legacy stream
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        h = ctypes.c_void_p()
        _check(L.rl_batch_create(ctypes.byref(self._bp), self.workspace.data_ptr(),
                                 self.stream.cuda_stream, ctypes.byref(h)))
        self.handle = h.value
        self.schedule = (4, 1, 8, 2)
        self.max_frames = max_frames

    def close(self):
        if getattr(self, "handle", None):
            self.stream.synchronize()
            lib().rl_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_timer(self, kernel: int, start=None, stop=None):
        """Record torch.cuda.Event pair (enable_timing=True) around a kernel."""
        _check(lib().rl_batch_set_timer(self.handle, kernel, start.cuda_event if start else None,
                                        stop.cuda_event if stop else None))

    def set_schedule(self, ipt: int, fast_waves: int, lds_levels: int = 8, score_window: int = 2):
        """Result-invariant launch schedule: search iterations per thread
        (2, 4, 8), all-rounds scoring width in waves (1, 2, 4), the tree
        levels the traversal reads from LDS (6, 8) and the rounds of the
        first all-rounds scoring pass (0 = all in one pass, 1..3; a batch's
        default is 2)."""
        _check(lib().rl_batch_set_schedule(self.handle, int(ipt), int(fast_waves), int(lds_levels), int(score_window)))
        self.schedule = (int(ipt), int(fast_waves), int(lds_levels), int(score_window))

    def set_degeneracy_screen(self, on: bool):
        """Result-invariant degeneracy screen of the search (rl_batch_set_degeneracy_screen)."""
        _check(lib().rl_batch_set_degeneracy_screen(self.handle, 1 if on else 0))

    def _requests(self, reqs, record=True):
        torch = _torch()
        self.stream.wait_stream(torch.cuda.current_stream(self.device))   # frames were made there
        arr = (Request * len(reqs))()
        for i, q in enumerate(reqs):
            if isinstance(q, AdaptRequest):
                if record:
                    q.depth.record_stream(self.stream)
                    q.rgb.record_stream(self.stream)
                arr[i].room = q.room.handle
                arr[i].frame = _frame(q.depth, q.rgb, q.K)
                arr[i].kind = REQ_ADAPT
                H = np.asarray(q.pose, dtype=np.float32).reshape(16)
                for k in range(16):
                    arr[i].cam_to_world[k] = float(H[k])
                continue
            if record:
                q[1].record_stream(self.stream)
                q[2].record_stream(self.stream)
            room, depth, rgb, K = q[0], q[1], q[2], q[3]
            seed = q[4] if len(q) > 4 else 0
            nh = q[5] if len(q) > 5 else 0
            pu = q[6] if len(q) > 6 else 0
            arr[i].room = room.handle
            arr[i].frame = _frame(depth, rgb, K)
            arr[i].request_seed = int(seed)
            arr[i].n_hypotheses = int(nh)
            arr[i].pose_update = int(pu)
        return arr

    def relocalise(self, reqs, use_graph: bool = True) -> list:
        """reqs: sequence of (room, depth, rgb, K[, request_seed[, n_hypotheses[, pose_update]]]) and
        AdaptRequest; pose_update 0 = the room's value, 1 = LM on, -1 = off.  The adaptations run after
        every relocalisation of the batch, in order."""
        arr = self._requests(reqs)
        res = (Result * len(reqs))()
        _check(lib().rl_batch_relocalise(self.handle, arr, len(reqs), res, 1 if use_graph else 0))
        return [_result(r) for r in res]

    def relocalise_async(self, reqs, dev_results, use_graph: bool = True, record: bool = True):
        """Queues the batch; dev_results: torch uint8 CUDA tensor of >= len(reqs) * sizeof(Result) bytes.
        record=False: the frame tensors' memory is kept by the caller until the
        batch has completed (no record_stream with torch's allocator)."""
        arr = self._requests(reqs, record)
        dev_results.record_stream(self.stream)
        _check(lib().rl_batch_relocalise_async(self.handle, arr, len(reqs), dev_results.data_ptr(),
                                               1 if use_graph else 0))

    @staticmethod
    def decode(host_bytes: np.ndarray, n: int) -> list:
        out = []
        raw = np.ascontiguousarray(host_bytes).view(np.uint8)
        for i in range(n):
            r = Result.from_buffer_copy(raw[i * ctypes.sizeof(Result):(i + 1) * ctypes.sizeof(Result)].tobytes())
            out.append(_result(r))
        return out


def depth_scores_noalloc(depth, rgb, K, surfaces: np.ndarray, poses12: np.ndarray, min_depth: float = 0.5,
                         max_depth: float = 4.0):
    """Depth-raycast scores of Eq. 6-7 per pose, (s, mu, counts (n, 2)), with the
    library's fixed device work space (no room, nothing allocated); runs on
    torch's current stream."""
    torch = _torch()
    f = _frame(depth, rgb, K)
    S = np.ascontiguousarray(surfaces, dtype=np.float32).reshape(-1, 16)
    P = np.ascontiguousarray(poses12, dtype=np.float32).reshape(-1, 12)
    s = np.zeros(P.shape[0], dtype=np.float64)
    mu = np.zeros(P.shape[0], dtype=np.float64)
    cnt = np.zeros((P.shape[0], 2), dtype=np.int64)
    st = torch.cuda.current_stream(depth.device).cuda_stream
    _check(lib().rl_depth_scores_noalloc(ctypes.byref(f), S.ctypes.data, S.shape[0], P.ctypes.data, P.shape[0],
                                         float(min_depth), float(max_depth), st, s.ctypes.data, mu.ctypes.data,
                                         cnt.ctypes.data))
    return s, mu, cnt


def rounds_for(N: int, n_cull: int, n_out: int) -> int:
    """RANSAC rounds for N hypotheses (initial cull, then halving to n_out)."""
    n, rounds, first = N, 0, True
    while first or n > n_out:
        keep = n_cull if (first and n_cull < n) else ((n + 1) // 2 if n > n_out else n)
        n, rounds, first = keep, rounds + 1, False
    return rounds
