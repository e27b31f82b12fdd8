"""CPU oracle of the relocaliser's per-frame path (Cavallari et al., TPAMI
2019, arXiv 1810.12163).

TEST INFRASTRUCTURE ONLY: the test-suite, the package smoke check and the
benchmark's CPU-baseline leg are the only users.  It shares no code with the
GPU path (it neither imports the package nor loads its library), and the GPU
path never falls back to it.

The arithmetic lives in ``rl_oracle.c`` (plain C, FP64 except the float32
feature/routing definition); this module builds it with gcc, loads it with
ctypes and composes the per-frame steps in the paper's order:

* adaptation (Sec. 3.2.2): grid pixels -> leaves -> world points -> reservoirs;
* modes (Sec. 3.2.2 step 3): Really Quick Shift per dirty leaf;
* relocalisation (Sec. 3.2.3): dense traversal, eligible pixels, hypothesis
  generation with the three checks and Kabsch, preemptive RANSAC rounds on
  Eq. 5, and the optional final inlier refit.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rl_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_CFLAGS = ["-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared"]

RES_NONE = 0xFFFF


def build(force: bool = True) -> str:
    """Compile the oracle library with gcc (contraction off, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", *_CFLAGS, "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        _lib = ctypes.CDLL(_LIB)
        _declare(_lib)
    return _lib


P = ctypes.c_void_p
I32 = ctypes.c_int
U64 = ctypes.c_uint64
F32 = ctypes.c_float
F64 = ctypes.c_double


def _declare(L):
    L.oracle_set_threads.argtypes = [I32]
    L.oracle_set_threads.restype = I32
    L.oracle_philox4x32.argtypes = [P, P, P]
    L.oracle_traverse.argtypes = [P, P, I32, I32, P, I32, I32, I32, P, I32, P]
    L.oracle_adapt.argtypes = [P, P, I32, I32, P, P, P, I32, I32, I32, I32, U64, P, P, P]
    L.oracle_adapt.restype = ctypes.c_long
    L.oracle_rqs_leaf.argtypes = [P, I32, F64, F64, I32, I32, F64, P, P]
    L.oracle_rqs_leaf.restype = I32
    L.oracle_update_modes.argtypes = [P, P, P, I32, I32, I32, F64, F64, I32, I32, F64, P, P, I32]
    L.oracle_update_modes.restype = ctypes.c_long
    L.oracle_update_modes_range.argtypes = [P, P, I32, I32, I32, F64, F64, I32, I32, F64, P, P,
                                            ctypes.c_long, ctypes.c_long]
    L.oracle_update_modes_range.restype = ctypes.c_long
    L.oracle_kabsch.argtypes = [P, P, I32, P, P, P]
    L.oracle_kabsch.restype = I32
    L.oracle_hypotheses.argtypes = [P, P, I32, I32, P, P, P, P, I32, I32, I32, P, I32, I32, I32,
                                    F32, F64, F64, U64, U64, P, P, P, P, P, P]
    L.oracle_pixel_energy.argtypes = [P, I32, I32, P, P, P, P, I32, I32, I32, P, I32, I32]
    L.oracle_pixel_energy.restype = F64
    L.oracle_ransac.argtypes = [P, I32, I32, P, P, P, P, I32, I32, I32, P, I32, P, P, I32,
                                I32, I32, I32, I32, U64, U64, P, P, P, P, I32, P, I32, P, P,
                                I32, I32, P]
    L.oracle_lm_refine.argtypes = [P, I32, I32, P, P, P, P, I32, I32, I32, P, I32, I32, I32, P]
    L.oracle_lm_refine.restype = F64
    L.oracle_lm_linearise.argtypes = [P, I32, I32, P, P, P, P, I32, I32, I32, P, I32, I32, P, P, P]
    L.oracle_lm_linearise.restype = F64
    L.oracle_se3_exp.argtypes = [P, P, P]
    L.oracle_ransac.restype = I32
    L.oracle_refine.argtypes = [P, I32, I32, P, P, P, P, I32, I32, I32, P, P, I32, F64, I32, P, P]
    L.oracle_refine.restype = I32
    L.oracle_plane_scores.argtypes = [P, I32, I32, P, P, I32, P, I32, P]
    L.oracle_depth_scores.argtypes = [P, I32, I32, P, P, I32, P, I32, F32, F32, P, P, P]


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def philox4x32(counter, key):
    """Philox4x32-10 block for a 4-word counter and 2-word key (uint32)."""
    c = _c(np.asarray(counter, dtype=np.uint32), np.uint32)
    k = _c(np.asarray(key, dtype=np.uint32), np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox4x32(_p(c), _p(k), _p(out))
    return out


def kabsch(xc, xw):
    """Returns (ok, R 3x3, t 3, singular values) with x^W ~ R x^C + t."""
    xc = _c(xc, np.float64).reshape(-1, 3)
    xw = _c(xw, np.float64).reshape(-1, 3)
    R = np.zeros(9)
    t = np.zeros(3)
    sv = np.zeros(3)
    ok = lib().oracle_kabsch(_p(xc), _p(xw), xc.shape[0], _p(R), _p(t), _p(sv))
    return bool(ok), R.reshape(3, 3), t, sv


def rqs_leaf(entries, sigma, tau_c, min_size, max_modes, lam):
    """Modes of one reservoir. entries: (n, 4) float32 (xyz + colour bits).
    Returns (rows (nm, 16) float32, detail (nm, 16) float64)."""
    e = _c(entries, np.float32).reshape(-1, 4)
    rows = np.zeros((max(max_modes, 1), 16), dtype=np.float32)
    det = np.zeros((max(max_modes, 1), 16), dtype=np.float64)
    nm = lib().oracle_rqs_leaf(_p(e), e.shape[0], sigma, tau_c, min_size, max_modes, lam,
                               _p(rows), _p(det))
    return rows[:nm], det[:nm]


def pack_colour(rgb):
    """uint8 (n, 3) -> float32 bit pattern of r | g<<8 | b<<16."""
    rgb = np.asarray(rgb, dtype=np.uint32)
    return (rgb[:, 0] | (rgb[:, 1] << 8) | (rgb[:, 2] << 16)).view(np.float32)


def traverse(depth, rgb, K_unused, nodes, T, D, ref_width, pix=None):
    depth = _c(depth, np.float32)
    rgb = _c(rgb, np.uint8)
    h, w = depth.shape
    nodes = np.ascontiguousarray(nodes)
    pixa = None if pix is None else _c(pix, np.int32)
    n = w * h if pix is None else len(pixa)
    out = np.zeros((n, T), dtype=np.uint16)
    lib().oracle_traverse(_p(depth), _p(rgb), w, h, _p(nodes), T, D, ref_width, _p(pixa),
                          n, _p(out))
    return out


class Oracle:
    """One room: forest structure, reservoirs and modes, all in host memory."""

    def __init__(self, params: dict, nodes: np.ndarray):
        self.p = dict(params)
        self.T = int(params["n_trees"])
        self.D = int(params["depth"])
        self.L = 1 << self.D
        self.kappa = int(params["reservoir_capacity"])
        self.M = int(params["max_cluster_count"])
        self.ref_width = int(params["ref_width"])
        self.nodes = np.ascontiguousarray(nodes)
        assert self.nodes.shape == (self.T, self.L - 1)
        TL = self.T * self.L
        self.reservoir = np.zeros(TL * self.kappa * 4, dtype=np.float32)
        self.seen = np.zeros(TL, dtype=np.uint32)
        self.dirty = np.zeros(TL, dtype=np.uint8)
        self.modes = np.zeros(TL * self.M * 16, dtype=np.float32)
        self.nmodes = np.zeros(TL, dtype=np.uint8)
        self.rr_cursor = 0

    # -- adaptation ---------------------------------------------------------
    def adapt(self, depth, rgb, K, pose, reliable=True):
        if not reliable:
            return 0
        depth = _c(depth, np.float32)
        rgb = _c(rgb, np.uint8)
        h, w = depth.shape
        Kf = _c(np.asarray(K, dtype=np.float32), np.float32)
        H = _c(np.asarray(pose, dtype=np.float32).reshape(16), np.float32)
        return lib().oracle_adapt(_p(depth), _p(rgb), w, h, _p(Kf), _p(H), _p(self.nodes),
                                  self.T, self.D, self.ref_width, self.kappa,
                                  int(self.p["seed"]), _p(self.reservoir), _p(self.seen),
                                  _p(self.dirty))

    def update_modes(self, all_leaves=False):
        p = self.p
        return lib().oracle_update_modes(_p(self.reservoir), _p(self.seen), _p(self.dirty),
                                         self.T, self.D, self.kappa, float(p["clusterer_sigma"]),
                                         float(p["clusterer_tau"]), int(p["min_cluster_size"]),
                                         self.M, float(p["cov_regulariser"]), _p(self.modes),
                                         _p(self.nmodes), 1 if all_leaves else 0)

    def update_modes_round_robin(self, count: int):
        """Amortised schedule (Sec. 3.2.2): re-cluster the next `count` leaves
        in leaf-index order (t * 2^D + leaf), wrapping around."""
        p = self.p
        self.rr_cursor = lib().oracle_update_modes_range(
            _p(self.reservoir), _p(self.seen), self.T, self.D, self.kappa, float(p["clusterer_sigma"]),
            float(p["clusterer_tau"]), int(p["min_cluster_size"]), self.M, float(p["cov_regulariser"]),
            _p(self.modes), _p(self.nmodes), int(self.rr_cursor), int(count))
        return self.rr_cursor

    def reservoir_of(self, t, leaf):
        tl = t * self.L + leaf
        n = min(int(self.seen[tl]), self.kappa)
        e = self.reservoir[tl * self.kappa * 4:(tl * self.kappa + n) * 4]
        return e.reshape(n, 4)

    def modes_of(self, t, leaf):
        tl = t * self.L + leaf
        nm = int(self.nmodes[tl])
        return self.modes[tl * self.M * 16:(tl * self.M + nm) * 16].reshape(nm, 16)

    # -- relocalisation -----------------------------------------------------
    def traverse(self, depth, rgb, pix=None):
        return traverse(depth, rgb, None, self.nodes, self.T, self.D, self.ref_width, pix)

    def mode_counts(self, leaves):
        return mode_counts(leaves, self.nmodes, self.D)

    def relocalise(self, depth, rgb, K, request_seed=0, params=None, trace=True):
        """Full per-frame relocalisation; returns a dict of every stage's output."""
        p = dict(self.p if params is None else params)
        self.update_modes()
        leaves = self.traverse(depth, rgb)
        return estimate_pose(depth, rgb, K, leaves, self.nmodes, self.modes, self.T, self.D,
                             self.M, p, request_seed, trace)


def mode_counts(leaves, nmodes, D):
    """|M(u)| per pixel from an (npix, T) leaf array and the per-leaf mode counts."""
    L = 1 << D
    nm = np.zeros(leaves.shape[0], dtype=np.int32)
    for t in range(leaves.shape[1]):
        lf = leaves[:, t].astype(np.int64)
        ok = lf != RES_NONE
        nm[ok] += nmodes[t * L + lf[ok]]
    return nm


def eligible_pixels(depth, leaves, nmodes, D):
    """Pixels with valid depth and |M(u)| >= 1, in raster order (Sec. 3.2.3)."""
    d = np.asarray(depth, dtype=np.float32).reshape(-1)
    nm = mode_counts(leaves, nmodes, D)
    ok = (d > 0) & np.isfinite(d) & (nm >= 1)
    return np.flatnonzero(ok).astype(np.int32), nm


def estimate_pose(depth, rgb, K, leaves, nmodes, modes, T, D, M, p, request_seed=0, trace=True):
    """Sec. 3.2.3 from per-pixel leaves and per-leaf modes: eligible pixels,
    hypothesis generation, preemptive RANSAC and the optional final refit."""
    depth = _c(depth, np.float32)
    rgb = _c(rgb, np.uint8)
    leaves = _c(leaves, np.uint16)
    nmodes = _c(nmodes, np.uint8)
    modes = _c(modes, np.float32)
    h, w = depth.shape
    Kf = _c(np.asarray(K, dtype=np.float32), np.float32)
    eligible, nm = eligible_pixels(depth, leaves, nmodes, D)
    out = dict(leaves=leaves, nm=nm, eligible=eligible)
    N = int(p["max_pose_candidates"])
    hv = np.zeros(N, dtype=np.uint8)
    hit = np.zeros(N, dtype=np.int32)
    hpix = np.zeros((N, 3), dtype=np.int32)
    hmode = np.zeros((N, 3), dtype=np.int32)
    hpose = np.zeros((N, 12), dtype=np.float32)
    hpose64 = np.zeros((N, 12), dtype=np.float64)
    L = lib()
    L.oracle_hypotheses(_p(depth), _p(rgb), w, h, _p(Kf), _p(leaves), _p(nmodes), _p(modes), T, D,
                        M, _p(eligible), len(eligible), N,
                        int(p["max_candidate_generation_iterations"]), float(p["max_colour_linf"]),
                        float(p["min_squared_distance_between_sampled_modes"]),
                        float(p["max_translation_error_for_correct_pose"]), int(p["seed"]),
                        int(request_seed), _p(hv), _p(hit), _p(hpix), _p(hmode), _p(hpose),
                        _p(hpose64))
    out.update(hyp_valid=hv, hyp_iter=hit, hyp_pix=hpix, hyp_mode=hmode, hyp_pose=hpose,
               hyp_pose64=hpose64)
    eta = int(p["ransac_inliers_per_iteration"])
    n_out = int(p["max_relocalisations_to_output"])
    n_cull = int(p["max_pose_candidates_after_cull"])
    use_cov = int(p["use_prediction_covariance"])
    rcap = 64
    slots = np.zeros(max(n_out, 1), dtype=np.int32)
    energy = np.zeros(max(n_out, 1), dtype=np.float64)
    cnt = np.zeros(1, dtype=np.int32)
    Icap = eta * rcap
    Ilist = np.zeros(Icap, dtype=np.int32)
    round_n = np.zeros(rcap, dtype=np.int32)
    round_slots = np.zeros((rcap, N), dtype=np.int32) if trace else None
    round_energy = np.zeros((rcap, N), dtype=np.float64) if trace else None
    pose_update = int(p.get("pose_update", 0))
    refined = np.zeros((N, 12), dtype=np.float64)
    rounds = L.oracle_ransac(_p(depth), w, h, _p(Kf), _p(leaves), _p(nmodes), _p(modes), T, D, M,
                             _p(eligible), len(eligible), _p(hv), _p(hpose), N, eta, n_cull, n_out,
                             use_cov, int(p["seed"]), int(request_seed), _p(slots), _p(energy),
                             _p(cnt), _p(Ilist), Icap, _p(round_n), rcap, _p(round_slots),
                             _p(round_energy), pose_update, int(p.get("lm_iterations", 0)), _p(refined))
    k = int(cnt[0])
    nI = rounds * eta
    out.update(rounds=rounds, out_slots=slots[:k], out_energy=energy[:k],
               I=Ilist[:min(nI, Icap)], round_n=round_n[:rounds])
    if trace:
        out.update(round_slots=[round_slots[r, :round_n[r]] for r in range(rounds)],
                   round_energy=[round_energy[r, :round_n[r]] for r in range(rounds)])
    if k == 0:
        out.update(status="no_pose", pose=np.eye(4), energy=np.inf, mean_energy=np.inf,
                   n_inliers=0, refitted=False, winner=-1)
        return out
    win = int(slots[0])
    out.update(refined_pose64=refined)
    # the refined pose (FP64) rounded to float32, as a hypothesis pose is kept
    pose12 = refined[win].astype(np.float32) if pose_update else hpose[win].copy()
    n_inl, refitted = 0, False
    if int(p["final_refine"]):
        po = np.zeros(12)
        rf = ctypes.c_int(0)
        n_inl = L.oracle_refine(_p(depth), w, h, _p(Kf), _p(leaves), _p(nmodes), _p(modes), T, D,
                                M, _p(pose12), _p(Ilist), nI, float(p["inlier_threshold"]),
                                use_cov, _p(po), ctypes.byref(rf))
        refitted = bool(rf.value)
        final = po
    else:
        final = pose12.astype(np.float64)
    H = np.eye(4)
    H[:3, :3] = final[:9].reshape(3, 3)
    H[:3, 3] = final[9:]
    out.update(status="ok", pose=H, energy=float(energy[0]),
               mean_energy=float(energy[0]) / max(nI, 1), n_inliers=n_inl, refitted=refitted,
               winner=win)
    return out


def pixel_energy(depth, K, leaves, nmodes, modes, T, D, M, pose12, pix, use_cov=1):
    """One Eq. 5 term: min over M(u) of the Mahalanobis (or Euclidean) distance."""
    depth = _c(depth, np.float32)
    h, w = depth.shape
    Kf = _c(np.asarray(K, dtype=np.float32), np.float32)
    pose = _c(pose12, np.float32)
    return lib().oracle_pixel_energy(_p(depth), w, h, _p(Kf), _p(_c(leaves, np.uint16)),
                                     _p(_c(nmodes, np.uint8)), _p(_c(modes, np.float32)), T, D, M,
                                     _p(pose), int(pix), int(use_cov))


def surfaces_of(room) -> np.ndarray:
    """Surface records (16 float32 each) of an rlsynth room: p0, n, e1, e2,
    half-extents (a <= 0: infinite plane)."""
    out = np.zeros((len(room.surfaces), 16), dtype=np.float32)
    for i, s in enumerate(room.surfaces):
        out[i, 0:3] = s.p0
        out[i, 3:6] = s.n
        out[i, 6:9] = s.e1
        out[i, 9:12] = s.e2
        if s.half is not None:
            out[i, 12:14] = s.half
    return out


def plane_scores(depth, K, poses12, surfaces):
    """Mean distance of back-projected valid depth to the nearest surface, per pose."""
    depth = _c(depth, np.float32)
    h, w = depth.shape
    Kf = _c(np.asarray(K, dtype=np.float32), np.float32)
    P = _c(np.asarray(poses12, dtype=np.float32).reshape(-1, 12), np.float32)
    S = _c(surfaces, np.float32)
    out = np.zeros(P.shape[0])
    lib().oracle_plane_scores(_p(depth), w, h, _p(Kf), _p(P), P.shape[0], _p(S), S.shape[0], _p(out))
    return out


def depth_scores(depth, K, poses12, surfaces, min_depth: float, max_depth: float):
    """Depth-raycast scores of Eq. 6-7 per pose: (s, mu, counts) with counts
    (n_poses, 2) = (valid raycast pixels, pixels valid in both)."""
    depth = _c(depth, np.float32)
    h, w = depth.shape
    Kf = _c(np.asarray(K, dtype=np.float32), np.float32)
    P = _c(np.asarray(poses12, dtype=np.float32).reshape(-1, 12), np.float32)
    S = _c(surfaces, np.float32)
    s = np.zeros(P.shape[0])
    mu = np.zeros(P.shape[0])
    cnt = np.zeros((P.shape[0], 2), dtype=np.int64)
    lib().oracle_depth_scores(_p(depth), w, h, _p(Kf), _p(P), P.shape[0], _p(S), S.shape[0],
                              float(min_depth), float(max_depth), _p(s), _p(mu), _p(cnt))
    return s, mu, cnt


def se3_exp(xi):
    """exp of xi = (omega, v) in se(3): (R 3x3, t 3)."""
    xi = _c(xi, np.float64)
    R = np.zeros(9)
    t = np.zeros(3)
    lib().oracle_se3_exp(_p(xi), _p(R), _p(t))
    return R.reshape(3, 3), t


def _lm_args(depth, K, leaves, nmodes, modes, I):
    depth = _c(depth, np.float32)
    h, w = depth.shape
    return (depth, w, h, _c(np.asarray(K, dtype=np.float32), np.float32), _c(leaves, np.uint16),
            _c(nmodes, np.uint8), _c(modes, np.float32), _c(I, np.int32))


def lm_refine(depth, K, leaves, nmodes, modes, T, D, M, I, pose12, use_cov=1, iters=10):
    """Levenberg-Marquardt refinement in se(3) of one pose on E over the pixel
    list I; returns (energy, refined pose12 FP64)."""
    d, w, h, Kf, lv, nm, md, Ii = _lm_args(depth, K, leaves, nmodes, modes, I)
    pose = _c(np.array(pose12, dtype=np.float64), np.float64).copy()
    E = lib().oracle_lm_refine(_p(d), w, h, _p(Kf), _p(lv), _p(nm), _p(md), T, D, M, _p(Ii), len(Ii),
                               int(use_cov), int(iters), _p(pose))
    return E, pose


def lm_linearise(depth, K, leaves, nmodes, modes, T, D, M, I, pose12, use_cov=1):
    """(E, N 6x6, g 6) of the weighted normal equations at pose12."""
    d, w, h, Kf, lv, nm, md, Ii = _lm_args(depth, K, leaves, nmodes, modes, I)
    pose = _c(np.array(pose12, dtype=np.float64), np.float64)
    N = np.zeros(36)
    g = np.zeros(6)
    E = lib().oracle_lm_linearise(_p(d), w, h, _p(Kf), _p(lv), _p(nm), _p(md), T, D, M, _p(Ii), len(Ii),
                                  int(use_cov), _p(pose), _p(N), _p(g))
    return E, N.reshape(6, 6), g
