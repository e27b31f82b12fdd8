"""Oracle pins: the rejection side of hypothesis generation (Sec. 3.2.3).

The oracle's slot h keeps the FIRST generation iteration whose triplet passes
the colour check on the randomly chosen pair, the distance check, the
rigidity check and a non-degenerate Kabsch fit.  The acceptance side is
pinned elsewhere (accepted triplets satisfy the checks); these tests pin the
other side: every iteration before the accepted one must fail at least one
check, and an invalid slot must fail them all.  The checks are re-evaluated
here in plain numpy from the paper's definitions, with only the Philox draws
(pinned against rocRAND) and the documented draw mapping taken over:

* block 0 of iteration it (counter (HYP | 0, h, it, 0)): k* = the pair the
  colour check looks at, its list entry and its mode within M(u);
* block 1 (counter (HYP | 1, h, it, 0)): the other two pairs in increasing
  order, list entries then modes;
* an integer in [0, n) is (u * n) >> 32.

Two plausible mistakes this catches and the acceptance-side tests do not:
applying the colour check to another pair than k*, and rejecting an
iteration that passes every check.  The strict comparisons of the distance
check (reject iff d^2 < min, Sec. 3.2.3) and of the rigidity check (reject
iff the difference exceeds the tolerance) are pinned at their exact
boundaries on a constructed 3-pixel frame.
"""
import numpy as np
import pytest

import oracle
from tests import ideal_scene

TAG_HYP = 2


def _u(r, n):
    return (int(r) * int(n)) >> 32


class Frame:
    """What the checks read: eligible list, per-pixel mode lists M(u)
    (mean, colour), depth, colour and intrinsics."""

    def __init__(self, depth, rgb, K, leaves, nmodes, modes, T, D, M, eligible):
        self.depth = np.asarray(depth, np.float32).reshape(-1)
        self.rgb = np.asarray(rgb, np.uint8).reshape(-1, 3)
        self.w = np.asarray(depth).shape[1]
        self.K = [float(np.float32(v)) for v in K]
        self.eligible = np.asarray(eligible)
        L = 1 << D
        rows = np.asarray(modes, np.float32).reshape(T * L, M, 16)
        lv = np.asarray(leaves).reshape(-1, T)
        nm = np.asarray(nmodes).reshape(-1)
        self.mlist = {}
        for p in self.eligible:
            lst = []
            for t in range(T):                       # tree-major concatenation
                lf = int(lv[p, t])
                if lf == 0xFFFF:
                    continue
                for m in range(int(nm[t * L + lf])):
                    lst.append(rows[t * L + lf, m])
            self.mlist[int(p)] = lst

    def camera_point(self, p):
        fx, fy, cx, cy = self.K
        d = float(self.depth[p])
        x, y = p % self.w, p // self.w
        return np.array([d * ((x - cx) / fx), d * ((y - cy) / fy), d])


def draws(key, slot, it):
    a = [int(v) for v in oracle.philox4x32([(TAG_HYP << 28) | 0, slot, it, 0], key)]
    b = [int(v) for v in oracle.philox4x32([(TAG_HYP << 28) | 1, slot, it, 0], key)]
    kc = _u(a[0], 3)
    others = [k for k in range(3) if k != kc]
    rp = {kc: a[1], others[0]: b[0], others[1]: b[1]}
    rm = {kc: a[2], others[0]: b[2], others[1]: b[3]}
    return kc, [rp[k] for k in range(3)], [rm[k] for k in range(3)]


def colour_fails(fr, p, row, theta):
    """Check 1 on one (pixel, mode) pair: L-infinity colour distance on the
    0..255 scale above theta, in float32."""
    diff = np.abs(fr.rgb[p].astype(np.float32) - row[10:13].astype(np.float32))
    return bool(np.any(diff > np.float32(theta)))


def evaluate(fr, key, slot, it, prm, colour_pairs="kstar"):
    """Which check iteration `it` of slot `slot` fails first (0 = none):
    1 colour, 2 distance, 3 rigidity, 4 degenerate Kabsch fit.
    colour_pairs: which pairs check 1 reads ("kstar" as defined, or a wrong
    reading: "first" = always pair 0, "all" = every pair)."""
    n = len(fr.eligible)
    kc, rp, rm = draws(key, slot, it)
    pix = [int(fr.eligible[_u(rp[k], n)]) for k in range(3)]
    rows = [fr.mlist[pix[k]][_u(rm[k], len(fr.mlist[pix[k]]))] for k in range(3)]
    pairs = {"kstar": [kc], "first": [0], "all": [0, 1, 2]}[colour_pairs]
    if any(colour_fails(fr, pix[k], rows[k], prm["max_colour_linf"]) for k in pairs):
        return 1
    xw = np.array([r[:3] for r in rows], np.float64)
    xc = np.array([fr.camera_point(p) for p in pix])
    pairs_ab = [(0, 1), (0, 2), (1, 2)]
    dw2 = [float(np.sum((xw[a] - xw[b]) ** 2)) for a, b in pairs_ab]
    if min(dw2) < prm["min_squared_distance_between_sampled_modes"]:
        return 2
    dc = [float(np.linalg.norm(xc[a] - xc[b])) for a, b in pairs_ab]
    if max(abs(c - np.sqrt(w2)) for c, w2 in zip(dc, dw2)) > prm["max_translation_error_for_correct_pose"]:
        return 3
    A = (xc - xc.mean(0)).T @ (xw - xw.mean(0))
    s = np.linalg.svd(A, compute_uv=False)
    if not s[0] > 0 or s[1] < 1e-4 * s[0]:
        return 4
    return 0


def first_pass(fr, key, slot, prm, colour_pairs="kstar", limit=None):
    lim = prm["max_candidate_generation_iterations"] if limit is None else limit
    for it in range(lim):
        if evaluate(fr, key, slot, it, prm, colour_pairs) == 0:
            return it
    return -1


def check_slots(fr, key, prm, out, slots):
    """Every iteration before the accepted one fails, the accepted one
    passes; an invalid slot fails every iteration.  Returns the per-check
    rejection counts."""
    counts = np.zeros(5, np.int64)
    for s in slots:
        acc = int(out["hyp_iter"][s]) if out["hyp_valid"][s] else -1
        upto = acc if acc >= 0 else prm["max_candidate_generation_iterations"]
        for it in range(upto):
            c = evaluate(fr, key, s, it, prm)
            assert c != 0, f"slot {s}: iteration {it} passes every check but {acc} was accepted"
            counts[c] += 1
        if acc >= 0:
            assert evaluate(fr, key, s, acc, prm) == 0, f"slot {s}: accepted iteration {acc} fails a check"
            counts[0] += 1
    return counts


def _key(prm, request_seed=0):
    k = (int(prm["seed"]) + int(request_seed) * 0x9E3779B97F4A7C15) & (2 ** 64 - 1)
    return [k & 0xFFFFFFFF, k >> 32]


@pytest.fixture(scope="module")
def ideal():
    sc = ideal_scene.build(seed=5, M=4)
    out = oracle.estimate_pose(sc["depth"], sc["rgb"], sc["K"], sc["leaves"], sc["nmodes"],
                               sc["modes"], sc["T"], sc["D"], sc["M"], sc["params"], 0)
    fr = Frame(sc["depth"], sc["rgb"], sc["K"], sc["leaves"], sc["nmodes"], sc["modes"], sc["T"],
               sc["D"], sc["M"], out["eligible"])
    return sc, out, fr


def test_every_iteration_before_the_accepted_one_fails_a_check(ideal):
    sc, out, fr = ideal
    prm = sc["params"]
    counts = check_slots(fr, _key(prm), prm, out, range(prm["max_pose_candidates"]))
    assert counts[0] == 64                         # every slot of the ideal scene is valid
    assert counts[1:].sum() > 1000                 # thousands of rejected iterations re-evaluated
    assert counts[1] > 0 and counts[2] > 0         # colour and distance rejections both occur


@pytest.fixture(scope="module")
def mixed_colours():
    """The ideal scene with two geometrically correct modes per pixel, one of
    them with the complementary colour: a triplet of correct points then
    passes the distance and rigidity checks whatever its colours, so which
    pair the colour check reads decides the outcome."""
    sc = ideal_scene.build(seed=7, M=4, n_correct=2)
    M = sc["M"]
    modes = sc["modes"].reshape(-1, M, 16)
    rgb = sc["rgb"].reshape(-1, 3)
    for p, xw in sc["truth"].items():
        correct = [m for m in range(M) if np.array_equal(modes[p, m, :3], np.float32(xw))]
        assert len(correct) == 2
        modes[p, correct[1], 10:13] = 255.0 - rgb[p].astype(np.float32)
    out = oracle.estimate_pose(sc["depth"], sc["rgb"], sc["K"], sc["leaves"], sc["nmodes"],
                               sc["modes"], sc["T"], sc["D"], sc["M"], sc["params"], 0)
    fr = Frame(sc["depth"], sc["rgb"], sc["K"], sc["leaves"], sc["nmodes"], sc["modes"], sc["T"],
               sc["D"], sc["M"], out["eligible"])
    return sc, out, fr


def test_rejection_side_with_mixed_colours(mixed_colours):
    sc, out, fr = mixed_colours
    prm = sc["params"]
    counts = check_slots(fr, _key(prm), prm, out, range(prm["max_pose_candidates"]))
    assert counts[0] == 64 and counts[1] > 0


def test_colour_check_reads_the_drawn_pair(mixed_colours):
    """The first passing iteration under a wrong reading of check 1 (always
    pair 0, or every pair) differs from the oracle's for some slots, so the
    rejection-side test tells the readings apart."""
    sc, out, fr = mixed_colours
    prm = sc["params"]
    key = _key(prm)
    for wrong in ("first", "all"):
        differs = 0
        for s in range(32):
            alt = first_pass(fr, key, s, prm, colour_pairs=wrong, limit=int(out["hyp_iter"][s]) + 1)
            differs += int(alt != int(out["hyp_iter"][s]))
        assert differs > 0, wrong


def test_c1_frame_rejection_side():
    """32 slots of a 160x120 query of the adapted 160x120 room."""
    from rlsynth import workloads
    w = workloads.c1(room_id=0, n_queries=1)
    o = oracle.Oracle(w.params, w.nodes)
    for f in w.adapt:
        o.adapt(f.depth, f.rgb, f.K, f.pose)
    q = w.queries[0]
    out = o.relocalise(q.depth, q.rgb, q.K, request_seed=0)
    fr = Frame(q.depth, q.rgb, q.K, out["leaves"], o.nmodes, o.modes, o.T, o.D, o.M, out["eligible"])
    counts = check_slots(fr, _key(w.params), w.params, out, range(32))
    assert counts[0] >= 16                          # most of these slots find a hypothesis
    assert counts[1] > 0 and counts[2] + counts[3] > 0


# ---------------------------------------------------------------------------
# exact boundaries of the distance and rigidity checks on a constructed frame

def _three_pixel_frame():
    """An 8x8 frame with depth 1 at pixels (0,0), (4,0), (0,3) and none
    elsewhere; intrinsics fx = fy = 1, cx = cy = 0, so the camera points are
    (0,0,1), (4,0,1), (0,3,1) with pairwise distances 4, 3, 5 exactly.  Each
    pixel has its own leaf with one mode whose colour equals the pixel's; the
    world points (0,0,0), (6,0,0), (0,4.5,0) have pairwise distances 6, 4.5,
    7.5 (squared 36, 20.25, 56.25), so the rigidity differences are 2, 1.5,
    2.5, all exact in binary."""
    w = h = 8
    depth = np.zeros((h, w), np.float32)
    rgb = np.zeros((h, w, 3), np.uint8)
    pix = [0 * w + 0, 0 * w + 4, 3 * w + 0]
    world = [(0.0, 0.0, 0.0), (6.0, 0.0, 0.0), (0.0, 4.5, 0.0)]
    T, D, M = 1, 2, 1
    leaves = np.full((w * h, T), 0xFFFF, np.uint16)
    nmodes = np.zeros(T << D, np.uint8)
    modes = np.zeros(((T << D) * M, 16), np.float32)
    for k, p in enumerate(pix):
        depth.reshape(-1)[p] = 1.0
        rgb.reshape(-1, 3)[p] = (40 * (k + 1), 100, 200)
        leaves[p, 0] = k
        nmodes[k] = 1
        modes[k, 0:3] = world[k]
        modes[k, 3] = 1.0
        modes[k, 4] = modes[k, 7] = modes[k, 9] = 1.0
        modes[k, 10:13] = rgb.reshape(-1, 3)[p]
    K = (np.float32(1), np.float32(1), np.float32(0), np.float32(0))
    return depth, rgb, K, leaves, nmodes, modes.reshape(-1), T, D, M


def _params(min_sq, rigid):
    return dict(max_pose_candidates=32, max_candidate_generation_iterations=200, max_colour_linf=30.0,
                min_squared_distance_between_sampled_modes=min_sq,
                max_translation_error_for_correct_pose=rigid, seed=11, ransac_inliers_per_iteration=8,
                max_relocalisations_to_output=1, max_pose_candidates_after_cull=32,
                use_prediction_covariance=0, final_refine=0, inlier_threshold=0.05)


def _run(min_sq, rigid):
    depth, rgb, K, leaves, nmodes, modes, T, D, M = _three_pixel_frame()
    return oracle.estimate_pose(depth, rgb, K, leaves, nmodes, modes, T, D, M, _params(min_sq, rigid), 0)


def test_distance_check_is_strict_at_its_boundary():
    """Reject iff the smallest squared world distance is below the minimum:
    a triplet at exactly the minimum (20.25 m^2) passes, one ulp above it
    every triplet fails."""
    at = _run(20.25, 2.5)
    assert at["hyp_valid"].sum() == 32
    # every accepted triplet uses the three distinct pixels
    assert all(sorted(r) == [0, 4, 24] for r in at["hyp_pix"])
    above = _run(float(np.nextafter(20.25, np.inf)), 2.5)
    assert above["hyp_valid"].sum() == 0


def test_rigidity_check_is_strict_at_its_boundary():
    """Reject iff a camera/world distance difference exceeds the tolerance:
    the largest difference is exactly 2.5 m, so a tolerance of 2.5 accepts
    and one ulp below it rejects every triplet."""
    at = _run(0.09, 2.5)
    assert at["hyp_valid"].sum() == 32
    below = _run(0.09, float(np.nextafter(2.5, 0.0)))
    assert below["hyp_valid"].sum() == 0


def test_constructed_frame_accepts_the_first_distinct_triplet():
    """With the boundaries inclusive every iteration drawing three distinct
    pixels passes, and every iteration repeating a pixel fails the distance
    check, so each slot's hypothesis is its first distinct draw."""
    depth, rgb, K, leaves, nmodes, modes, T, D, M = _three_pixel_frame()
    prm = _params(0.09, 2.5)
    out = oracle.estimate_pose(depth, rgb, K, leaves, nmodes, modes, T, D, M, prm, 0)
    key = _key(prm)
    el = out["eligible"]
    assert list(el) == [0, 4, 24]
    for s in range(prm["max_pose_candidates"]):
        it = 0
        while True:
            _, rp, _ = draws(key, s, it)
            if len({_u(r, 3) for r in rp}) == 3:
                break
            it += 1
        assert int(out["hyp_iter"][s]) == it
