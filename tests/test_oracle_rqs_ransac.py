"""Oracle pins: mode finding (RQS, Sec. 3.2.2 step 3), the Eq. 5 energy, the
three hypothesis checks and preemptive RANSAC (Sec. 3.2.3) on constructed
inputs whose answers are known."""
import numpy as np
import pytest
import scipy.linalg

import oracle
from rlsynth import scene
from tests import ideal_scene


def blob(rng, centre, n, std, colour):
    pts = rng.normal(centre, std, size=(n, 3)).astype(np.float32)
    col = np.tile(np.asarray(colour, np.uint8), (n, 1))
    return pts, col


def entries(pts, col):
    e = np.zeros((len(pts), 4), np.float32)
    e[:, :3] = pts
    e[:, 3] = oracle.pack_colour(col)
    return e


def test_rqs_two_separated_blobs():
    rng = np.random.default_rng(0)
    a, ca = blob(rng, [1.0, 1.0, 1.0], 40, 0.01, (200, 10, 10))
    b, cb = blob(rng, [2.0, 1.0, 1.0], 25, 0.01, (10, 200, 10))
    perm = rng.permutation(65)
    pts = np.concatenate([a, b])[perm]
    col = np.concatenate([ca, cb])[perm]
    rows, det = oracle.rqs_leaf(entries(pts, col), 0.1, 0.05, 20, 10, 1e-6)
    assert rows.shape[0] == 2
    assert det[0, 12] == 40 and det[1, 12] == 25          # sorted by size
    for k, (p, c) in enumerate([(a, (200, 10, 10)), (b, (10, 200, 10))]):
        p64 = p.astype(np.float64)
        np.testing.assert_allclose(det[k, 0:3], p64.mean(0), rtol=0, atol=1e-12)
        cov = np.cov(p64.T, bias=True)
        got = np.array([[det[k, 3], det[k, 4], det[k, 5]], [det[k, 4], det[k, 6], det[k, 7]],
                        [det[k, 5], det[k, 7], det[k, 8]]])
        np.testing.assert_allclose(got, cov, rtol=1e-9, atol=1e-15)
        np.testing.assert_allclose(det[k, 9:12], c, atol=1e-12)
        # stored inverse of (Sigma + lambda I), rounded to float32
        inv = np.array([[rows[k, 4], rows[k, 5], rows[k, 6]], [rows[k, 5], rows[k, 7], rows[k, 8]],
                        [rows[k, 6], rows[k, 8], rows[k, 9]]], dtype=np.float64)
        np.testing.assert_allclose(inv @ (cov + 1e-6 * np.eye(3)), np.eye(3), atol=1e-5)
        np.testing.assert_allclose(rows[k, 0:3], p64.mean(0).astype(np.float32))


def test_rqs_size_filter_and_cap():
    rng = np.random.default_rng(1)
    parts = [blob(rng, [x, 0.5, 0.5], n, 0.01, (x * 40, 0, 0))
             for x, n in [(0.5, 30), (1.5, 50), (2.5, 15), (3.5, 40)]]
    pts = np.concatenate([p for p, _ in parts])
    col = np.concatenate([c for _, c in parts])
    rows, det = oracle.rqs_leaf(entries(pts, col), 0.1, 0.05, 20, 10, 1e-6)
    assert list(det[:, 12]) == [50, 40, 30]                # 15-point blob dropped
    rows, det = oracle.rqs_leaf(entries(pts, col), 0.1, 0.05, 20, 2, 1e-6)
    assert list(det[:, 12]) == [50, 40]                    # at most max_cluster_count
    rows, det = oracle.rqs_leaf(entries(pts, col), 0.1, 0.05, 60, 10, 1e-6)
    assert rows.shape[0] == 0


def test_rqs_equal_sizes_ordered_by_root_index_and_link_threshold():
    # points on a line: spacing 4 cm < tau links everything into one cluster,
    # spacing 6 cm > tau leaves every point its own root.
    line4 = np.array([[0.04 * k, 0, 0] for k in range(9)], np.float32)
    col = np.zeros((9, 3), np.uint8)
    rows, det = oracle.rqs_leaf(entries(line4, col), 0.1, 0.05, 1, 20, 1e-6)
    assert rows.shape[0] == 1 and det[0, 12] == 9
    line6 = line4 * 1.5
    rows, det = oracle.rqs_leaf(entries(line6, col), 0.1, 0.05, 1, 20, 1e-6)
    assert rows.shape[0] == 9 and np.all(det[:, 12] == 1)
    assert list(det[:, 13]) == list(range(9))             # ties: ascending root index
    np.testing.assert_allclose(det[:, 0], line6[:, 0], atol=1e-7)


def test_rqs_root_is_the_density_peak():
    rng = np.random.default_rng(3)
    pts = rng.normal([1, 1, 1], 0.01, size=(30, 3)).astype(np.float32)
    e = entries(pts, np.zeros((30, 3), np.uint8))
    rows, det = oracle.rqs_leaf(e, 0.1, 0.05, 1, 5, 1e-6)
    d2 = ((pts[:, None, :].astype(np.float64) - pts[None, :, :]) ** 2).sum(-1)
    rho = np.exp(-d2 / (2 * 0.1 ** 2)).sum(1)
    assert rows.shape[0] == 1 and int(det[0, 13]) == int(np.argmax(rho))


# ---------------------------------------------------------------------------
# energy (Eq. 5)

def test_pixel_energy_equals_the_matrix_square_root_form():
    rng = np.random.default_rng(4)
    sc = ideal_scene.build(seed=2, M=3)
    # random SPD inverse covariances on every mode
    modes = sc["modes"].reshape(-1, 16).copy()
    for r in range(modes.shape[0]):
        A = rng.normal(size=(3, 3))
        S = A @ A.T + 0.5 * np.eye(3)
        modes[r, 4:10] = [S[0, 0], S[0, 1], S[0, 2], S[1, 1], S[1, 2], S[2, 2]]
    pose = np.concatenate([sc["H"][:3, :3].reshape(-1), sc["H"][:3, 3]]).astype(np.float32)
    pose[9:] += np.float32([0.03, -0.02, 0.01])
    pix = np.flatnonzero(sc["depth"].reshape(-1) > 0)[::37]
    fx, fy, cx, cy = [float(v) for v in sc["K"]]
    R = pose[:9].reshape(3, 3).astype(np.float64)
    t = pose[9:].astype(np.float64)
    for p in pix:
        e = oracle.pixel_energy(sc["depth"], sc["K"], sc["leaves"], sc["nmodes"], modes, 1,
                                sc["D"], sc["M"], pose, p, 1)
        x, y = p % sc["w"], p // sc["w"]
        d = float(sc["depth"].reshape(-1)[p])
        hx = R @ np.array([d * (x - cx) / fx, d * (y - cy) / fy, d]) + t
        best = np.inf
        for m in range(sc["M"]):
            row = modes[p * sc["M"] + m].astype(np.float64)
            Sinv = np.array([[row[4], row[5], row[6]], [row[5], row[7], row[8]], [row[6], row[8], row[9]]])
            root = np.real(scipy.linalg.sqrtm(Sinv))          # Sigma^{-1/2}
            best = min(best, np.linalg.norm(root @ (hx - row[:3])))
        assert e >= 0 and abs(e - best) <= 1e-9 * max(1.0, best)
        e_euc = oracle.pixel_energy(sc["depth"], sc["K"], sc["leaves"], sc["nmodes"], modes, 1,
                                    sc["D"], sc["M"], pose, p, 0)
        best_e = min(np.linalg.norm(hx - modes[p * sc["M"] + m, :3].astype(np.float64))
                     for m in range(sc["M"]))
        assert abs(e_euc - best_e) <= 1e-12 * max(1.0, best_e)


# ---------------------------------------------------------------------------
# hypotheses + RANSAC on the ideal scene

@pytest.fixture(scope="module")
def ideal():
    sc = ideal_scene.build(seed=5, M=4)
    out = oracle.estimate_pose(sc["depth"], sc["rgb"], sc["K"], sc["leaves"], sc["nmodes"],
                               sc["modes"], sc["T"], sc["D"], sc["M"], sc["params"], 0)
    return sc, out


def test_ransac_recovers_the_true_pose(ideal):
    sc, out = ideal
    assert out["status"] == "ok"
    dt, dr = scene.pose_error(out["pose"], sc["H"])
    assert dt < 1e-4 and dr < 1e-3, (dt, dr)
    # the winner (pre-refit) also is the true pose, and its energy is ~0
    w = out["winner"]
    Hw = np.eye(4)
    Hw[:3, :3] = out["hyp_pose64"][w, :9].reshape(3, 3)
    Hw[:3, 3] = out["hyp_pose64"][w, 9:]
    assert scene.pose_error(Hw, sc["H"])[0] < 1e-4
    assert out["mean_energy"] < 0.05          # float32 storage of modes only
    assert out["refitted"] and out["n_inliers"] >= 0.9 * len(out["I"])


def test_true_pose_has_near_zero_energy_and_wrong_poses_do_not(ideal):
    sc, out = ideal
    pose = np.concatenate([sc["H"][:3, :3].reshape(-1), sc["H"][:3, 3]]).astype(np.float32)
    bad = pose.copy()
    bad[9] += 0.05
    e_true = [oracle.pixel_energy(sc["depth"], sc["K"], sc["leaves"], sc["nmodes"], sc["modes"], 1,
                                  sc["D"], sc["M"], pose, p) for p in out["eligible"][::20]]
    e_bad = [oracle.pixel_energy(sc["depth"], sc["K"], sc["leaves"], sc["nmodes"], sc["modes"], 1,
                                 sc["D"], sc["M"], bad, p) for p in out["eligible"][::20]]
    assert max(e_true) < 0.01 and min(e_bad) > 1.0


def test_accepted_hypotheses_satisfy_the_three_checks(ideal):
    sc, out = ideal
    p = sc["params"]
    M = sc["M"]
    modes = sc["modes"].reshape(-1, M, 16)
    fx, fy, cx, cy = [float(v) for v in sc["K"]]
    d = sc["depth"].reshape(-1)
    rgb = sc["rgb"].reshape(-1, 3)
    nvalid = 0
    for s in np.flatnonzero(out["hyp_valid"]):
        nvalid += 1
        pix, mi = out["hyp_pix"][s], out["hyp_mode"][s]
        xw = np.array([modes[pix[k], mi[k], :3] for k in range(3)], np.float64)
        xc = np.array([[d[q] * ((q % sc["w"]) - cx) / fx, d[q] * ((q // sc["w"]) - cy) / fy, d[q]]
                       for q in pix], np.float64)
        for a, b in [(0, 1), (0, 2), (1, 2)]:
            dw = np.linalg.norm(xw[a] - xw[b])
            dc = np.linalg.norm(xc[a] - xc[b])
            assert dw * dw >= p["min_squared_distance_between_sampled_modes"]
            assert abs(dc - dw) <= p["max_translation_error_for_correct_pose"]
        # the colour check passes on at least one pair (the drawn one)
        assert any(np.max(np.abs(rgb[pix[k]].astype(np.float32) - modes[pix[k], mi[k], 10:13])) <= 30
                   for k in range(3))
        # the stored pose is Kabsch on the triplet
        ok, R, t, _ = oracle.kabsch(xc, xw)
        assert ok
        np.testing.assert_allclose(out["hyp_pose64"][s, :9], R.reshape(-1), atol=1e-12)
    assert nvalid == 64


def test_hypothesis_draws_follow_the_documented_mapping(ideal):
    sc, out = ideal
    el = out["eligible"]
    n = len(el)
    seed = sc["params"]["seed"]
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for s in range(8):
        it = int(out["hyp_iter"][s])
        a = [int(v) for v in oracle.philox4x32([(2 << 28) | 0, s, it, 0], key)]
        b = [int(v) for v in oracle.philox4x32([(2 << 28) | 1, s, it, 0], key)]
        kc = (a[0] * 3) >> 32
        others = [k for k in range(3) if k != kc]
        rp = {kc: a[1], others[0]: b[0], others[1]: b[1]}
        rm = {kc: a[2], others[0]: b[2], others[1]: b[3]}
        pix = [int(el[(rp[k] * n) >> 32]) for k in range(3)]
        assert pix == list(out["hyp_pix"][s])
        modes_idx = [(rm[k] * sc["M"]) >> 32 for k in range(3)]
        assert modes_idx == list(out["hyp_mode"][s])


def test_round_structure_and_cumulative_energy(ideal):
    sc, out = ideal
    assert out["rounds"] == 6 and list(out["round_n"]) == [32, 16, 8, 4, 2, 1]
    prev = set(np.flatnonzero(out["hyp_valid"]).tolist())
    for r in range(out["rounds"]):
        slots, en = out["round_slots"][r], out["round_energy"][r]
        assert set(slots.tolist()) <= prev
        prev = set(slots.tolist())
        order = np.lexsort((slots, en))
        assert np.array_equal(order, np.arange(len(slots)))
    # energies accumulate over the cumulative pixel set: equal to a full re-evaluation
    w = out["winner"]
    full = sum(oracle.pixel_energy(sc["depth"], sc["K"], sc["leaves"], sc["nmodes"], sc["modes"], 1,
                                   sc["D"], sc["M"], out["hyp_pose"][w], p) for p in out["I"])
    assert abs(full - out["energy"]) <= 1e-9 * max(1.0, full)
    assert len(out["I"]) == 6 * 50


def test_initial_cull_and_output_count():
    sc = ideal_scene.build(seed=6, M=3)
    p = dict(sc["params"], max_pose_candidates_after_cull=16, max_relocalisations_to_output=4)
    out = oracle.estimate_pose(sc["depth"], sc["rgb"], sc["K"], sc["leaves"], sc["nmodes"],
                               sc["modes"], sc["T"], sc["D"], sc["M"], p, 3)
    assert list(out["round_n"]) == [16, 8, 4]
    assert len(out["out_slots"]) == 4
    assert np.all(np.diff(out["out_energy"]) >= 0)


def test_no_pose_when_nothing_is_eligible():
    sc = ideal_scene.build(seed=7, M=2)
    zero = np.zeros_like(sc["depth"])
    out = oracle.estimate_pose(zero, sc["rgb"], sc["K"], sc["leaves"], sc["nmodes"], sc["modes"],
                               sc["T"], sc["D"], sc["M"], sc["params"], 0)
    assert out["status"] == "no_pose" and out["energy"] == np.inf
    out = oracle.estimate_pose(sc["depth"], sc["rgb"], sc["K"], sc["leaves"],
                               np.zeros_like(sc["nmodes"]), sc["modes"], sc["T"], sc["D"], sc["M"],
                               sc["params"], 0)
    assert out["status"] == "no_pose" and len(out["eligible"]) == 0


def test_refit_over_noise_free_inliers_is_exact():
    sc = ideal_scene.build(seed=8, M=1)          # every mode correct
    p = dict(sc["params"])
    out = oracle.estimate_pose(sc["depth"], sc["rgb"], sc["K"], sc["leaves"], sc["nmodes"],
                               sc["modes"], sc["T"], sc["D"], sc["M"], p, 0)
    assert out["refitted"] and out["n_inliers"] == len(out["I"])
    dt, dr = scene.pose_error(out["pose"], sc["H"])
    assert dt < 2e-6 and dr < 1e-4


# ---------------------------------------------------------------------------
# model-based score (analytic scene) used by the cascade

def test_plane_score_is_zero_at_the_true_pose_and_grows_with_error():
    room = scene.make_room(4)
    H = scene.random_pose(room, np.random.default_rng(9))
    w, h = 80, 60
    K = scene.intrinsics(w, h)
    depth, _ = scene.render(room, H, w, h, seed=3, noise_sigma=0.0, dropout=0.0)
    S = oracle.surfaces_of(room)
    pose = np.concatenate([H[:3, :3].reshape(-1), H[:3, 3]]).astype(np.float32)
    shifted = pose.copy()
    shifted[9] += 0.05
    s = oracle.plane_scores(depth, K, np.stack([pose, shifted]), S)
    assert s[0] < 1e-5                       # float32 depth and pose only
    # a 5 cm shift moves every point at most 5 cm from the surface it lay on,
    # and points on surfaces not parallel to the shift strictly off it
    assert s[0] + 1e-3 < s[1] <= 0.05 + 1e-6


def test_plane_score_rectangle_distance_closed_form():
    # one quad in the z = 0 plane, half-extents (1, 1); a camera at the origin
    # looking down +z sees points at depth d; pose chosen so the points land
    # at known offsets from the quad
    S = np.zeros((1, 16), np.float32)
    S[0, 3:6] = [0, 0, 1]
    S[0, 6:9] = [1, 0, 0]
    S[0, 9:12] = [0, 1, 0]
    S[0, 12:14] = [1, 1]
    depth = np.zeros((1, 4), np.float32)
    depth[0, 1] = 2.0                          # pixel (1, 0): K maps it to x = d * (1 - 0) / 1
    K = (np.float32(1.0), np.float32(1.0), np.float32(0.0), np.float32(0.0))
    pose = np.array([1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, -2.0], np.float32)   # x^W = x^C - (0, 0, 2)
    # x^C = (2, 0, 2) -> y = (2, 0, 0): in plane, 1 beyond the edge in a -> distance 1
    assert abs(oracle.plane_scores(depth, K, pose[None], S)[0] - 1.0) < 1e-12
    pose2 = pose.copy()
    pose2[11] = -1.0                          # y = (2, 0, 1): sqrt(1 + 1)
    assert abs(oracle.plane_scores(depth, K, pose2[None], S)[0] - np.sqrt(2.0)) < 1e-12
    S[0, 12:14] = 0                           # infinite plane: only the normal offset counts
    assert abs(oracle.plane_scores(depth, K, pose2[None], S)[0] - 1.0) < 1e-12


# ---------------------------------------------------------------------------
# amortised mode update (Sec. 3.2.2): K leaves per frame, round robin

def _adapted_c1_oracle():
    from rlsynth import workloads
    w = workloads.c1(room_id=3, n_queries=1)
    o = oracle.Oracle(w.params, w.nodes)
    for f in w.adapt:
        o.adapt(f.depth, f.rgb, f.K, f.pose)
    return w, o


def test_round_robin_touches_exactly_its_range_and_wraps():
    w, o = _adapted_c1_oracle()
    ref = oracle.Oracle(w.params, w.nodes)
    ref.reservoir[:], ref.seen[:] = o.reservoir, o.seen
    ref.update_modes(all_leaves=True)            # the exact definition, pinned above
    TL = o.T * o.L
    assert int((ref.nmodes > 0).sum()) > 50
    o.rr_cursor = TL - 20                          # a range that wraps: last 20 leaves, first 30
    nxt = o.update_modes_round_robin(50)
    assert nxt == 30
    inside = np.zeros(TL, bool)
    inside[TL - 20:] = True
    inside[:30] = True
    np.testing.assert_array_equal(o.nmodes[inside], ref.nmodes[inside])
    assert not o.nmodes[~inside].any()             # nothing outside the range was written
    M = o.M
    for tl in np.flatnonzero(inside):
        n = int(ref.nmodes[tl])
        np.testing.assert_array_equal(o.modes[tl * M * 16:(tl * M + n) * 16], ref.modes[tl * M * 16:(tl * M + n) * 16])


def test_round_robin_over_the_whole_forest_equals_the_exact_update():
    w, o = _adapted_c1_oracle()
    ref = oracle.Oracle(w.params, w.nodes)
    ref.reservoir[:], ref.seen[:] = o.reservoir, o.seen
    ref.update_modes(all_leaves=True)
    TL = o.T * o.L
    steps = 0
    while steps * 48 < TL:
        o.update_modes_round_robin(48)
        steps += 1
    assert o.rr_cursor == (steps * 48) % TL
    np.testing.assert_array_equal(o.nmodes, ref.nmodes)
    np.testing.assert_array_equal(o.modes, ref.modes)
