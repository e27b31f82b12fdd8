"""Oracle pins for the model-based hypothesis score (Sec. 3.2.4, Eq. 6-8):
closed forms for planes seen from known poses, the exact 10% valid-fraction
rule on a rectangle whose pixel footprint is counted by brute force, and the
independent frame renderer of the synthetic scenes at the frame's own pose."""
import math

import numpy as np

import oracle
from rlsynth import scene

W, H = 64, 48
K = scene.intrinsics(W, H)


def pose12(R, t):
    return np.concatenate([np.asarray(R, np.float64).reshape(-1), np.asarray(t, np.float64)])


def surf(p0, n, e1=(0, 0, 0), e2=(0, 0, 0), half=(0.0, 0.0)):
    s = np.zeros(16, np.float32)
    s[0:3], s[3:6], s[6:9], s[9:12], s[12:14] = p0, n, e1, e2, half
    return s[None, :]


def rot_y(a):
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]])


def pixel_rays():
    x, y = np.meshgrid(np.arange(W, dtype=np.float64), np.arange(H, dtype=np.float64))
    fx, fy, cx, cy = [float(v) for v in K]
    return np.stack([(x - cx) / fx, (y - cy) / fy, np.ones_like(x)], -1)      # (H, W, 3)


def test_fronto_parallel_plane_closed_form():
    # camera at the origin looking along +z; plane z = 2; live depth 2.25 on the
    # left half, 0 (invalid) on the right half
    S = surf((0, 0, 2), (0, 0, -1))
    d = np.full((H, W), 2.25, np.float32)
    d[:, W // 2:] = 0
    s, mu, cnt = oracle.depth_scores(d, K, pose12(np.eye(3), (0, 0, 0))[None], S, 0.5, 4.0)
    assert cnt[0, 0] == W * H and cnt[0, 1] == W * H // 2
    assert mu[0] == 0.25 and s[0] == 0.25


def test_rotated_camera_tilted_plane_closed_form():
    # plane n . x = c seen from a camera at t rotated about y: along the world
    # ray R d^C from t the hit depth is (c - n . t) / (n . R d^C) = (c - n . t) / ((R^T n) . d^C)
    a = math.radians(25.0)
    R = rot_y(a)
    t = np.array([0.3, -0.2, 0.1])
    n = np.array([math.sin(0.4), 0.0, math.cos(0.4)])
    c = 2.5
    p0 = n * c
    S = surf(p0, n)
    Dt = (c - n @ t) / (pixel_rays() @ (R.T @ n))
    assert np.all(Dt > 0.5) and np.all(Dt < 4.0)
    live = (Dt + 0.01 * np.sin(np.arange(W * H)).reshape(H, W)).astype(np.float32)
    s, mu, cnt = oracle.depth_scores(live, K, pose12(R, t)[None].astype(np.float32), S, 0.5, 4.0)
    # the pose is rounded to float32 for the call: the closed form uses the same rounding
    Rf = pose12(R, t).astype(np.float32).astype(np.float64)
    R32, t32 = Rf[:9].reshape(3, 3), Rf[9:]
    n32 = np.asarray(S[0, 3:6], np.float64)
    c32 = n32 @ np.asarray(S[0, 0:3], np.float64)
    Dt32 = (c32 - n32 @ t32) / (pixel_rays() @ (R32.T @ n32))
    want = np.mean(np.abs(live.astype(np.float64) - Dt32))
    assert cnt[0, 0] == W * H and cnt[0, 1] == W * H
    assert abs(mu[0] - want) <= 1e-12 * want and s[0] == mu[0]
    # a transposed rotation would score the same frame differently
    s_t, _, _ = oracle.depth_scores(live, K, pose12(R.T, t)[None], S, 0.5, 4.0)
    assert abs(s_t[0] - s[0]) > 1e-3


def quad_footprint(Z, a, b):
    fx, fy, cx, cy = [float(v) for v in K]
    n = 0
    for y in range(H):
        for x in range(W):
            n += abs((x - cx) / fx * Z) <= a and abs((y - cy) / fy * Z) <= b
    return n


def test_rectangle_footprint_and_the_valid_fraction_rule():
    # a rectangle at depth 2 facing the camera, centred on the optical axis:
    # pixel (x, y) hits it iff |(x - cx) Z / fx| <= a and |(y - cy) Z / fy| <= b
    Z = 2.0
    d = np.full((H, W), 2.0, np.float32)
    seen = {}
    for a in np.linspace(0.05, 0.8, 31):
        b = 0.75 * a
        S = surf((0, 0, Z), (0, 0, -1), (1, 0, 0), (0, 1, 0), (a, b))
        s, mu, cnt = oracle.depth_scores(d, K, pose12(np.eye(3), (0, 0, 0))[None], S, 0.5, 4.0)
        n = quad_footprint(Z, a, b)
        assert cnt[0, 0] == n and cnt[0, 1] == n
        finite = 10 * n >= W * H
        assert np.isfinite(s[0]) == finite
        if finite:
            assert s[0] == 0.0
        seen[finite] = True
    assert seen == {True: True, False: True}          # both sides of the 10% rule were exercised


def test_no_valid_pixels_and_depth_range():
    S = surf((0, 0, 2), (0, 0, -1))
    I = pose12(np.eye(3), (0, 0, 0))[None]
    # no valid live depth: +inf, mu undefined
    s, mu, cnt = oracle.depth_scores(np.zeros((H, W), np.float32), K, I, S, 0.5, 4.0)
    assert s[0] == math.inf and math.isnan(mu[0]) and cnt[0, 0] == W * H and cnt[0, 1] == 0
    # camera turned away from the plane: nothing is hit
    s, _, cnt = oracle.depth_scores(np.ones((H, W), np.float32), K, pose12(rot_y(math.pi), (0, 0, 0))[None],
                                    S, 0.5, 4.0)
    assert s[0] == math.inf and cnt[0, 0] == 0
    # the plane beyond max_depth is invalid; with no upper limit it is valid
    S5 = surf((0, 0, 5), (0, 0, -1))
    _, _, cnt = oracle.depth_scores(np.ones((H, W), np.float32), K, I, S5, 0.5, 4.0)
    assert cnt[0, 0] == 0
    _, _, cnt = oracle.depth_scores(np.ones((H, W), np.float32), K, I, S5, 0.5, 0.0)
    assert cnt[0, 0] == W * H


def test_rendered_frame_scores_zero_at_its_pose_and_worse_when_moved():
    room = scene.make_room(3)
    rng = np.random.default_rng(5)
    Hc = scene.random_pose(room, rng)
    d, _ = scene.render(room, Hc, W, H, seed=1, noise_sigma=0.0, dropout=0.0, K=K)
    S = oracle.surfaces_of(room)
    R0, t0 = Hc[:3, :3], Hc[:3, 3]
    poses = [pose12(R0, t0)]
    for sgn in (1.0, -1.0):
        poses.append(pose12(R0, t0 + sgn * 0.02 * R0[:, 2]))          # 2 cm along the optical axis
        for ax in (0, 1):                                               # 2 degrees about camera x, y
            k = np.zeros(3)
            k[ax] = sgn * math.radians(2.0)
            Kx = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
            a = np.linalg.norm(k)
            dR = np.eye(3) + math.sin(a) / a * Kx + (1 - math.cos(a)) / a**2 * Kx @ Kx
            poses.append(pose12(R0 @ dR, t0))
    s, mu, cnt = oracle.depth_scores(d, K, np.asarray(poses, np.float32), S, scene.DEPTH_MIN, scene.DEPTH_MAX)
    n_live = int(np.count_nonzero(d > 0))
    assert cnt[0, 1] == n_live and cnt[0, 0] >= n_live
    assert s[0] < 1e-5                                # float32 rounding of the rendered depth and pose
    assert np.all(s[1:] > 20 * s[0]) and int(np.argmin(s)) == 0
