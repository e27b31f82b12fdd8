"""rl_depth_scores_noalloc (the depth-raycast score of Sec. 3.2.4, Eq. 6-7,
with the library's fixed device work space) against rl_depth_scores (the same
score in a room's work space): identical outputs on two calls in a row, the
second on a smaller frame with fewer poses, and the same results whichever
entry point ran before; limits rejected before any work."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
rl = pytest.importorskip("paper_1810_12163_amd")

from rlsynth import scene, workloads  # noqa: E402

pytestmark = pytest.mark.gpu


def _poses(pose, n, seed):
    rng = np.random.default_rng(seed)
    R0, t0 = pose[:3, :3], pose[:3, 3]
    out = [np.concatenate([R0.reshape(-1), t0])]
    for _ in range(n - 1):
        ax = rng.normal(size=3)
        ax *= np.radians(3.0) * rng.uniform() / np.linalg.norm(ax)
        th = np.linalg.norm(ax)
        Kx = np.array([[0, -ax[2], ax[1]], [ax[2], 0, -ax[0]], [-ax[1], ax[0], 0]])
        dR = np.eye(3) + np.sin(th) / th * Kx + (1 - np.cos(th)) / th**2 * Kx @ Kx
        out.append(np.concatenate([(R0 @ dR).reshape(-1), t0 + rng.normal(size=3) * 0.03]))
    return np.asarray(out, np.float32)


def _same(a, b):
    for x, y in zip(a, b):
        np.testing.assert_array_equal(np.asarray(x), np.asarray(y))


@pytest.fixture(scope="module")
def setup():
    w = workloads.c1()
    room = rl.Room(w.params, w.nodes, 640, 480, device="cuda:0")
    sroom = scene.make_room(0)
    rng = np.random.default_rng(77)
    pose = scene.random_pose(sroom, rng)
    d, c = scene.render(sroom, pose, 640, 480, seed=78)
    yield room, scene.surface_records(sroom), pose, d, c
    room.close()


def test_noalloc_depth_scores_equal_the_room_path(setup):
    room, S, pose, d, c = setup
    K = scene.intrinsics(640, 480)
    P1 = _poses(pose, 24, 1)
    dd, cc = torch.from_numpy(d).cuda(), torch.from_numpy(c).cuda()
    print("[noalloc] call 1: 640x480, 24 poses", flush=True)
    big = rl.depth_scores_noalloc(dd, cc, K, S, P1, 0.5, 4.0)
    # second call, smaller: a ragged 324x244 crop (77 full tiles and a partial
    # one), 5 poses, no upper depth limit
    dc = np.ascontiguousarray(d[:244, :324])
    rc = np.ascontiguousarray(c[:244, :324])
    P2 = _poses(pose, 5, 2)
    dsm, csm = torch.from_numpy(dc).cuda(), torch.from_numpy(rc).cuda()
    print("[noalloc] call 2: 324x244, 5 poses", flush=True)
    small = rl.depth_scores_noalloc(dsm, csm, K, S, P2, 0.5, 0.0)
    torch.cuda.synchronize()
    print("[noalloc] room path on the same inputs", flush=True)
    _same(big, room.depth_scores(dd, cc, K, S, P1, 0.5, 4.0))
    _same(small, room.depth_scores(dsm, csm, K, S, P2, 0.5, 0.0))
    assert big[0].shape == (24,) and small[0].shape == (5,)
    assert np.all(np.isfinite(big[0])) and np.argmin(big[0]) == 0 and big[0][0] < 0.01
    assert np.all(big[2][:, 1] > 0) and np.all(small[2][:, 1] > 0)
    # the fixed work space keeps the last call's contents: a third call, the
    # large one again, still equals its first result
    _same(big, rl.depth_scores_noalloc(dd, cc, K, S, P1, 0.5, 4.0))


def test_noalloc_rejects_sizes_beyond_its_work_space(setup):
    room, S, pose, d, c = setup
    K = scene.intrinsics(640, 480)
    dd, cc = torch.from_numpy(d).cuda(), torch.from_numpy(c).cuda()
    P = _poses(pose, 2, 3)
    with pytest.raises(rl.RlError):
        rl.depth_scores_noalloc(dd, cc, K, S, np.zeros((65, 12), np.float32), 0.5, 4.0)
    with pytest.raises(rl.RlError):
        rl.depth_scores_noalloc(dd, cc, K, np.zeros((65, 16), np.float32), P, 0.5, 4.0)
    with pytest.raises(rl.RlError):
        rl.depth_scores_noalloc(dd, cc, K, S, P, -1.0, 4.0)
    # 2048 x 1028 = 2,105,344 pixels > 2^21: rejected on the host
    big_d = torch.zeros((1028, 2048), dtype=torch.float32, device="cuda")
    big_c = torch.zeros((1028, 2048, 3), dtype=torch.uint8, device="cuda")
    with pytest.raises(rl.RlError):
        rl.depth_scores_noalloc(big_d, big_c, K, S, P, 0.5, 4.0)
    # the largest accepted frame: 2048 x 1024 = 2^21 pixels, all depth invalid
    ok_d = big_d[:1024].contiguous()
    ok_c = big_c[:1024].contiguous()
    s, mu, cnt = rl.depth_scores_noalloc(ok_d, ok_c, K, S, P, 0.5, 4.0)
    assert np.all(np.isinf(s)) and np.all(np.isnan(mu)) and np.all(cnt[:, 1] == 0)
