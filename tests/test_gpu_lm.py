"""HIP path vs the oracle with the Levenberg-Marquardt refinement on
(Sec. 3.2.3, step (ii)): the small config (160x120, one depth-8 tree,
64 hypotheses, eta 100, halving to one) with LM in every round after the
first, Mahalanobis and Euclidean.

Bar: pixel lists and per-round survivor sets equal; energies to 1e-4
relative; refined poses of the final survivors and the result pose to 1e-5."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
import paper_1810_12163_amd as rl  # noqa: E402
from rlsynth import scene, workloads  # noqa: E402
from tests.gpu_util import dev, gpu_state, pose_diff  # noqa: E402


@pytest.fixture(scope="module")
def lm_rooms():
    print("\n[lm fixture] c1 workload, rooms with LM (Mahalanobis, Euclidean) and without", flush=True)
    w = workloads.c1(n_queries=3)
    rooms = {}
    for name, over in (("cov", dict(pose_update=1, lm_iterations=10)),
                       ("l2", dict(pose_update=1, lm_iterations=10, use_prediction_covariance=0)),
                       ("off", dict(pose_update=0)),
                       ("zero", dict(pose_update=1, lm_iterations=0))):
        p = dict(w.params, **over)
        room = rl.Room(p, w.nodes, 160, 120)
        for f in w.adapt:
            d, c = dev(f)
            room.adapt(d, c, f.K, f.pose)
        room.update_modes()
        rooms[name] = (p, room)
    torch.cuda.synchronize()
    return w, rooms


def _ref(w, p, room, q, seed):
    leaves = room.buffer_np(rl.BUF_LEAVES, np.uint16).reshape(-1, 8)[:q.depth.size, :p["n_trees"]].copy()
    _, _, nm, modes = gpu_state(room, p["n_trees"], 1 << p["depth"], p["reservoir_capacity"],
                                p["max_cluster_count"])
    return oracle.estimate_pose(q.depth, q.rgb, q.K, leaves, nm, modes.reshape(-1), p["n_trees"], p["depth"],
                                p["max_cluster_count"], p, seed)


@pytest.mark.parametrize("kind", ["cov", "l2"])
@pytest.mark.parametrize("qi", [0, 1, 2])
def test_lm_stage_parity(lm_rooms, kind, qi):
    w, rooms = lm_rooms
    p, room = rooms[kind]
    q = w.queries[qi]
    seed = 31 + qi
    room.set_trace(True)
    d, c = dev(q)
    res = room.relocalise(d, c, q.K, request_seed=seed)
    ref = _ref(w, p, room, q, seed)
    print(f"[lm {kind} q{qi}] status {res['status']} rounds {res['rounds']} (oracle {ref['rounds']})", flush=True)
    assert res["status"] == ref["status"]
    if ref["status"] != "ok":
        room.set_trace(False)
        return
    N = p["max_pose_candidates"]
    eta = p["ransac_inliers_per_iteration"]
    assert res["rounds"] == ref["rounds"] >= 3
    np.testing.assert_array_equal(room.buffer_np(rl.BUF_ILIST, np.int32)[:ref["rounds"] * eta], ref["I"])
    ts = room.buffer_np(rl.BUF_TRACE_SLOTS, np.int32).reshape(-1, N)
    te = room.buffer_np(rl.BUF_TRACE_ENERGY, np.float64).reshape(-1, N)
    worst = 0.0
    for r in range(ref["rounds"]):
        k = len(ref["round_slots"][r])
        np.testing.assert_array_equal(ts[r, :k], ref["round_slots"][r])
        rel = np.abs(te[r, :k] - ref["round_energy"][r]) / np.abs(ref["round_energy"][r])
        worst = max(worst, float(rel.max()))
    assert worst <= 1e-4, worst
    # refined poses of the last round's survivors
    last = ref["round_slots"][-1]
    P64 = room.buffer_np(rl.BUF_POSE64, np.float64).reshape(-1, 12)
    dp = float(np.abs(P64[last] - ref["refined_pose64"][last]).max())
    print(f"[lm {kind} q{qi}] worst energy rel {worst:.2e}, refined pose diff {dp:.2e}", flush=True)
    assert dp < 1e-5
    assert res["winner"] == ref["winner"]
    assert pose_diff(res["pose"], ref["pose"]) < 1e-5
    assert abs(res["energy"] - ref["energy"]) <= 1e-4 * abs(ref["energy"])
    room.set_trace(False)


def test_zero_iterations_and_the_per_call_switch(lm_rooms):
    """LM with zero iterations re-scores the cumulative I at unchanged poses:
    the plain path's survivors in every round, energies to 1e-12, the same
    pose.  The per-call switch turns LM on for a room created without it and
    then gives exactly the result of a room created with it."""
    w, rooms = lm_rooms
    q = w.queries[0]
    d, c = dev(q)
    p, off = rooms["off"]
    _, zero = rooms["zero"]
    _, cov = rooms["cov"]
    N = p["max_pose_candidates"]
    runs = {}
    for name, room in (("off", off), ("zero", zero)):
        room.set_trace(True)
        res = room.relocalise(d, c, q.K, request_seed=7)
        runs[name] = (res, room.buffer_np(rl.BUF_TRACE_SLOTS, np.int32).reshape(-1, N).copy(),
                      room.buffer_np(rl.BUF_TRACE_ENERGY, np.float64).reshape(-1, N).copy())
        room.set_trace(False)
    (a, ta, ea), (b, tb, eb) = runs["off"], runs["zero"]
    assert a["status"] == b["status"] == "ok" and a["rounds"] == b["rounds"] >= 3
    n, first = a["n_valid"], True
    for r in range(a["rounds"]):           # survivors kept by each round
        cull = p["max_pose_candidates_after_cull"]
        n = cull if (first and cull < n) else ((n + 1) // 2 if n > p["max_relocalisations_to_output"] else n)
        first = False
        np.testing.assert_array_equal(ta[r, :n], tb[r, :n])
        np.testing.assert_allclose(eb[r, :n], ea[r, :n], rtol=1e-12, atol=0)
    assert a["winner"] == b["winner"] and np.array_equal(a["pose"], b["pose"])
    assert abs(a["energy"] - b["energy"]) <= 1e-12 * abs(a["energy"])
    on = off.relocalise(d, c, q.K, request_seed=7, pose_update=1)
    ref = cov.relocalise(d, c, q.K, request_seed=7)
    assert on["winner"] == ref["winner"] and np.array_equal(on["pose"], ref["pose"]) and on["energy"] == ref["energy"]


def test_lm_batch_equals_plain(lm_rooms):
    """A batch mixing LM rooms (10 iterations, and one with none) and a plain
    room gives exactly the plain path's result for every request, with graph
    replay and direct launches."""
    w, rooms = lm_rooms
    reqs = []
    for i, kind in enumerate(["cov", "off", "l2", "zero", "cov", "off"]):
        q = w.queries[i % 3]
        d, c = dev(q)
        reqs.append((rooms[kind][1], d, c, q.K, 50 + i))
    want = [rm.relocalise(d, c, K, request_seed=s) for (rm, d, c, K, s) in reqs]
    batch = rl.Batch(8, 160, 120, 64, 100, 8, 1, 5)
    for use_graph in (True, False, True):
        got = batch.relocalise(reqs, use_graph=use_graph)
        for a, b in zip(got, want):
            assert a["status"] == b["status"] and a["winner"] == b["winner"] and a["rounds"] == b["rounds"]
            assert np.array_equal(a["pose"], b["pose"]) and a["energy"] == b["energy"]
    batch.close()
    # 40 LM requests: the batch's passes take two pixel tiles per wave (lane
    # halves), the plain calls one; the partial sums, and so the results,
    # are the same
    many = [(rooms["cov" if i % 2 else "l2"][1], *dev(w.queries[i % 3]), w.queries[i % 3].K, 700 + i)
            for i in range(40)]
    want40 = [rm.relocalise(d, c, K, request_seed=s) for (rm, d, c, K, s) in many]
    big = rl.Batch(64, 160, 120, 64, 100, 8, 1, 5)
    got = big.relocalise(many, use_graph=True)
    for a, b in zip(got, want40):
        assert a["status"] == b["status"] and a["winner"] == b["winner"] and a["rounds"] == b["rounds"]
        assert np.array_equal(a["pose"], b["pose"]) and a["energy"] == b["energy"]
    big.close()
    errs = [scene.pose_error(r["pose"].astype(np.float64), w.queries[i % 3].pose)
            for i, r in enumerate(want) if r["status"] == "ok"]
    print(f"[lm batch] pose errors (m, deg) {[(round(a, 3), round(b, 2)) for a, b in errs]}", flush=True)
