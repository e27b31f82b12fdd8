"""HIP path vs the oracle at the full size of the 640x480 workload: five
depth-15 trees, reservoirs of 1024 entries, 50 adaptation frames (every
4th-grid pixel), 1024 hypotheses, eta 500, ten halving rounds and the final
inlier refit.  Everything the oracle can afford is compared in full:
arrival counters and every filled reservoir entry (bit-exact), leaves of every
pixel, the eligible list, every hypothesis, every round; modes on sampled
leaves (the fullest reservoirs plus a random sample)."""
import numpy as np
import pytest

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
import paper_1810_12163_amd as rl  # noqa: E402
from rlsynth import scene, workloads  # noqa: E402
from tests.gpu_util import compare_modes, dev, pose_diff, reservoir_mismatches  # noqa: E402


@pytest.fixture(scope="module")
def c2():
    print("\n[c2 fixture] rendering 50 adaptation frames + 2 queries", flush=True)
    w = workloads.c2(n_adapt=50, n_queries=2)
    o = oracle.Oracle(w.params, w.nodes)
    room = rl.Room(w.params, w.nodes, 640, 480)
    for f in w.adapt:
        o.adapt(f.depth, f.rgb, f.K, f.pose)
        d, c = dev(f)
        room.adapt(d, c, f.K, f.pose)
    torch.cuda.synchronize()
    print("[c2 fixture] adapted", flush=True)
    return w, o, room


def test_c2_reservoirs_bit_exact(c2):
    w, o, room = c2
    seen = room.buffer_np(rl.BUF_SEEN, np.uint32).copy()
    np.testing.assert_array_equal(seen, o.seen)
    assert int(seen.sum()) > 4_000_000
    res = room.buffer_np(rl.BUF_RESERVOIR, np.float32).reshape(o.T * o.L, o.kappa, 4)
    bad, total = reservoir_mismatches(seen, res, o.reservoir, o.kappa)
    assert bad == 0, (bad, total)
    assert total > 2_000_000
    del res


def test_c2_modes_sampled_leaves(c2):
    w, o, room = c2
    room.update_modes()
    nm_g = room.buffer_np(rl.BUF_NMODES, np.uint8).copy()
    modes_g = room.buffer_np(rl.BUF_MODES, np.float32).reshape(o.T * o.L, o.M, 16)
    seen = o.seen
    order = np.argsort(-seen.astype(np.int64), kind="stable")
    rng = np.random.default_rng(0)
    nonempty = np.flatnonzero(seen > 0)
    sample = np.unique(np.concatenate([order[:300], rng.choice(nonempty, 1500, replace=False)]))
    p = w.params
    nm_o = np.zeros_like(nm_g)
    modes_o = np.zeros((o.T * o.L, o.M, 16), np.float32)
    for tl in sample:
        t, leaf = divmod(int(tl), o.L)
        rows, _ = oracle.rqs_leaf(o.reservoir_of(t, leaf), p["clusterer_sigma"], p["clusterer_tau"],
                                  p["min_cluster_size"], o.M, p["cov_regulariser"])
        nm_o[tl] = rows.shape[0]
        modes_o[tl, :rows.shape[0]] = rows
    assert int(nm_o[sample].sum()) > 500
    bad, worst = compare_modes(nm_g, modes_g, nm_o, modes_o.reshape(-1), o.M, sample)
    assert bad == 0 and worst < 1e-5, (bad, worst)


def test_c2_relocalise_full_stage_parity(c2):
    w, o, room = c2
    q = w.queries[0]
    room.set_trace(True)
    d, c = dev(q)
    seed = 3
    res = room.relocalise(d, c, q.K, request_seed=seed)
    P = q.depth.size
    leaves_g = room.buffer_np(rl.BUF_LEAVES, np.uint16).reshape(-1, 8)[:P, :o.T].copy()
    np.testing.assert_array_equal(leaves_g, o.traverse(q.depth, q.rgb))
    nm_g = room.buffer_np(rl.BUF_NMODES, np.uint8).copy()
    modes_g = room.buffer_np(rl.BUF_MODES, np.float32).copy()
    ref = oracle.estimate_pose(q.depth, q.rgb, q.K, leaves_g, nm_g, modes_g, o.T, o.D, o.M, w.params, seed)
    n_el = res["n_eligible"]
    assert n_el == len(ref["eligible"]) > 100_000
    np.testing.assert_array_equal(room.buffer_np(rl.BUF_ELIGIBLE, np.int32)[:n_el], ref["eligible"])
    N = w.params["max_pose_candidates"]
    hy = room.buffer_np(rl.BUF_HYPS, rl.HYP_DTYPE)[:N]
    v = ref["hyp_valid"].astype(bool)
    np.testing.assert_array_equal(hy["valid"].astype(bool), v)
    assert v.sum() >= 8
    np.testing.assert_array_equal(hy["iter"][v], ref["hyp_iter"][v])
    np.testing.assert_array_equal(hy["pix"][v], ref["hyp_pix"][v])
    np.testing.assert_array_equal(hy["mode"][v], ref["hyp_mode"][v])
    np.testing.assert_allclose(hy["R"][v], ref["hyp_pose"][v][:, :9], atol=1e-5)
    np.testing.assert_allclose(hy["t"][v], ref["hyp_pose"][v][:, 9:], atol=1e-5)
    assert res["rounds"] == ref["rounds"]
    eta = w.params["ransac_inliers_per_iteration"]
    np.testing.assert_array_equal(room.buffer_np(rl.BUF_ILIST, np.int32)[:ref["rounds"] * eta], ref["I"])
    ts = room.buffer_np(rl.BUF_TRACE_SLOTS, np.int32).reshape(-1, N)
    te = room.buffer_np(rl.BUF_TRACE_ENERGY, np.float64).reshape(-1, N)
    for r in range(ref["rounds"]):
        k = len(ref["round_slots"][r])
        np.testing.assert_array_equal(ts[r, :k], ref["round_slots"][r])
        np.testing.assert_allclose(te[r, :k], ref["round_energy"][r], rtol=1e-4)
    assert res["status"] == "ok" and res["winner"] == ref["winner"]
    assert res["refitted"] == ref["refitted"] and res["n_inliers"] == ref["n_inliers"]
    assert pose_diff(res["pose"], ref["pose"]) < 1e-5
    assert abs(res["energy"] - ref["energy"]) <= 1e-4 * abs(ref["energy"])
    dt, dr = scene.pose_error(res["pose"].astype(np.float64), q.pose)
    print(f"[c2] pose error vs ground truth: {dt * 100:.2f} cm, {dr:.2f} deg; "
          f"valid hypotheses {int(v.sum())}", flush=True)
    room.set_trace(False)


# ---------------------------------------------------------------------------
# cascade pieces: per-call RANSAC settings, decimated stage, model score

@pytest.fixture(scope="module")
def c3_room(c2):
    w, o, room = c2
    from rlsynth import presets
    p3 = presets.preset("c3c")            # room sized for 4096 hypotheses, 16 outputs
    r3 = rl.Room(p3, w.nodes, 640, 480)
    for f in w.adapt:
        d, c = dev(f)
        r3.adapt(d, c, f.K, f.pose)
    r3.update_modes()
    return p3, r3


def _stage_ref(room, q, params, seed, T, D, M, nodes, ref_width):
    leaves = oracle.traverse(q.depth, q.rgb, None, nodes, T, D, ref_width)
    nm = room.buffer_np(rl.BUF_NMODES, np.uint8).copy()
    modes = room.buffer_np(rl.BUF_MODES, np.float32).copy()
    return oracle.estimate_pose(q.depth, q.rgb, q.K, leaves, nm, modes, T, D, M, params, seed)


def test_c3_decimated_stage_matches_oracle(c2, c3_room):
    w, o, _ = c2
    p3, r3 = c3_room
    q = workloads.decimate(w.queries[1])
    d, c = dev(q)
    res = r3.relocalise(d, c, q.K, request_seed=21, n_hypotheses=256, n_cull=256, n_out=1, final_refine=1)
    params = dict(p3, max_pose_candidates=256, max_pose_candidates_after_cull=256,
                  max_relocalisations_to_output=1, final_refine=1)
    ref = _stage_ref(r3, q, params, 21, o.T, o.D, o.M, w.nodes, p3["ref_width"])
    print(f"[c3 stage a] valid {res['n_valid']}, rounds {res['rounds']} (oracle {ref['rounds']})", flush=True)
    assert res["n_valid"] == int(ref["hyp_valid"].sum()) > 0
    assert res["rounds"] == ref["rounds"] >= 1 and res["winner"] == ref["winner"]
    assert pose_diff(res["pose"], ref["pose"]) < 1e-5
    assert abs(res["energy"] - ref["energy"]) <= 1e-4 * abs(ref["energy"])


def test_lm_640x480_matches_oracle(c2, c3_room):
    """LM refinement at 640x480 (1024 hypothesis slots, cull to 64, halving
    to one) in every round after the first, over up to (rounds x 500) pixels:
    survivors of every round, the survivors' refined poses (1e-5), energies
    (1e-4 relative) and the winner."""
    w, o, _ = c2
    p3, r3 = c3_room
    q = w.queries[0]
    d, c = dev(q)
    r3.set_trace(True)
    res = r3.relocalise(d, c, q.K, request_seed=41, n_hypotheses=1024, n_cull=64, n_out=1, final_refine=0,
                        pose_update=1)
    params = dict(p3, max_pose_candidates=1024, max_pose_candidates_after_cull=64,
                  max_relocalisations_to_output=1, final_refine=0, pose_update=1)
    ref = _stage_ref(r3, q, params, 41, o.T, o.D, o.M, w.nodes, p3["ref_width"])
    print(f"[lm 640x480] valid {res['n_valid']}, rounds {res['rounds']} (oracle {ref['rounds']}), "
          f"winner {res['winner']} (oracle {ref['winner']})", flush=True)
    assert res["n_valid"] == int(ref["hyp_valid"].sum())
    assert res["rounds"] == ref["rounds"] >= 2
    N = 1024                                 # trace rows are strided by the call's hypothesis count
    ts = r3.buffer_np(rl.BUF_TRACE_SLOTS, np.int32).reshape(-1, N)
    te = r3.buffer_np(rl.BUF_TRACE_ENERGY, np.float64).reshape(-1, N)
    P64 = r3.buffer_np(rl.BUF_POSE64, np.float64).reshape(-1, 12)
    for r in range(ref["rounds"]):
        k = len(ref["round_slots"][r])
        np.testing.assert_array_equal(ts[r, :k], ref["round_slots"][r])
        np.testing.assert_allclose(te[r, :k], ref["round_energy"][r], rtol=1e-4)
    outs = ref["round_slots"][-1]
    dp = float(np.abs(P64[outs] - ref["refined_pose64"][outs]).max())
    print(f"[lm 640x480] refined pose diff {dp:.2e}", flush=True)
    assert dp < 1e-5
    assert res["winner"] == ref["winner"] and pose_diff(res["pose"], ref["pose"]) < 1e-5
    r3.set_trace(False)


def test_c3_wide_stage_keeps_16_and_model_score_matches(c2, c3_room):
    w, o, _ = c2
    p3, r3 = c3_room
    q = w.queries[1]
    d, c = dev(q)
    r3.set_trace(True)
    res = r3.relocalise(d, c, q.K, request_seed=22, n_hypotheses=4096, n_cull=4096, n_out=16, final_refine=0)
    ref = _stage_ref(r3, q, dict(p3, final_refine=0), 22, o.T, o.D, o.M, w.nodes, p3["ref_width"])
    print(f"[c3 stage c] valid {res['n_valid']}, rounds {res['rounds']} (oracle {ref['rounds']}), "
          f"kept {res['n_out']}", flush=True)
    assert res["n_valid"] == int(ref["hyp_valid"].sum()) > 0
    assert res["rounds"] == ref["rounds"] and res["n_out"] == len(ref["out_slots"]) >= min(2, res["n_valid"])
    # every round, including those entered by more than 64 survivors (one
    # scoring launch and one selection per round) and the rounds scored at once
    N = 4096
    ts = r3.buffer_np(rl.BUF_TRACE_SLOTS, np.int32).reshape(-1, N)
    te = r3.buffer_np(rl.BUF_TRACE_ENERGY, np.float64).reshape(-1, N)
    entering = [int(ref["hyp_valid"].sum())] + [len(s) for s in ref["round_slots"][:-1]]
    assert entering[0] > 64, entering          # the per-round path runs
    for r in range(ref["rounds"]):
        k = len(ref["round_slots"][r])
        np.testing.assert_array_equal(ts[r, :k], ref["round_slots"][r])
        np.testing.assert_allclose(te[r, :k], ref["round_energy"][r], rtol=1e-4)
    r3.set_trace(False)
    print(f"[c3 stage c] survivors entering each round {entering}", flush=True)
    slots, poses = r3.survivors(res["n_out"])
    np.testing.assert_array_equal(slots, ref["out_slots"])
    S = oracle.surfaces_of(w.room)
    got = r3.plane_scores(d, c, q.K, S, poses)
    want = oracle.plane_scores(q.depth, q.K, poses, S)
    np.testing.assert_allclose(got, want, rtol=1e-9, atol=1e-12)
    gt = np.concatenate([q.pose[:3, :3].reshape(-1), q.pose[:3, 3]]).astype(np.float32)
    s_gt = r3.plane_scores(d, c, q.K, S, gt[None])[0]
    assert s_gt < 0.005                     # noisy depth: a few mm at the true pose


def _same_depth_scores(got, want):
    (s, mu, cnt), (s_o, mu_o, cnt_o) = got, want
    np.testing.assert_array_equal(cnt, cnt_o)
    np.testing.assert_array_equal(np.isinf(s), np.isinf(s_o))
    np.testing.assert_array_equal(np.isnan(mu), np.isnan(mu_o))
    f = np.isfinite(s_o)
    np.testing.assert_allclose(s[f], s_o[f], rtol=1e-12, atol=0)
    m = ~np.isnan(mu_o)
    np.testing.assert_allclose(mu[m], mu_o[m], rtol=1e-12, atol=0)


def test_depth_scores_match_oracle(c2):
    """Eq. 6-7 depth-raycast scores at 640x480 for the true pose, 2 cm / 2 degree
    perturbations, poses below the floor looking away from the room (one with
    too few valid raycast pixels: +inf) and a ragged 324x244 crop: both counts bit-exact,
    s and mu to 1e-12 relative; an all-invalid live frame gives +inf / NaN."""
    w, o, room = c2
    S = oracle.surfaces_of(w.room)
    q = w.queries[1]
    R0, t0 = q.pose[:3, :3], q.pose[:3, 3]
    poses = [np.concatenate([R0.reshape(-1), t0])]
    rng = np.random.default_rng(4)
    for k in range(13):
        ax = rng.normal(size=3)
        ax *= np.radians(2.0) * rng.uniform() / np.linalg.norm(ax)
        th = np.linalg.norm(ax)
        Kx = np.array([[0, -ax[2], ax[1]], [ax[2], 0, -ax[0]], [-ax[1], ax[0], 0]])
        dR = np.eye(3) + np.sin(th) / th * Kx + (1 - np.cos(th)) / th**2 * Kx @ Kx
        poses.append(np.concatenate([(R0 @ dR).reshape(-1), t0 + rng.normal(size=3) * 0.02]))
    # below the floor looking down, away from the room: the wall planes leave
    # 32% of the raycast valid from (1, 1.5, -0.5) and 8.6% (+inf) from (2, 2, -1)
    down = np.array([[0, 1, 0], [1, 0, 0], [0, 0, -1]], np.float64)
    for t in ([1.0, 1.5, -0.5], [2.0, 2.0, -1.0]):
        poses.append(np.concatenate([down.reshape(-1), t]))
    P = np.asarray(poses, np.float32)
    d, c = dev(q)
    got = room.depth_scores(d, c, q.K, S, P, 0.5, 4.0)
    want = oracle.depth_scores(q.depth, q.K, P, S, 0.5, 4.0)
    print(f"[depth scores] s {np.round(want[0], 4)}", flush=True)
    _same_depth_scores(got, want)
    assert int(np.argmin(got[0])) == 0 and got[0][0] < 0.01
    assert np.isinf(got[0][-1])
    # ragged crop (79056 pixels: 77 full tiles and a partial one), no upper depth limit
    dc = q.depth[:244, :324].copy()
    cc = q.rgb[:244, :324].copy()
    Kc = q.K
    got = room.depth_scores(torch.from_numpy(dc).cuda(), torch.from_numpy(cc).cuda(), Kc, S, P, 0.5, 0.0)
    _same_depth_scores(got, oracle.depth_scores(dc, Kc, P, S, 0.5, 0.0))
    # no valid live depth
    z = np.zeros_like(dc)
    got = room.depth_scores(torch.from_numpy(z).cuda(), torch.from_numpy(cc).cuda(), Kc, S, P[:3], 0.5, 4.0)
    assert np.all(np.isinf(got[0])) and np.all(np.isnan(got[1])) and np.all(got[2][:, 1] == 0)
    with pytest.raises(rl.RlError):
        room.depth_scores(d, c, q.K, S, P, -1.0, 4.0)


def test_paper_stage_settings_match_oracle(c2, c3_room):
    """Each relocaliser of the paper's cascade (Table 8's RANSAC settings:
    2048 hypotheses, cull to 64, eta 256, per-stage iterations, thresholds,
    covariance and LM), run on the shared forest through per-call settings,
    equals the oracle run with the same settings."""
    from paper_1810_12163_amd.cascade import paper_stages
    w, o, _ = c2
    p3, r3 = c3_room
    q = w.queries[1]
    d, c = dev(q)
    for i, st in enumerate(paper_stages()):
        cs = st.call_settings()
        res = r3.relocalise(d, c, q.K, request_seed=60 + i, **cs)
        params = dict(p3, max_pose_candidates=cs["n_hypotheses"], max_pose_candidates_after_cull=cs["n_cull"],
                      max_relocalisations_to_output=cs["n_out"], pose_update=cs["pose_update"],
                      max_candidate_generation_iterations=cs["max_iterations"],
                      ransac_inliers_per_iteration=cs["eta"],
                      min_squared_distance_between_sampled_modes=float(np.float32(cs["min_squared_distance"])),
                      max_translation_error_for_correct_pose=float(np.float32(cs["max_translation_error"])))
        if cs["use_covariance"] >= 0:
            params["use_prediction_covariance"] = cs["use_covariance"]
        ref = _stage_ref(r3, q, params, 60 + i, o.T, o.D, o.M, w.nodes, p3["ref_width"])
        print(f"[paper stage {st.name}] valid {res['n_valid']} (oracle {int(ref['hyp_valid'].sum())}), "
              f"rounds {res['rounds']}, winner {res['winner']} (oracle {ref['winner']})", flush=True)
        assert res["n_valid"] == int(ref["hyp_valid"].sum()) > 0
        assert res["rounds"] == ref["rounds"] and res["winner"] == ref["winner"]
        assert pose_diff(res["pose"], ref["pose"]) < 1e-5
        assert abs(res["energy"] - ref["energy"]) <= 1e-4 * abs(ref["energy"])


def test_cascade_fallback_and_ranking(c2, c3_room):
    from paper_1810_12163_amd.cascade import Cascade, Stage
    w, o, _ = c2
    p3, r3 = c3_room
    S = oracle.surfaces_of(w.room)
    q = w.queries[0]
    d, c = dev(q)
    stages = [Stage("a", 256, decimate=True), Stage("b", 1024, final_refine=1), Stage("c", 4096, n_out=16)]
    accept = Cascade(r3, [dataclasses_replace(s, threshold=float("inf")) for s in stages], S)
    out = accept.relocalise(d, c, q.K, request_seed=3)
    assert out["stage"] == "a" and len(out["trail"]) == 1
    full = Cascade(r3, [dataclasses_replace(s, threshold=0.0) for s in stages], S)
    out = full.relocalise(d, c, q.K, request_seed=3)
    assert [t[0] for t in out["trail"]] == ["a", "b", "c"] and out["stage"] == "c"
    assert out["model_score"] == float(np.min(out["ranked"]))
    # stage c ranked its survivors by the Eq. 6-7 depth score, as the oracle scores them
    slots, poses = r3.survivors(len(out["ranked"]))
    np.testing.assert_allclose(out["ranked"], oracle.depth_scores(q.depth, q.K, poses, S, 0.5, 4.0)[0],
                               rtol=1e-12, atol=0)
    # the paper's fallback thresholds: 5 cm after stage a, 7.5 cm after stage b
    th = [0.05, 0.075, float("inf")]
    paper = Cascade(r3, [dataclasses_replace(s, threshold=t) for s, t in zip(stages, th)], S)
    out = paper.relocalise(d, c, q.K, request_seed=3)
    print(f"[cascade 5cm/7.5cm] trail {out['trail']}", flush=True)
    for (name, sc), t in zip(out["trail"][:-1], th):
        assert sc > t
    assert out["trail"][-1][1] <= th[len(out["trail"]) - 1] or out["stage"] == "c"


def test_mixed_batch_equals_plain(c2, c3_room):
    """Batches mixing two rooms (different cull / output / refit settings),
    three resolutions (640x480, 320x240, 160x120) and hypothesis counts
    (1024, 512, 256) give exactly the plain path's result for every request,
    with direct launches and graph replay, in any order."""
    w, o, room = c2
    p3, r3 = c3_room
    q0, q1 = w.queries[0], w.queries[1]
    dec = workloads.decimate
    plan = [(room, q0, 1), (r3, q1, 2), (room, dec(q1), 3), (r3, dec(q0), 4),
            (room, dec(dec(q0)), 5), (r3, dec(dec(q1)), 6), (room, q1, 7)]
    reqs = []
    for rm, q, s in plan:
        d, c = dev(q)
        reqs.append((rm, d, c, q.K, s, workloads.HYPOTHESES[q.depth.shape[1]]))
    plain = [rm.relocalise(d, c, K, request_seed=s, n_hypotheses=N) for (rm, d, c, K, s, N) in reqs]
    print(f"[mixed batch] plain statuses {[r['status'] for r in plain]}, rounds {[r['rounds'] for r in plain]}",
          flush=True)
    batch = rl.Batch(8, 640, 480, 1024, 500, 12, 5, 50)

    def same(got, want):
        for a, b in zip(got, want):
            assert a["status"] == b["status"] and a["winner"] == b["winner"]
            assert a["rounds"] == b["rounds"] and a["n_out"] == b["n_out"] and a["n_valid"] == b["n_valid"]
            assert np.array_equal(a["pose"], b["pose"]) and a["energy"] == b["energy"]

    for use_graph in (False, True, True):
        same(batch.relocalise(reqs, use_graph=use_graph), plain)
    same(batch.relocalise(reqs[::-1], use_graph=True), plain[::-1])
    batch.close()


def test_every_schedule_gives_identical_results(c2, c3_room):
    """Every launch schedule (search iterations per thread 2/4/8, all-rounds
    scoring width 1/2/4 waves, 6 or 8 tree levels of the traversal read from
    LDS, the all-rounds scoring in one pass or in a first window of 1-3 rounds
    and the rest) gives bit-identical results, batched (graph replay and
    direct launches) and plain; a request of 256 hypotheses enters the
    all-rounds scoring at its first round under the 4-wave width (its window
    then includes the initial cull), the 1024-hypothesis requests after
    per-round scoring.  The tuner then leaves one of them set."""
    from paper_1810_12163_amd import autotune
    w, o, room = c2
    p3, r3 = c3_room
    q0, q1 = w.queries[0], w.queries[1]
    dec = workloads.decimate
    plan = [(room, q0, 11), (r3, dec(q1), 12), (room, dec(dec(q0)), 13), (r3, q1, 14)]
    reqs = []
    for rm, q, s in plan:
        d, c = dev(q)
        reqs.append((rm, d, c, q.K, s, workloads.HYPOTHESES[q.depth.shape[1]]))
    want = [rm.relocalise(d, c, K, request_seed=s, n_hypotheses=N) for (rm, d, c, K, s, N) in reqs]

    def same(got, ref, tag):
        for a, b in zip(got, ref):
            assert a["status"] == b["status"] and a["winner"] == b["winner"], tag
            assert a["rounds"] == b["rounds"] and a["n_out"] == b["n_out"] and a["n_valid"] == b["n_valid"], tag
            assert np.array_equal(a["pose"], b["pose"]) and a["energy"] == b["energy"], tag

    batch = rl.Batch(4, 640, 480, 1024, 500, 12, 5, 50)
    for sc in autotune.candidates():
        print(f"[schedule] batch ipt={sc[0]} fast_waves={sc[1]} lds_levels={sc[2]} window={sc[3]}", flush=True)
        batch.set_schedule(*sc)
        same(batch.relocalise(reqs, use_graph=True), want, sc)
        same(batch.relocalise(reqs, use_graph=sc[:2] == (8, 4)), want, sc)
    for sc in ((2, 4, 6, 2), (8, 2, 8, 0), (4, 4, 6, 1), (4, 1, 8, 3)):
        print(f"[schedule] plain ipt={sc[0]} fast_waves={sc[1]} lds_levels={sc[2]} window={sc[3]}", flush=True)
        for rm in (room, r3):
            rm.set_schedule(*sc)
        same([rm.relocalise(d, c, K, request_seed=s, n_hypotheses=N) for (rm, d, c, K, s, N) in reqs], want, sc)
    for rm in (room, r3):
        rm.set_schedule(*autotune.DEFAULT)
    best, timings = autotune.tune_batch(batch, reqs, reps=2, warmup=1)
    assert best in timings and batch.schedule == best
    same(batch.relocalise(reqs, use_graph=True), want, best)
    with pytest.raises(rl.RlError):
        batch.set_schedule(3, 1)
    with pytest.raises(rl.RlError):
        room.set_schedule(4, 8)
    with pytest.raises(rl.RlError):
        room.set_schedule(4, 1, 7)
    with pytest.raises(rl.RlError):
        batch.set_schedule(4, 1, 8, 4)
    batch.close()


def dataclasses_replace(s, **kw):
    import dataclasses
    return dataclasses.replace(s, **kw)


def test_c2_colour_check_bits_equal_the_float_test(c2):
    """Every eligible pixel's record holds |M(u)| and, for every mode of M(u),
    the outcome of the colour check as the oracle evaluates it (L-infinity in
    float32 against the mode's mean colour), for the full 640x480 frame."""
    w, o, room = c2
    q = w.queries[1]
    d, c = dev(q)
    res = room.relocalise(d, c, q.K, request_seed=9)
    n_el = res["n_eligible"]
    P = q.depth.size
    el = room.buffer_np(rl.BUF_ELIGIBLE, np.int32)[:n_el].copy()
    rec = room.buffer_np(rl.BUF_EREC, np.uint64)[:n_el].copy()        # one word per entry (|M(u)| <= 56)
    leaves = room.buffer_np(rl.BUF_LEAVES, np.uint16).reshape(-1, 8)[:P, :o.T].astype(np.int64)
    nmodes = room.buffer_np(rl.BUF_NMODES, np.uint8).reshape(o.T, o.L)
    modes = room.buffer_np(rl.BUF_MODES, np.float32).reshape(o.T, o.L, o.M, 16)
    theta = np.float32(w.params["max_colour_linf"])
    lv = leaves[el]                                               # (n, T)
    cnt = nmodes[np.arange(o.T)[None, :], lv].astype(np.int64)    # (n, T)
    total = cnt.sum(1)
    np.testing.assert_array_equal((rec & np.uint64(0xFF)).astype(np.int64), total)
    px = q.rgb.reshape(-1, 3)[el].astype(np.float32)              # (n, 3)
    checked = 0
    m0 = np.zeros(n_el, np.int64)
    for t in range(o.T):
        for j in range(o.M):
            has = j < cnt[:, t]
            col = modes[t, lv[:, t], j, 10:13]                        # (n, 3) float32
            ok = ~np.any(np.abs(px - col) > theta, axis=1)
            m = m0 + j
            bit = ((rec >> (np.uint64(8) + m.astype(np.uint64))) & np.uint64(1)).astype(bool)
            sel = has & (m < 56)
            np.testing.assert_array_equal(bit[sel], ok[sel])
            checked += int(sel.sum())
        m0 = m0 + cnt[:, t]
    print(f"[colour bits] {n_el} entries, {checked} (pixel, mode) checks", flush=True)
    assert checked > 1_000_000


# ---------------------------------------------------------------------------
# Table 8's Forest row of the Fast / Intermediate / Slow relocalisers
# (reservoirs of 2048, up to 50 modes per leaf, link distance 0.2 m, clusters
# of at least 5 points): five trees give up to 250 modes per pixel, so every
# eligible-list record spans several 64-bit words and the tree-major walks of
# M(u) cross many tree boundaries.

@pytest.fixture(scope="module")
def forest_row(c2):
    from rlsynth import presets
    w, _, _ = c2
    p = presets.preset("fast")
    print("\n[forest row] adapting a kappa 2048 / M 50 room from the 50 frames", flush=True)
    o = oracle.Oracle(p, w.nodes)
    room = rl.Room(p, w.nodes, 640, 480)
    for f in w.adapt:
        o.adapt(f.depth, f.rgb, f.K, f.pose)
        d, c = dev(f)
        room.adapt(d, c, f.K, f.pose)
    room.update_modes()
    torch.cuda.synchronize()
    yield p, o, room
    room.close()


def test_forest_row_reservoirs_and_modes(forest_row):
    p, o, room = forest_row
    seen = room.buffer_np(rl.BUF_SEEN, np.uint32).copy()
    np.testing.assert_array_equal(seen, o.seen)
    res = room.buffer_np(rl.BUF_RESERVOIR, np.float32).reshape(o.T * o.L, o.kappa, 4)
    bad, total = reservoir_mismatches(seen, res, o.reservoir, o.kappa)
    assert bad == 0 and total > 2_000_000, (bad, total)
    del res
    nm_g = room.buffer_np(rl.BUF_NMODES, np.uint8).copy()
    modes_g = room.buffer_np(rl.BUF_MODES, np.float32).reshape(o.T * o.L, o.M, 16)
    order = np.argsort(-seen.astype(np.int64), kind="stable")
    rng = np.random.default_rng(1)
    sample = np.unique(np.concatenate([order[:60], rng.choice(np.flatnonzero(seen > 0), 400, replace=False)]))
    nm_o = np.zeros_like(nm_g)
    modes_o = np.zeros((o.T * o.L, o.M, 16), np.float32)
    for tl in sample:
        t, leaf = divmod(int(tl), o.L)
        rows, _ = oracle.rqs_leaf(o.reservoir_of(t, leaf), p["clusterer_sigma"], p["clusterer_tau"],
                                  p["min_cluster_size"], o.M, p["cov_regulariser"])
        nm_o[tl] = rows.shape[0]
        modes_o[tl, :rows.shape[0]] = rows
    assert int(nm_o[sample].max()) == o.M                 # full leaves reach the 50-mode cap
    bad, worst = compare_modes(nm_g, modes_g, nm_o, modes_o.reshape(-1), o.M, sample)
    assert bad == 0 and worst < 1e-5, (bad, worst)


def _colour_bits_equal_float_test(room, q, o, theta, el, rec):
    """Every colour-check bit of every eligible entry (all record words)
    against the float32 L-infinity test; returns (#checks, |M(u)| per entry)."""
    P = q.depth.size
    leaves = room.buffer_np(rl.BUF_LEAVES, np.uint16).reshape(-1, 8)[:P, :o.T].astype(np.int64)
    nmodes = room.buffer_np(rl.BUF_NMODES, np.uint8).reshape(o.T, o.L)
    modes = room.buffer_np(rl.BUF_MODES, np.float32).reshape(o.T, o.L, o.M, 16)
    lv = leaves[el]
    cnt = nmodes[np.arange(o.T)[None, :], lv].astype(np.int64)
    total = cnt.sum(1)
    np.testing.assert_array_equal((rec[:, 0] & np.uint64(0xFF)).astype(np.int64), total)
    px = q.rgb.reshape(-1, 3)[el].astype(np.float32)
    rows = np.arange(len(el))
    checked = 0
    m0 = np.zeros(len(el), np.int64)
    for t in range(o.T):
        for j in range(o.M):
            has = j < cnt[:, t]
            if not has.any():
                continue
            col = modes[t, lv[:, t], j, 10:13]
            ok = ~np.any(np.abs(px - col) > np.float32(theta), axis=1)
            m = m0 + j
            word = np.where(m < 56, 0, 1 + (m - 56) // 64)
            shift = np.where(m < 56, 8 + m, (m - 56) % 64).astype(np.uint64)
            bit = ((rec[rows, word] >> shift) & np.uint64(1)).astype(bool)
            np.testing.assert_array_equal(bit[has], ok[has], err_msg=f"tree {t} mode {j}")
            checked += int(has.sum())
        m0 = m0 + cnt[:, t]
    return checked, total


@pytest.mark.parametrize("stage", ["fast", "intermediate"])
def test_forest_row_multiword_records_and_rounds(c2, forest_row, stage):
    """640x480 frame on the Forest-row room with Table 8's RANSAC settings of
    the Fast (no LM) and Intermediate (LM, Euclidean) relocalisers, except 6000
    generation iterations (with about 200 modes per pixel, 500-1000 iterations
    leave only a handful of the 2048 slots valid): leaves, eligible list,
    every word of every eligible record, every hypothesis, every round's
    survivors and energies, the LM-refined poses and the result equal the
    oracle's."""
    from rlsynth import presets
    w, _, _ = c2
    p, o, room = forest_row
    sp = presets.preset(stage)
    q = w.queries[0]
    d, c = dev(q)
    seed = 31 if stage == "fast" else 32
    kw = dict(n_hypotheses=sp["max_pose_candidates"], n_cull=sp["max_pose_candidates_after_cull"],
              n_out=sp["max_relocalisations_to_output"], final_refine=0, pose_update=sp["pose_update"],
              max_iterations=6000, eta=sp["ransac_inliers_per_iteration"],
              use_covariance=sp["use_prediction_covariance"],
              min_squared_distance=sp["min_squared_distance_between_sampled_modes"],
              max_translation_error=sp["max_translation_error_for_correct_pose"])
    room.set_trace(True)
    res = room.relocalise(d, c, q.K, request_seed=seed, **kw)
    P = q.depth.size
    leaves_g = room.buffer_np(rl.BUF_LEAVES, np.uint16).reshape(-1, 8)[:P, :o.T].copy()
    np.testing.assert_array_equal(leaves_g, o.traverse(q.depth, q.rgb))
    nm_g = room.buffer_np(rl.BUF_NMODES, np.uint8).copy()
    modes_g = room.buffer_np(rl.BUF_MODES, np.float32).copy()
    params = dict(p, max_pose_candidates=kw["n_hypotheses"], max_pose_candidates_after_cull=kw["n_cull"],
                  max_relocalisations_to_output=kw["n_out"], final_refine=0, pose_update=kw["pose_update"],
                  max_candidate_generation_iterations=kw["max_iterations"], ransac_inliers_per_iteration=kw["eta"],
                  use_prediction_covariance=kw["use_covariance"],
                  min_squared_distance_between_sampled_modes=float(np.float32(kw["min_squared_distance"])),
                  max_translation_error_for_correct_pose=float(np.float32(kw["max_translation_error"])))
    ref = oracle.estimate_pose(q.depth, q.rgb, q.K, leaves_g, nm_g, modes_g, o.T, o.D, o.M, params, seed)
    n_el = res["n_eligible"]
    assert n_el == len(ref["eligible"]) > 100_000
    el = room.buffer_np(rl.BUF_ELIGIBLE, np.int32)[:n_el].copy()
    np.testing.assert_array_equal(el, ref["eligible"])
    ew = 1 + (o.T * o.M - 56 + 63) // 64
    rec = room.buffer_np(rl.BUF_EREC, np.uint64).reshape(-1, ew)[:n_el].copy()
    checked, total = _colour_bits_equal_float_test(room, q, o, p["max_colour_linf"], el, rec)
    print(f"[forest row {stage}] {n_el} entries, |M(u)| max {total.max()}, > 56 on {(total > 56).sum()}, "
          f"> 184 on {(total > 184).sum()}; {checked} colour bits", flush=True)
    assert (total > 56).sum() > 10_000 and (total > 184).sum() > 1000   # second and fourth words in use
    N = kw["n_hypotheses"]
    hy = room.buffer_np(rl.BUF_HYPS, rl.HYP_DTYPE)[:N]
    v = ref["hyp_valid"].astype(bool)
    np.testing.assert_array_equal(hy["valid"].astype(bool), v)
    assert v.sum() >= 8
    np.testing.assert_array_equal(hy["iter"][v], ref["hyp_iter"][v])
    np.testing.assert_array_equal(hy["pix"][v], ref["hyp_pix"][v])
    np.testing.assert_array_equal(hy["mode"][v], ref["hyp_mode"][v])
    assert int(hy["mode"][v].max()) >= 56                 # triplet modes beyond the first record word
    # with LM the survivors of the first round hold their refined poses
    # (compared below); the others keep the Kabsch pose
    kab = v.copy()
    if kw["pose_update"]:
        kab[ref["round_slots"][0]] = False
    np.testing.assert_allclose(hy["R"][kab], ref["hyp_pose"][kab][:, :9], atol=1e-5)
    np.testing.assert_allclose(hy["t"][kab], ref["hyp_pose"][kab][:, 9:], atol=1e-5)
    assert res["rounds"] == ref["rounds"] >= 2
    eta = kw["eta"]
    np.testing.assert_array_equal(room.buffer_np(rl.BUF_ILIST, np.int32)[:ref["rounds"] * eta], ref["I"])
    ts = room.buffer_np(rl.BUF_TRACE_SLOTS, np.int32).reshape(-1, N)
    te = room.buffer_np(rl.BUF_TRACE_ENERGY, np.float64).reshape(-1, N)
    for r in range(ref["rounds"]):
        k = len(ref["round_slots"][r])
        np.testing.assert_array_equal(ts[r, :k], ref["round_slots"][r])
        np.testing.assert_allclose(te[r, :k], ref["round_energy"][r], rtol=1e-4)
    if kw["pose_update"]:
        P64 = room.buffer_np(rl.BUF_POSE64, np.float64).reshape(-1, 12)
        outs = ref["round_slots"][-1]
        assert float(np.abs(P64[outs] - ref["refined_pose64"][outs]).max()) < 1e-5
    assert res["status"] == ref["status"] == "ok" and res["winner"] == ref["winner"]
    assert pose_diff(res["pose"], ref["pose"]) < 1e-5
    assert abs(res["energy"] - ref["energy"]) <= 1e-4 * abs(ref["energy"])
    dt, dr = scene.pose_error(res["pose"].astype(np.float64), q.pose)
    print(f"[forest row {stage}] valid {int(v.sum())}, rounds {res['rounds']}, error {dt * 100:.2f} cm "
          f"{dr:.2f} deg", flush=True)
    room.set_trace(False)


def test_round_robin_split_rows_equal_one_workgroup_per_leaf(c2):
    """A round-robin mode step of at most 256 leaves computes its densities
    and links in row chunks of 256 points spread over workgroups; a longer
    step keeps one workgroup per leaf for them.  On rooms whose first tree has
    256 leaves (depth 8) and full reservoirs of 1024 points, a 256-leaf step
    (split) and a 300-leaf step (not split) over the same reservoirs give the
    same mode counts and rows, bit for bit, on the 256 leaves both cover."""
    from rlsynth import forest, presets
    w, _, _ = c2
    p = dict(w.params, depth=8, n_trees=2)
    nodes = forest.make_forest(77, **dict(presets.FOREST["c1"], n_trees=2))
    rooms = []
    for K in (256, 300):
        print(f"[rr split] leaves per frame {K}", flush=True)
        room = rl.Room(p, nodes, 640, 480)
        for f in w.adapt[:12]:
            d, c = dev(f)
            room.adapt(d, c, f.K, f.pose)
        room.set_mode_schedule(K)
        f = w.adapt[12]
        d, c = dev(f)
        room.adapt(d, c, f.K, f.pose)
        rooms.append(room)
    torch.cuda.synchronize()
    A, B = rooms
    M = p["max_cluster_count"]
    seen = A.buffer_np(rl.BUF_SEEN, np.uint32)[:256].copy()
    assert seen.max() >= p["reservoir_capacity"] and (seen > 256).sum() >= 8, seen.max()
    nA = A.buffer_np(rl.BUF_NMODES, np.uint8)[:256].astype(np.int64)
    nB = B.buffer_np(rl.BUF_NMODES, np.uint8)[:256].astype(np.int64)
    assert np.array_equal(nA, nB) and nA.sum() > 0
    mA = A.buffer_np(rl.BUF_MODES, np.uint32).reshape(-1, M, 16)[:256]
    mB = B.buffer_np(rl.BUF_MODES, np.uint32).reshape(-1, M, 16)[:256]
    used = np.arange(M)[None, :] < nA[:, None]
    assert np.array_equal(mA[used], mB[used])
    for room in rooms:
        room.close()
