"""HIP path vs the oracle on identical seeded inputs (small config: 160x120,
one depth-8 tree, kappa 64, 64 hypotheses, eta 100).

Bar: leaf indices, eligible pixels, reservoir contents and counters,
sampled triplets and accepted iterations bit-exact; mode counts exact and
mode rows to float32 rounding; hypothesis poses to 1e-5; energies to 1e-4
relative; the final pose to 1e-5 (and within 1 cm / 1 degree).  Stage parity
feeds the GPU's own upstream arrays to the oracle."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle  # noqa: E402
import paper_1810_12163_amd as rl  # noqa: E402
from rlsynth import scene, workloads  # noqa: E402
from tests.gpu_util import compare_modes, dev, gpu_state, pose_diff, reservoir_mismatches  # noqa: E402


@pytest.fixture(scope="module")
def c1():
    print("\n[c1 fixture] building workload, oracle and GPU room", flush=True)
    w = workloads.c1(n_queries=3)
    o = oracle.Oracle(w.params, w.nodes)
    room = rl.Room(w.params, w.nodes, 160, 120)
    for f in w.adapt:
        o.adapt(f.depth, f.rgb, f.K, f.pose)
        d, c = dev(f)
        room.adapt(d, c, f.K, f.pose)
    torch.cuda.synchronize()
    return w, o, room


def test_c1_reservoirs_bit_exact(c1):
    w, o, room = c1
    T, L, kappa, M = o.T, o.L, o.kappa, o.M
    seen, res, _, _ = gpu_state(room, T, L, kappa, M)
    np.testing.assert_array_equal(seen, o.seen)
    bad, total = reservoir_mismatches(seen, res, o.reservoir, kappa)
    assert total > 1000 and bad == 0, (bad, total)
    dirty = room.buffer_np(rl.BUF_DIRTY, np.uint32)
    np.testing.assert_array_equal(dirty != 0, o.dirty != 0)


def test_c1_modes(c1):
    w, o, room = c1
    room.update_modes()
    o.update_modes()
    _, _, nm_g, modes_g = gpu_state(room, o.T, o.L, o.kappa, o.M)
    assert int(o.nmodes.sum()) > 20
    bad, worst = compare_modes(nm_g, modes_g, o.nmodes, o.modes, o.M, range(o.T * o.L))
    assert bad == 0 and worst < 1e-5, (bad, worst)
    assert not np.any(room.buffer_np(rl.BUF_DIRTY, np.uint32))


@pytest.mark.parametrize("qi", [0, 1, 2])
def test_c1_relocalise_stage_parity(c1, qi):
    w, o, room = c1
    q = w.queries[qi]
    room.set_trace(True)
    d, c = dev(q)
    seed = 11 + qi
    res = room.relocalise(d, c, q.K, request_seed=seed)
    h, wd = q.depth.shape
    P = h * wd
    T = o.T
    # leaves: bit-exact against the oracle's own traversal
    leaves_g = room.buffer_np(rl.BUF_LEAVES, np.uint16).reshape(-1, 8)[:P, :T]
    leaves_o = o.traverse(q.depth, q.rgb)
    np.testing.assert_array_equal(leaves_g, leaves_o)
    # modes used by the GPU (identical to the oracle's, checked above)
    _, _, nm_g, modes_g = gpu_state(room, o.T, o.L, o.kappa, o.M)
    ref = oracle.estimate_pose(q.depth, q.rgb, q.K, leaves_g, nm_g, modes_g.reshape(-1), T, o.D, o.M,
                               w.params, seed)
    n_el = res["n_eligible"]
    assert n_el == len(ref["eligible"]) > 1000
    el_g = room.buffer_np(rl.BUF_ELIGIBLE, np.int32)[:n_el]
    np.testing.assert_array_equal(el_g, ref["eligible"])
    nm_px = room.buffer_np(rl.BUF_NM, np.uint8)[:P]
    np.testing.assert_array_equal(nm_px.astype(np.int32), ref["nm"])
    # hypotheses: triplets, modes and iterations bit-exact, poses to 1e-5
    N = w.params["max_pose_candidates"]
    hy = room.buffer_np(rl.BUF_HYPS, rl.HYP_DTYPE)[:N]
    np.testing.assert_array_equal(hy["valid"].astype(bool), ref["hyp_valid"].astype(bool))
    v = ref["hyp_valid"].astype(bool)
    if not v.any():
        assert res["status"] == ref["status"] == "no_pose" and res["n_valid"] == 0
        return
    np.testing.assert_array_equal(hy["iter"][v], ref["hyp_iter"][v])
    np.testing.assert_array_equal(hy["pix"][v], ref["hyp_pix"][v])
    np.testing.assert_array_equal(hy["mode"][v], ref["hyp_mode"][v])
    np.testing.assert_allclose(hy["R"][v], ref["hyp_pose"][v][:, :9], atol=1e-5)
    np.testing.assert_allclose(hy["t"][v], ref["hyp_pose"][v][:, 9:], atol=1e-5)
    # RANSAC rounds: survivors per round equal, energies to 1e-4 relative
    assert res["rounds"] == ref["rounds"]
    eta = w.params["ransac_inliers_per_iteration"]
    Ig = room.buffer_np(rl.BUF_ILIST, np.int32)[:ref["rounds"] * eta]
    np.testing.assert_array_equal(Ig, ref["I"])
    ts = room.buffer_np(rl.BUF_TRACE_SLOTS, np.int32).reshape(-1, N)
    te = room.buffer_np(rl.BUF_TRACE_ENERGY, np.float64).reshape(-1, N)
    for r in range(ref["rounds"]):
        k = len(ref["round_slots"][r])
        np.testing.assert_array_equal(ts[r, :k], ref["round_slots"][r])
        np.testing.assert_allclose(te[r, :k], ref["round_energy"][r], rtol=1e-4)
    # result
    assert res["status"] == ref["status"] == "ok"
    assert res["winner"] == ref["winner"]
    assert pose_diff(res["pose"], ref["pose"]) < 1e-5
    assert abs(res["energy"] - ref["energy"]) <= 1e-4 * abs(ref["energy"])
    dt, dr = scene.pose_error(res["pose"].astype(np.float64), ref["pose"])
    assert dt < 0.01 and dr < 1.0
    room.set_trace(False)


def test_c1_deterministic(c1):
    w, o, room = c1
    q = w.queries[0]
    d, c = dev(q)
    a = room.relocalise(d, c, q.K, request_seed=5)
    hy_a = room.buffer_np(rl.BUF_HYPS, rl.HYP_DTYPE).copy()
    b = room.relocalise(d, c, q.K, request_seed=5)
    hy_b = room.buffer_np(rl.BUF_HYPS, rl.HYP_DTYPE).copy()
    assert np.array_equal(a["pose"], b["pose"]) and a["energy"] == b["energy"]
    assert hy_a.tobytes() == hy_b.tobytes()
    room.relocalise(d, c, q.K, request_seed=6)
    hy_c = room.buffer_np(rl.BUF_HYPS, rl.HYP_DTYPE).copy()
    assert hy_c.tobytes() != hy_a.tobytes()          # another request seed, another stream


def test_no_pose_cases(c1):
    w, o, room = c1
    q = w.queries[0]
    d, c = dev(q)
    res = room.relocalise(torch.zeros_like(d), c, q.K)
    assert res["status"] == "no_pose" and res["n_eligible"] == 0 and res["energy"] == float("inf")
    assert np.array_equal(res["pose"], np.eye(4, dtype=np.float32))
    fresh = rl.Room(w.params, w.nodes, 160, 120)          # no adaptation: no modes anywhere
    res = fresh.relocalise(d, c, q.K)
    assert res["status"] == "no_pose" and res["n_eligible"] == 0
    fresh.close()


def test_invalid_arguments_rejected_before_launch(c1):
    w, o, room = c1
    q = w.queries[0]
    d, c = dev(q)
    with pytest.raises(rl.RlError):
        room.relocalise(d[:, :158].contiguous(), c[:, :158].contiguous(), q.K)     # width not /4
    big = torch.zeros((240, 320), dtype=torch.float32, device="cuda")
    with pytest.raises(rl.RlError):
        room.relocalise(big, torch.zeros((240, 320, 3), dtype=torch.uint8, device="cuda"), q.K)
    with pytest.raises(rl.RlError):
        room.adapt(d, c, q.K, np.diag([2.0, 1, 1, 1]))                              # not rigid
    with pytest.raises(rl.RlError):
        room.relocalise(d, c, (0.0, 1.0, 80.0, 60.0))                               # bad intrinsics
    bad_nodes = w.nodes.copy()
    bad_nodes["kind"][0, 3] = 7
    with pytest.raises(rl.RlError):
        rl.Room(w.params, bad_nodes, 160, 120)
    p = dict(w.params, pose_update=2)
    with pytest.raises(rl.RlError):
        rl.Room(p, w.nodes, 160, 120)
    # unreliable frames are not inserted
    before = room.buffer_np(rl.BUF_SEEN, np.uint32).copy()
    room.adapt(d, c, q.K, q.pose, reliable=False)
    np.testing.assert_array_equal(room.buffer_np(rl.BUF_SEEN, np.uint32), before)


def test_batch_equals_plain(c1):
    """Batched relocalisation (graph replay and direct launches) gives exactly
    the plain path's result for every (room, frame, seed), whatever the mix."""
    w, o, room = c1
    w2 = workloads.c1(room_id=1, n_queries=2)
    room2 = rl.Room(w2.params, w2.nodes, 160, 120)
    for f in w2.adapt:
        d, c = dev(f)
        room2.adapt(d, c, f.K, f.pose)
    frames = [(room, w.queries[i], 100 + i) for i in range(3)] + [(room2, w2.queries[i], 7 + i) for i in range(2)]
    frames = frames + [(room, w.queries[0], 999)]
    devf = [(r, *dev(q), q.K, s) for (r, q, s) in frames]
    plain = [r.relocalise(d, c, K, request_seed=s) for (r, d, c, K, s) in devf]
    batch = rl.Batch(8, 160, 120, 64, 100, 6, 1, 5)
    for use_graph in (False, True, True):
        got = batch.relocalise(devf, use_graph=use_graph)
        for a, b in zip(got, plain):
            assert a["status"] == b["status"] and a["winner"] == b["winner"]
            assert np.array_equal(a["pose"], b["pose"]) and a["energy"] == b["energy"]
    # a different mix and order reuses nothing it should not
    got = batch.relocalise(devf[::-1][:4], use_graph=True)
    for a, b in zip(got, plain[::-1][:4]):
        assert np.array_equal(a["pose"], b["pose"]) and a["energy"] == b["energy"]
    batch.close()
    # 12 requests over both rooms: equal work (the job table grouped by room)
    # and unequal hypothesis counts (longest first over the XCDs); a job's
    # place in the table changes no result
    big = rl.Batch(16, 160, 120, 64, 100, 6, 1, 5)
    for counts in ((64,) * 12, (64, 32, 16, 64, 48, 32, 64, 16, 32, 64, 48, 16)):
        reqs = [(room if k % 3 else room2, *dev((w if k % 3 else w2).queries[k % 2]),
                 (w if k % 3 else w2).queries[k % 2].K, 300 + k, counts[k]) for k in range(12)]
        want = [r.relocalise(d, c, K, request_seed=sd, n_hypotheses=nh) for (r, d, c, K, sd, nh) in reqs]
        for use_graph in (False, True):
            got = big.relocalise(reqs, use_graph=use_graph)
            for a, b in zip(got, want):
                assert a["status"] == b["status"] and a["winner"] == b["winner"] and a["n_valid"] == b["n_valid"]
                assert np.array_equal(a["pose"], b["pose"]) and a["energy"] == b["energy"]
    big.close()
    room2.close()


def test_adapt_from_back_to_back_temporaries():
    """Frames uploaded into short-lived tensors and adapted with no host wait
    in between: the room must read every frame before its memory is reused."""
    w = workloads.c1(room_id=2, n_queries=1)
    o = oracle.Oracle(w.params, w.nodes)
    room = rl.Room(w.params, w.nodes, 160, 120)
    frames = w.adapt * 6
    for f in frames:
        room.adapt(torch.from_numpy(f.depth).cuda(), torch.from_numpy(f.rgb).cuda(), f.K, f.pose)
        junk = torch.full((120 * 160 * 8,), 7, dtype=torch.uint8, device="cuda")   # churn the allocator
        del junk
    for f in frames:
        o.adapt(f.depth, f.rgb, f.K, f.pose)
    seen, res, _, _ = gpu_state(room, o.T, o.L, o.kappa, o.M)
    np.testing.assert_array_equal(seen, o.seen)
    bad, total = reservoir_mismatches(seen, res, o.reservoir, o.kappa)
    assert total > 1000 and bad == 0, (bad, total)
    room.close()


def test_round_robin_mode_schedule_matches_oracle():
    """Amortised mode update (K leaves per adapted frame, round robin): after
    every adapted frame the GPU's modes equal the oracle's schedule (counts
    exact, rows to float32 rounding); relocalising does not update them."""
    w = workloads.c1(room_id=4, n_queries=1)
    o = oracle.Oracle(w.params, w.nodes)
    room = rl.Room(w.params, w.nodes, 160, 120)
    K = 48
    room.set_mode_schedule(K)
    TL = o.T * o.L
    frames = w.adapt * 2                      # 8 frames: 384 leaves, wraps past 256
    for i, f in enumerate(frames):
        o.adapt(f.depth, f.rgb, f.K, f.pose)
        o.update_modes_round_robin(K)
        d, c = dev(f)
        room.adapt(d, c, f.K, f.pose)
        _, _, nm_g, modes_g = gpu_state(room, o.T, o.L, o.kappa, o.M)
        bad, worst = compare_modes(nm_g, modes_g, o.nmodes, o.modes, o.M, range(TL))
        assert bad == 0 and worst < 1e-5, (i, bad, worst)
    assert int((o.nmodes > 0).sum()) > 50
    q = w.queries[0]
    d, c = dev(q)
    res = room.relocalise(d, c, q.K, request_seed=5)
    _, _, nm_g, modes_g = gpu_state(room, o.T, o.L, o.kappa, o.M)
    np.testing.assert_array_equal(nm_g, o.nmodes)            # no exact update happened
    leaves = o.traverse(q.depth, q.rgb)
    ref = oracle.estimate_pose(q.depth, q.rgb, q.K, leaves, nm_g, modes_g.reshape(-1), o.T, o.D, o.M,
                               w.params, 5)
    assert res["status"] == ref["status"] and res["winner"] == ref["winner"]
    if res["status"] == "ok":
        assert pose_diff(res["pose"], ref["pose"]) < 1e-5
    # the exact update is still available on request and reaches the exact modes
    room.update_modes()
    o.update_modes(all_leaves=False)
    _, _, nm_g, modes_g = gpu_state(room, o.T, o.L, o.kappa, o.M)
    bad, worst = compare_modes(nm_g, modes_g, o.nmodes, o.modes, o.M, range(TL))
    assert bad == 0 and worst < 1e-5
    room.close()


def test_generated_forest_room_matches_oracle(c1, tmp_path):
    """A room on the library's own random forest (rl_forest_generate) routes,
    adapts and relocalises as the oracle does on the same nodes; a saved
    room loaded into a fresh room of the same shape gives the same state and
    the same result, and a room of another shape refuses the file."""
    w, _, _ = c1
    nodes = rl.forest_generate(1, 8, 4242)
    o = oracle.Oracle(w.params, nodes)
    room = rl.Room(w.params, nodes, 160, 120)
    for f in w.adapt:
        o.adapt(f.depth, f.rgb, f.K, f.pose)
        d, c = dev(f)
        room.adapt(d, c, f.K, f.pose)
    room.update_modes()
    q = w.queries[0]
    d, c = dev(q)
    res = room.relocalise(d, c, q.K, request_seed=3)
    ref = o.relocalise(q.depth, q.rgb, q.K, 3)
    leaves = room.buffer_np(rl.BUF_LEAVES, np.uint16).reshape(-1, 8)[:q.depth.size, :1]
    np.testing.assert_array_equal(leaves, ref["leaves"])
    assert res["status"] == ref["status"]
    if ref["status"] == "ok":
        assert res["winner"] == ref["winner"] and pose_diff(res["pose"], ref["pose"]) < 1e-5
    # persistence
    path = tmp_path / "room.bin"
    room.save(path)
    fresh = rl.Room(w.params, nodes, 160, 120)
    fresh.load(path)
    for which in (rl.BUF_NODES, rl.BUF_RESERVOIR, rl.BUF_SEEN, rl.BUF_MODES, rl.BUF_NMODES, rl.BUF_CBOX):
        assert np.array_equal(fresh.buffer_np(which, np.uint8), room.buffer_np(which, np.uint8)), which
    again = fresh.relocalise(d, c, q.K, request_seed=3)
    assert again["status"] == res["status"] and np.array_equal(again["pose"], res["pose"])
    assert again["energy"] == res["energy"] or (np.isinf(again["energy"]) and np.isinf(res["energy"]))
    other = rl.Room(dict(w.params, max_cluster_count=4), nodes, 160, 120)
    with pytest.raises(rl.RlError):
        other.load(path)
    (tmp_path / "junk.bin").write_bytes(b"not a room")
    with pytest.raises(rl.RlError):
        fresh.load(tmp_path / "junk.bin")
    for r in (room, fresh, other):
        r.close()


def _single_row_frame():
    """A noise-free 160x120 frame of room 0 whose depth is kept on one image
    row only, a row crossing exactly two surfaces (at least 50 pixels each).
    Three pixels on one surface back-project to collinear camera points, so
    their Kabsch fit is degenerate (Sec. 3.2.3); triplets spanning both
    surfaces are not."""
    w, h = 160, 120
    room = scene.make_room(0)
    rng = np.random.default_rng(123)
    while True:
        H = scene.random_pose(room, rng)
        z, _, sid = scene.raycast(room, H, w, h)
        for y in range(8, 113, 4):
            ok = np.isfinite(z[y]) & (z[y] >= 0.5) & (z[y] <= 4.0)
            ids, cnt = np.unique(sid[y], return_counts=True)
            if ok.all() and len(ids) == 2 and cnt.min() >= 50:
                depth, rgb = scene.render(room, H, w, h, seed=5, noise_sigma=0.0, dropout=0.0)
                row = np.zeros_like(depth)
                row[y] = depth[y]
                return row, rgb, H, scene.intrinsics(w, h)


def test_degenerate_triplets_skipped_as_the_oracle_does():
    """A frame on which iterations pass checks 1-3 with collinear (degenerate)
    triplets before the accepted one: the triplets, iterations and poses of
    every slot equal the oracle's, with the search's degeneracy screen on and
    with it off (then every such triplet reaches the exact test, which rejects
    it and continues the slot's scan), and both give identical results."""
    from tests.test_oracle_hypothesis_rejection import Frame, _key, evaluate
    from rlsynth import forest, presets
    p = presets.preset("c1")
    nodes = forest.make_forest(1000, **presets.FOREST["c1"])
    depth, rgb, H, K = _single_row_frame()
    o = oracle.Oracle(p, nodes)
    room = rl.Room(p, nodes, 160, 120)
    d = torch.from_numpy(depth).cuda()
    c = torch.from_numpy(rgb).cuda()
    for _ in range(8):                        # eight identical adaptations: clusters of >= 5 points
        o.adapt(depth, rgb, K, H)
        room.adapt(d, c, K, H)
    o.update_modes()
    room.update_modes()
    _, _, nm_g, modes_g = gpu_state(room, o.T, o.L, o.kappa, o.M)
    bad, worst = compare_modes(nm_g, modes_g, o.nmodes, o.modes, o.M, range(o.T * o.L))
    assert bad == 0 and worst < 1e-5, (bad, worst)
    leaves = o.traverse(depth, rgb)
    N = p["max_pose_candidates"]
    seed = 0
    ref = oracle.estimate_pose(depth, rgb, K, leaves, nm_g, modes_g.reshape(-1), o.T, o.D, o.M, p, seed)
    v = ref["hyp_valid"].astype(bool)
    assert v.sum() >= 32
    # the construction's point: slots whose accepted iteration follows an
    # iteration that passes checks 1-3 with a degenerate fit (numpy re-evaluation)
    fr = Frame(depth, rgb, K, leaves, nm_g, modes_g.reshape(-1), o.T, o.D, o.M, ref["eligible"])
    key = _key(p, seed)
    degenerate_first = [s for s in np.flatnonzero(v)
                        if any(evaluate(fr, key, int(s), it, p) == 4 for it in range(int(ref["hyp_iter"][s])))]
    print(f"[degenerate] {int(v.sum())} valid slots, {len(degenerate_first)} accepted after a degenerate "
          f"triplet passed checks 1-3", flush=True)
    assert len(degenerate_first) >= 3
    results = []
    for screen in (True, False):
        room.set_degeneracy_screen(screen)
        res = room.relocalise(d, c, K, request_seed=seed)
        hy = room.buffer_np(rl.BUF_HYPS, rl.HYP_DTYPE)[:N].copy()
        np.testing.assert_array_equal(hy["valid"].astype(bool), v)
        np.testing.assert_array_equal(hy["iter"][v], ref["hyp_iter"][v])
        np.testing.assert_array_equal(hy["pix"][v], ref["hyp_pix"][v])
        np.testing.assert_array_equal(hy["mode"][v], ref["hyp_mode"][v])
        np.testing.assert_allclose(hy["R"][v], ref["hyp_pose"][v][:, :9], atol=1e-5)
        np.testing.assert_allclose(hy["t"][v], ref["hyp_pose"][v][:, 9:], atol=1e-5)
        assert res["status"] == ref["status"] == "ok" and res["winner"] == ref["winner"]
        assert pose_diff(res["pose"], ref["pose"]) < 1e-5
        results.append((res, hy))
    (a, ha), (b, hb) = results
    assert ha.tobytes() == hb.tobytes() and np.array_equal(a["pose"], b["pose"]) and a["energy"] == b["energy"]
    room.set_degeneracy_screen(True)
    room.close()


def test_back_to_back_async_batches_equal_plain(c1):
    """Two asynchronous batches with different requests queued back to back
    (no host wait in between), then a third reusing the first's request list:
    each result equals the plain path's."""
    w, o, room = c1
    frames = [(room, w.queries[i % 3], 300 + i) for i in range(5)]
    devf = [(r, *dev(q), q.K, s) for (r, q, s) in frames]
    plain = [r.relocalise(d, c, K, request_seed=s) for (r, d, c, K, s) in devf]
    batch = rl.Batch(4, 160, 120, 64, 100, 6, 1, 5)
    nbytes = ctypes.sizeof(rl.Result) * 4
    outs = [torch.empty(nbytes, dtype=torch.uint8, device="cuda") for _ in range(3)]
    plans = [devf[:3], devf[3:], devf[:3][::-1]]
    wants = [plain[:3], plain[3:], plain[:3][::-1]]
    for reqs, out in zip(plans, outs):
        batch.relocalise_async(reqs, out, use_graph=True)
    batch.stream.synchronize()
    for reqs, out, want in zip(plans, outs, wants):
        got = rl.Batch.decode(out.cpu().numpy(), len(reqs))
        for a, b in zip(got, want):
            assert a["status"] == b["status"] and a["winner"] == b["winner"]
            assert np.array_equal(a["pose"], b["pose"]) and a["energy"] == b["energy"]
    batch.close()


def _same_room_state(A, B, tag):
    """Arrival counters, dirty flags and mode counts equal; the filled part of
    every reservoir and every mode row in use equal bit for bit."""
    p = A.params
    TL, kappa, M = p["n_trees"] << p["depth"], p["reservoir_capacity"], p["max_cluster_count"]
    for buf, dt in ((rl.BUF_SEEN, np.uint32), (rl.BUF_DIRTY, np.uint32), (rl.BUF_NMODES, np.uint8)):
        assert np.array_equal(A.buffer_np(buf, dt), B.buffer_np(buf, dt)), (tag, buf)
    seen = A.buffer_np(rl.BUF_SEEN, np.uint32).copy()
    ra = A.buffer_np(rl.BUF_RESERVOIR, np.uint32).reshape(TL, kappa, 4)
    rb = B.buffer_np(rl.BUF_RESERVOIR, np.uint32).reshape(TL, kappa, 4)
    used = np.arange(kappa)[None, :] < np.minimum(seen, kappa)[:, None]
    assert np.array_equal(ra[used], rb[used]), (tag, "reservoir")
    nm = A.buffer_np(rl.BUF_NMODES, np.uint8).astype(np.int64)
    ma = A.buffer_np(rl.BUF_MODES, np.uint32).reshape(TL, M, 16)
    mb = B.buffer_np(rl.BUF_MODES, np.uint32).reshape(TL, M, 16)
    used = np.arange(M)[None, :] < nm[:, None]
    assert np.array_equal(ma[used], mb[used]), (tag, "modes")


@pytest.mark.parametrize("leaves_per_frame", [0, 64, (64, 300)])
def test_batched_adaptations_equal_plain_sequence(leaves_per_frame):
    """Adaptation requests inside batches (two rooms, mixed with
    relocalisations, one batch replayed from a graph and one launched
    directly): each batch's relocalisations see the rooms as they were before
    its adaptations, and afterwards reservoirs, arrival counters, dirty flags
    and modes equal those of plain adapt calls in request order, bit for bit,
    under the exact and the round-robin mode schedule.  (64, 300): two-tree
    rooms whose round-robin steps share one launch, the first split into row
    chunks (at most 256 leaves), the second not."""
    from rlsynth import forest, presets
    specs = [workloads.c1(room_id=r, n_queries=2) for r in (0, 1)]
    mixed = isinstance(leaves_per_frame, tuple)
    T = 2 if mixed else 1
    nodes = [forest.make_forest(1000 + r, **dict(presets.FOREST["c1"], n_trees=2)) if mixed else w.nodes
             for r, w in enumerate(specs)]
    params = [dict(w.params, n_trees=T) for w in specs]
    schedules = leaves_per_frame if mixed else (leaves_per_frame, leaves_per_frame)

    def make():
        out = []
        for r, w in enumerate(specs):
            room = rl.Room(params[r], nodes[r], 160, 120)
            room.set_mode_schedule(schedules[r])
            for f in w.adapt[:2]:
                room.adapt(*dev(f), f.K, f.pose)
            out.append(room)
        return out

    A, B = make(), make()
    M = params[0]["max_cluster_count"]
    batch = rl.Batch(8, 160, 120, 64, 100, 6, T, T * M)
    frames = {}

    def F(f):
        if id(f) not in frames:
            frames[id(f)] = dev(f)
        return frames[id(f)]

    plans = [
        [("r", 0, specs[0].queries[0], 11), ("a", 0, specs[0].adapt[2]), ("r", 1, specs[1].queries[0], 12),
         ("a", 1, specs[1].adapt[2]), ("a", 0, specs[0].adapt[3]), ("r", 0, specs[0].queries[1], 13)],
        [("a", 1, specs[1].adapt[3]), ("r", 0, specs[0].queries[0], 21), ("r", 1, specs[1].queries[1], 22)],
    ]
    for k, plan in enumerate(plans):
        items = []
        for step in plan:
            if step[0] == "r":
                _, r, q, seed = step
                items.append((A[r], *F(q), q.K, seed))
            else:
                _, r, f = step
                items.append(rl.AdaptRequest(A[r], *F(f), f.K, f.pose))
        got = batch.relocalise(items, use_graph=(k == 0))
        # plain: the relocalisations first, then the adaptations in order
        for step, g in zip(plan, got):
            if step[0] == "r":
                _, r, q, seed = step
                want = B[r].relocalise(*F(q), q.K, request_seed=seed)
                assert g["status"] == want["status"] and g["winner"] == want["winner"], step
                assert np.array_equal(g["pose"], want["pose"]) and g["energy"] == want["energy"], step
            else:
                assert g["status"] == "ok" and g["winner"] == -1 and g["rounds"] == 0
        for step in plan:
            if step[0] == "a":
                _, r, f = step
                B[r].adapt(*F(f), f.K, f.pose)
        torch.cuda.synchronize()
        for r in (0, 1):
            if schedules[r] == 0:
                A[r].update_modes()
                B[r].update_modes()
            torch.cuda.synchronize()
            _same_room_state(A[r], B[r], (k, r))
    # a room's own stream continues after a batch's adaptation of it
    f = specs[0].adapt[0]
    A[0].adapt(*F(f), f.K, f.pose)
    B[0].adapt(*F(f), f.K, f.pose)
    q = specs[0].queries[1]
    a, b = A[0].relocalise(*F(q), q.K, request_seed=5), B[0].relocalise(*F(q), q.K, request_seed=5)
    assert np.array_equal(a["pose"], b["pose"]) and a["energy"] == b["energy"]
    with pytest.raises(rl.RlError):
        batch.relocalise([rl.AdaptRequest(A[0], *F(f), f.K, np.diag([2.0, 1.0, 1.0, 1.0]))])
    batch.close()
    for room in A + B:
        room.close()


def test_adapt_every_grid_pixel_into_one_leaf_bit_exact():
    """Adaptation when every grid pixel of a 640x480 frame reaches the same
    leaf of each tree (constant depth and colour: every feature is 0): 18,921
    arrivals per leaf and frame, spread over 19 chunks, most of them Algorithm
    R replacements with several arrivals of a frame drawing the same slot
    (the later one wins).  Three frames at different poses; arrival counters
    and every reservoir entry equal the oracle's bit for bit."""
    from rlsynth import forest, presets
    p = dict(presets.preset("c2"), reservoir_capacity=64)
    nodes = forest.make_forest(1000, **presets.FOREST["c2"])
    o = oracle.Oracle(p, nodes)
    room = rl.Room(p, nodes, 640, 480)
    K = scene.intrinsics(640, 480)
    depth = np.full((480, 640), 2.0, np.float32)
    rgb = np.full((480, 640, 3), 90, np.uint8)
    rng = np.random.default_rng(17)
    geom = scene.make_room(0)
    for k in range(3):
        H = scene.random_pose(geom, rng)
        o.adapt(depth, rgb, K, H)
        room.adapt(torch.from_numpy(depth).cuda(), torch.from_numpy(rgb).cuda(), K, H)
    seen = room.buffer_np(rl.BUF_SEEN, np.uint32).copy()
    np.testing.assert_array_equal(seen, o.seen)
    assert int(seen.max()) == 3 * 159 * 119 and int((seen > 0).sum()) == o.T
    res = room.buffer_np(rl.BUF_RESERVOIR, np.float32).reshape(o.T * o.L, o.kappa, 4)
    bad, total = reservoir_mismatches(seen, res, o.reservoir, o.kappa)
    assert bad == 0 and total == o.T * o.kappa, (bad, total)
    dirty = room.buffer_np(rl.BUF_DIRTY, np.uint32)
    np.testing.assert_array_equal(dirty != 0, o.dirty != 0)
    room.close()


def _same_result(a, b):
    assert a["status"] == b["status"] and a["winner"] == b["winner"] and a["n_valid"] == b["n_valid"]
    assert np.array_equal(a["pose"], b["pose"]) and a["energy"] == b["energy"]


def test_frames_read_in_place_pitched_rgba_and_decimated(c1):
    """Frames in any row pitch, RGB or RGBA, and the 2x decimated frame read
    in place (every second pixel of every second row) give the results of the
    same pixels in tightly packed RGB buffers: relocalisation, adaptation and
    the depth-raycast score, bit for bit."""
    w, o, room = c1
    q = w.queries[0]
    d, c = dev(q)
    ref = room.relocalise(d, c, q.K, request_seed=9)
    # rows padded to 176 pixels, colour as RGBA
    dp = torch.zeros((120, 176), dtype=torch.float32, device="cuda")
    dp[:, :160] = d
    cp = torch.full((120, 184, 4), 255, dtype=torch.uint8, device="cuda")
    cp[:, :160, :3] = c
    _same_result(room.relocalise(dp[:, :160], cp[:, :160], q.K, request_seed=9), ref)
    _same_result(room.relocalise(dp[:, :160], cp[:, :160, :3], q.K, request_seed=9), ref)
    # the 2x decimated view of a 320x240 frame against its packed copy
    geom = scene.make_room(0)
    d2, c2 = scene.render(geom, q.pose, 320, 240, seed=31)
    D2, C2 = torch.from_numpy(d2).cuda(), torch.from_numpy(c2).cuda()
    fx, fy, cx, cy = scene.intrinsics(320, 240)
    Kd = (fx / 2, fy / 2, cx / 2, cy / 2)
    packed = room.relocalise(D2[::2, ::2].contiguous(), C2[::2, ::2].contiguous(), Kd, request_seed=4)
    _same_result(room.relocalise(D2[::2, ::2], C2[::2, ::2], Kd, request_seed=4), packed)
    assert packed["n_eligible"] > 0
    # depth-raycast scores from views
    S = scene.surface_records(geom)
    P = np.concatenate([q.pose[:3, :3].reshape(-1), q.pose[:3, 3]])[None].astype(np.float32)
    a = room.depth_scores(dp[:, :160], cp[:, :160], q.K, S, P, 0.5, 4.0)
    b = room.depth_scores(d, c, q.K, S, P, 0.5, 4.0)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)
    # adaptation from a pitched RGBA view and from packed buffers
    rooms = [rl.Room(w.params, w.nodes, 160, 120) for _ in range(2)]
    for f in w.adapt:
        fd, fc = dev(f)
        rooms[0].adapt(fd, fc, f.K, f.pose)
        pd = torch.zeros((120, 168), dtype=torch.float32, device="cuda")
        pd[:, :160] = fd
        pc = torch.zeros((120, 160, 4), dtype=torch.uint8, device="cuda")
        pc[..., :3] = fc
        rooms[1].adapt(pd[:, :160], pc, f.K, f.pose)
    rooms[0].update_modes()
    rooms[1].update_modes()
    _same_room_state(rooms[0], rooms[1], "adapt from views")
    for r in rooms:
        r.close()
    # views the library cannot read in place are refused
    with pytest.raises(TypeError):
        room.relocalise(d[:, ::3], c[:, ::3], q.K)


@pytest.mark.parametrize("leaves_per_frame", [0, 64])
def test_mode_version_counts_mode_updates(leaves_per_frame):
    """rl_result.mode_version: the mode updates a relocalisation's room had
    received; equal for the plain and the batched path, unchanged between two
    relocalisations with no adaptation in between, and advanced by an
    adaptation (at the next relocalisation under the exact schedule, at the
    adaptation itself under the round-robin one)."""
    w = workloads.c1(n_queries=1)
    room = rl.Room(w.params, w.nodes, 160, 120)
    room.set_mode_schedule(leaves_per_frame)
    q = w.queries[0]
    d, c = dev(q)
    v0 = room.relocalise(d, c, q.K)["mode_version"]
    assert v0 == 0
    versions = []
    batch = rl.Batch(2, 160, 120, 64, 100, 6, 1, 5)
    for f in w.adapt:
        room.adapt(*dev(f), f.K, f.pose)
        a = room.relocalise(d, c, q.K, request_seed=1)
        b = room.relocalise(d, c, q.K, request_seed=2)
        g = batch.relocalise([(room, d, c, q.K, 1)])[0]
        assert a["mode_version"] == b["mode_version"] == g["mode_version"]
        _same_result(a, g)
        versions.append(a["mode_version"])
    assert versions == list(range(1, len(w.adapt) + 1))
    # an adaptation inside a batch reports the version after its own update
    f = w.adapt[0]
    got = batch.relocalise([(room, d, c, q.K, 3), rl.AdaptRequest(room, *dev(f), f.K, f.pose)])
    assert got[0]["mode_version"] == versions[-1]
    after = room.relocalise(d, c, q.K)["mode_version"]
    assert after == versions[-1] + 1
    if leaves_per_frame:
        assert got[1]["mode_version"] == after
    batch.close()
    room.close()
