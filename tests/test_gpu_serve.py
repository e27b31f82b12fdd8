"""Continuous batching on the GPU: every relocalisation served in a mix of
rooms, resolutions and interleaved adaptations equals the same request run
alone through the plain path, in arrival order, bit for bit."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1810_12163_amd as rl  # noqa: E402
from paper_1810_12163_amd import serve  # noqa: E402
from rlsynth import workloads  # noqa: E402
from tests.gpu_util import dev  # noqa: E402


@pytest.mark.parametrize("leaves_per_frame", [0, 64])
def test_served_equals_alone(leaves_per_frame):
    """Under the exact mode schedule and under the amortised one."""
    specs = [workloads.c1(room_id=r, n_queries=3) for r in (0, 1, 2)]

    def make_rooms():
        out = []
        for w in specs:
            room = rl.Room(w.params, w.nodes, 160, 120)
            room.set_mode_schedule(leaves_per_frame)
            for f in w.adapt:
                d, c = dev(f)
                room.adapt(d, c, f.K, f.pose)
            out.append(room)
        return out

    served_rooms, alone_rooms = make_rooms(), make_rooms()
    rng = np.random.default_rng(0)
    plan = []
    for i in range(60):
        r = int(rng.integers(3))
        if rng.uniform() < 0.25:
            plan.append(("adapt", r, specs[r].adapt[int(rng.integers(4))]))
        else:
            plan.append(("relocalise", r, specs[r].queries[int(rng.integers(3))]))
    frames = {id(f): dev(f) for _, _, f in plan}
    server = serve.Server(max_batch=8, max_width=160, max_height=120, max_hypotheses=64, max_eta=100,
                          max_rounds=6, n_trees=1, max_modes_per_pixel=5, contexts=2)
    reqs = []
    for i, (kind, r, f) in enumerate(plan):
        d, c = frames[id(f)]
        reqs.append(serve.Request(rid=i, kind=kind, room=served_rooms[r], depth=d, rgb=c, K=f.K,
                                  pose=f.pose if kind == "adapt" else None))
    stats = serve.run_open_loop(server, reqs, np.linspace(0.0, 0.03, len(reqs)))
    assert stats["n"] == sum(1 for k, _, _ in plan if k == "relocalise")
    assert stats["batches"] >= 2 and stats["refused"] == 0
    for i, (kind, r, f) in enumerate(plan):
        d, c = frames[id(f)]
        if kind == "adapt":
            alone_rooms[r].adapt(d, c, f.K, f.pose)
            continue
        a = alone_rooms[r].relocalise(d, c, f.K, request_seed=i)
        s = reqs[i].result
        assert s["status"] == a["status"] and s["winner"] == a["winner"], i
        assert np.array_equal(s["pose"], a["pose"]) and s["energy"] == a["energy"], i
    server.close()


def test_served_equals_alone_640x480_host_frames():
    """Two 640x480 rooms (five depth-15 trees): requests arrive with frames in
    host memory, the server's memory budget leaves it four frame slots, so
    most requests wait for a slot; every relocalisation still equals the same
    request run alone in arrival order."""
    from rlsynth import presets
    p = presets.preset("c2")
    specs = []
    for r in (0, 1):
        room, nodes, adapt = workloads.room_setup(r, 8)
        qs = workloads.queries_for(room, [f.pose for f in adapt], 3, room_id=r)
        specs.append((nodes, adapt, qs))
    room_bytes = sum(rl.room_state_bytes(p, 640, 480))
    ctx = serve.batch_workspace_bytes(16, 640, 480, 1024, 500, 10, 5, 50)
    budget = 2 * room_bytes + 2 * ctx + 4 * serve.FramePool.slot_bytes(640, 480)
    server = serve.Server(max_batch=16, max_width=640, max_height=480, max_hypotheses=1024, max_eta=500,
                          max_rounds=10, n_trees=5, max_modes_per_pixel=50, contexts=2, memory_budget=budget,
                          frame_slots=64)
    assert len(server.ctx) == 2
    served = [server.create_room(p, nodes) for nodes, _, _ in specs]
    assert all(r is not None for r in served) and server.create_room(p, specs[0][0]) is None
    alone = [rl.Room(p, nodes, 640, 480) for nodes, _, _ in specs]
    for k, (nodes, adapt, _) in enumerate(specs):
        for f in adapt[:6]:
            for room in (served[k], alone[k]):
                d, c = dev(f)
                room.adapt(d, c, f.K, f.pose)
    rng = np.random.default_rng(1)
    plan = []
    for i in range(24):
        r = int(rng.integers(2))
        if rng.uniform() < 0.25:
            plan.append(("adapt", r, specs[r][1][6 + int(rng.integers(2))]))
        else:
            plan.append(("relocalise", r, specs[r][2][int(rng.integers(3))]))
    host = {id(f): (torch.from_numpy(f.depth).pin_memory(), torch.from_numpy(f.rgb).pin_memory())
            for _, _, f in plan}
    reqs = [serve.Request(rid=i, kind=kind, room=served[r], host_depth=host[id(f)][0], host_rgb=host[id(f)][1],
                          K=f.K, pose=f.pose if kind == "adapt" else None)
            for i, (kind, r, f) in enumerate(plan)]
    stats = serve.run_open_loop(server, reqs, np.zeros(len(reqs)))
    assert server.pool.n_slots == 4
    print(f"[served 640x480] {stats}", flush=True)
    assert stats["refused"] == 0 and stats["deferred"] > 0 and stats["n"] == sum(k == "relocalise" for k, _, _ in plan)
    for i, (kind, r, f) in enumerate(plan):
        d, c = dev(f)
        if kind == "adapt":
            alone[r].adapt(d, c, f.K, f.pose)
            continue
        a = alone[r].relocalise(d, c, f.K, request_seed=i)
        s = reqs[i].result
        assert s["status"] == a["status"] and s["winner"] == a["winner"], i
        assert np.array_equal(s["pose"], a["pose"]) and s["energy"] == a["energy"], i
    assert len(server.pool.free) == 4                  # every slot returned
    server.close()
    for room in alone:
        room.close()
