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
