"""Serving scheduler policy without a GPU: per-room arrival order is kept
(a relocalisation sees exactly the adaptations of its room that arrived before
it), batches respect their cap, admission refuses beyond the queue bound and
every request is eventually issued."""
import collections
import os
import random

import pytest

from paper_1810_12163_amd.serve import Request, form_batch


class FakeRoom:
    def __init__(self, name):
        self.name = name


def simulate(seed, n_rooms=4, n_req=300, max_batch=5):
    rng = random.Random(seed)
    rooms = [FakeRoom(i) for i in range(n_rooms)]
    reqs = [Request(rid=i, kind="adapt" if rng.random() < 0.3 else "relocalise", room=rng.choice(rooms))
            for i in range(n_req)]
    pending = collections.deque()
    issued = []                      # (batch, position in batch, request)
    k = 0
    nb = 0
    while k < n_req or pending:
        for _ in range(rng.randint(0, 6)):          # arrivals of this pass
            if k < n_req:
                pending.append(reqs[k])
                k += 1
        if rng.random() < 0.6:                      # is a context free?
            batch, keep = form_batch(pending, max_batch)
            assert len(batch) <= max_batch
            assert [q.rid for q in batch] == sorted(q.rid for q in batch)
            for i, q in enumerate(batch):
                issued.append((nb, i, q))
            assert [q.rid for q in keep] == sorted(q.rid for q in keep)
            pending = keep
            nb += 1
        assert nb < 10_000
    return reqs, issued


@pytest.mark.parametrize("seed", range(20))
def test_per_room_arrival_order(seed):
    """Per room, in arrival order: a relocalisation after an adaptation runs in
    a later batch (a batch's relocalisations run before its adaptations and
    see the rooms as they were); otherwise a later request is never in an
    earlier batch, and adaptations of one batch keep their order."""
    reqs, issued = simulate(seed)
    assert sorted(q.rid for _, _, q in issued) == list(range(len(reqs)))
    when = {q.rid: (b, i) for b, i, q in issued}
    by_room = collections.defaultdict(list)
    for q in reqs:
        by_room[q.room.name].append(q)
    for rq in by_room.values():
        for x, y in zip(rq, rq[1:]):
            if x.kind == "adapt" and y.kind != "adapt":
                assert when[x.rid][0] < when[y.rid][0], (x, y)
            else:
                assert when[x.rid] < when[y.rid], (x, y)


def test_batch_fills_across_rooms_and_adapt_blocks_later_relocalisations_of_its_room():
    rooms = [FakeRoom(i) for i in range(3)]
    pending = collections.deque([
        Request(0, "relocalise", rooms[0]), Request(1, "relocalise", rooms[1]),
        Request(2, "adapt", rooms[0]), Request(3, "relocalise", rooms[0]),
        Request(4, "relocalise", rooms[2]), Request(5, "adapt", rooms[1]),
        Request(6, "adapt", rooms[2]), Request(7, "relocalise", rooms[1]),
        Request(8, "adapt", rooms[0]),
    ])
    batch, keep = form_batch(pending, 8)
    # 3 waits for adapt 2 of its room; 8 may not pass 3; 7 waits for adapt 5
    assert [q.rid for q in batch] == [0, 1, 2, 4, 5, 6]
    assert [q.rid for q in keep] == [3, 7, 8]
    batch, keep = form_batch(keep, 8)
    assert [q.rid for q in batch] == [3, 7, 8] and not keep


def test_full_batch_keeps_the_rest_in_order():
    rooms = [FakeRoom(i) for i in range(2)]
    pending = collections.deque([Request(i, "relocalise" if i % 3 else "adapt", rooms[i % 2]) for i in range(7)])
    batch, keep = form_batch(pending, 3)
    # 2 (room 0) waits for adapt 0 of its room; adapt 3 (room 1) fills the batch
    assert [q.rid for q in batch] == [0, 1, 3] and [q.rid for q in keep] == [2, 4, 5, 6]
    batch, keep = form_batch(pending, 0)
    assert not batch and len(keep) == 7


def test_admission_refuses_beyond_the_queue_bound():
    from paper_1810_12163_amd import serve
    s = serve.Server.__new__(serve.Server)          # policy-only: no device state needed
    s.pending = collections.deque()
    s.backlog = collections.deque()
    s.refused = []
    s.host_s = collections.Counter()
    s.max_queue = 3
    rooms = [FakeRoom(0)]
    ok = [s.admit(Request(i, "relocalise", rooms[0]), float(i)) for i in range(5)]
    assert ok == [True, True, True, False, False]
    assert [q.rid for q in s.refused] == [3, 4] and all(q.refused for q in s.refused)


def _policy_server(n_slots, max_queue=64, budget=None):
    """A server reduced to its admission state, with a frame pool in host
    memory (no device work)."""
    from paper_1810_12163_amd import serve
    s = serve.Server.__new__(serve.Server)
    s.pending = collections.deque()
    s.backlog = collections.deque()
    s.refused = []
    s.deferred = 0
    s.max_backlog = 0
    s.max_queue = max_queue
    s.host_s = collections.Counter()
    s.ledger = serve.Ledger(budget)
    s.pool = serve.FramePool(n_slots, 16, 8, "cpu") if n_slots else None
    return s


def _host_req(i, room, h=8, w=16):
    import torch
    from paper_1810_12163_amd.serve import Request
    d = torch.full((h, w), float(i), dtype=torch.float32)
    c = torch.full((h, w, 3), i % 256, dtype=torch.uint8)
    return Request(i, "relocalise", room, host_depth=d, host_rgb=c)


def test_requests_wait_for_frame_slots_in_arrival_order():
    """With two frame slots, later requests wait in the backlog (not refused)
    and take slots in arrival order as earlier requests release theirs; the
    frame copied into a slot is the request's own."""
    pytest.importorskip("torch")
    s = _policy_server(2)
    room = FakeRoom(0)
    reqs = [_host_req(i, room) for i in range(5)]
    assert all(s.admit(q, float(i)) for i, q in enumerate(reqs))
    assert [q.rid for q in s.pending] == [0, 1] and [q.rid for q in s.backlog] == [2, 3, 4]
    assert s.deferred == 3 and s.max_backlog == 3 and not s.refused
    for q in list(s.pending):
        assert float(q.depth[0, 0]) == q.rid and int(q.rgb[0, 0, 0]) == q.rid
    s._release(s.pending.popleft())          # request 0 completes
    s._refill()
    assert [q.rid for q in s.pending] == [1, 2] and [q.rid for q in s.backlog] == [3, 4]
    assert float(s.pending[1].depth[0, 0]) == 2.0
    # a smaller frame uses the head of a slot
    small = _host_req(9, room, h=4, w=8)
    s._release(s.pending.popleft())
    s._release(s.pending.popleft())
    s._refill()
    assert [q.rid for q in s.pending] == [3, 4] and not s.backlog
    assert s.admit(small, 9.0) is True and s.backlog[0] is small     # no free slot: waits
    s._release(s.pending.popleft())
    s._refill()
    assert small.depth.shape == (4, 8) and float(small.depth[3, 7]) == 9.0


def test_queue_bound_counts_waiting_requests():
    pytest.importorskip("torch")
    s = _policy_server(1, max_queue=3)
    room = FakeRoom(0)
    ok = [s.admit(_host_req(i, room), float(i)) for i in range(5)]
    assert ok == [True, True, True, False, False]
    assert len(s.pending) == 1 and len(s.backlog) == 2 and len(s.refused) == 2


def test_ledger_refuses_what_does_not_fit():
    from paper_1810_12163_amd.serve import Ledger
    led = Ledger(100)
    assert led.charge("a", 60) and led.used == 60
    assert not led.charge("b", 41) and "b" not in led.items
    assert led.charge("b", 40) and led.used == 100 and not led.fits(1)
    led.release("a")
    assert led.fits(60) and not led.fits(61)
    assert Ledger(None).charge("x", 1 << 60)


def test_room_admission_by_budget():
    """A room whose persistent state and scratch exceed what is left of the
    budget is refused before any device memory is taken."""
    rl = pytest.importorskip("paper_1810_12163_amd")
    if not os.path.exists(rl.LIB_PATH):
        pytest.skip("librl.so not built")
    pb, sb = rl.room_state_bytes(rl.preset("c2"), 640, 480)
    s = _policy_server(0, budget=pb + sb - 1)
    s.rooms = []
    s.max_width, s.max_height = 640, 480
    assert s.create_room(rl.preset("c2"), None) is None and s.ledger.used == 0


def test_one_buffer_host_frame_lands_in_its_slot():
    """A frame packed as one host buffer (depth bytes, then colour bytes) is
    copied into a slot in one piece; the slot's views give back the frame."""
    torch = pytest.importorskip("torch")
    import numpy as np
    from paper_1810_12163_amd.serve import Request
    s = _policy_server(1)
    rng = np.random.default_rng(0)
    d = rng.uniform(0.5, 4.0, size=(4, 8)).astype(np.float32)
    c = rng.integers(0, 256, size=(4, 8, 3), dtype=np.uint8)
    buf = torch.from_numpy(np.concatenate([d.view(np.uint8).reshape(-1), c.reshape(-1)]))
    q = Request(0, "relocalise", FakeRoom(0), host_frame=buf, frame_hw=(4, 8))
    assert s.admit(q, 0.0) and q.slot == 0
    assert np.array_equal(q.depth.numpy(), d) and np.array_equal(q.rgb.numpy(), c)
