"""Serving scheduler policy without a GPU: per-room arrival order is kept
(a relocalisation sees exactly the adaptations of its room that arrived before
it), batches respect their cap, admission refuses beyond the queue bound and
every request is eventually issued."""
import collections
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
    issued = []                      # (pass, order within pass, request)
    k = 0
    p = 0
    while k < n_req or pending:
        for _ in range(rng.randint(0, 6)):          # arrivals of this pass
            if k < n_req:
                pending.append(reqs[k])
                k += 1
        free = rng.random() < 0.6                   # is a context free?
        batch, adapts, keep = form_batch(pending, max_batch if free else 0)
        assert len(batch) <= max_batch
        assert not batch or free
        order = 0
        for q in adapts:
            issued.append((p, order, q))
            order += 1
        for q in batch:
            issued.append((p, order, q))            # batch submitted after the adapts
        assert [q.rid for q in keep] == sorted(q.rid for q in keep)
        pending = keep
        p += 1
        assert p < 10_000
    return reqs, issued


@pytest.mark.parametrize("seed", range(20))
def test_per_room_arrival_order(seed):
    reqs, issued = simulate(seed)
    assert sorted(q.rid for _, _, q in issued) == list(range(len(reqs)))
    when = {q.rid: (p, o) for p, o, q in issued}
    by_room = collections.defaultdict(list)
    for q in reqs:
        by_room[q.room.name].append(q)
    for rq in by_room.values():
        for a, b in zip(rq, rq[1:]):
            if a.kind == "relocalise" and b.kind == "relocalise":
                assert when[a.rid][0] <= when[b.rid][0]     # may share a batch
            else:
                assert when[a.rid] < when[b.rid], (a, b)     # adapts are barriers


def test_batch_fills_across_rooms_and_adapt_blocks_only_its_room():
    rooms = [FakeRoom(i) for i in range(3)]
    pending = collections.deque([
        Request(0, "relocalise", rooms[0]), Request(1, "relocalise", rooms[1]),
        Request(2, "adapt", rooms[0]), Request(3, "relocalise", rooms[0]),
        Request(4, "relocalise", rooms[2]), Request(5, "adapt", rooms[1]),
        Request(6, "adapt", rooms[2]), Request(7, "relocalise", rooms[1]),
    ])
    batch, adapts, keep = form_batch(pending, 8)
    assert [q.rid for q in batch] == [0, 1, 4]
    assert [q.rid for q in adapts] == []           # each follows a batched request of its room
    assert [q.rid for q in keep] == [2, 3, 5, 6, 7]
    batch, adapts, keep = form_batch(keep, 8)
    assert [q.rid for q in adapts] == [2, 5, 6]
    assert [q.rid for q in batch] == [3, 7]
    assert not keep


def test_no_free_context_still_issues_ready_adapts():
    rooms = [FakeRoom(i) for i in range(2)]
    pending = collections.deque([Request(0, "adapt", rooms[0]), Request(1, "relocalise", rooms[1]),
                                 Request(2, "adapt", rooms[1]), Request(3, "relocalise", rooms[0])])
    batch, adapts, keep = form_batch(pending, 0)
    assert not batch and [q.rid for q in adapts] == [0]
    assert [q.rid for q in keep] == [1, 2, 3]


def test_admission_refuses_beyond_the_queue_bound():
    from paper_1810_12163_amd import serve
    s = serve.Server.__new__(serve.Server)          # policy-only: no device state needed
    s.pending = collections.deque()
    s.refused = []
    s.max_queue = 3
    rooms = [FakeRoom(0)]
    ok = [s.admit(Request(i, "relocalise", rooms[0]), float(i)) for i in range(5)]
    assert ok == [True, True, True, False, False]
    assert [q.rid for q in s.refused] == [3, 4] and all(q.refused for q in s.refused)
