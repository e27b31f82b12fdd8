"""Continuous-batching relocalisation server over many resident rooms.

Every room's forest, reservoirs and modes stay resident in device memory.
Requests (relocalise or adapt, any room, any resolution) arrive over time;
the server

* admits them by device-memory budget: every resident room, every batch
  context and a pool of frame slots are charged against one HBM budget
  (rooms that do not fit are refused); a request whose frame comes from the
  host is copied into a free frame slot, and waits in an arrival-order
  backlog while every slot is taken (refused only when the queue is full),
* keeps up to ``contexts`` batches in flight at once, each on its own stream
  with its own workspace, their number capped by the device-memory budget,
* whenever a context is free, forms a batch from the pending requests
  (relocalisations and adaptations, up to ``max_batch``) and submits it
  asynchronously, so requests that arrive while other batches run overlap
  with them on the device,
* serves each room's requests in arrival order: a relocalisation sees exactly
  the adaptations of its room that arrived before it.  A batch runs its
  relocalisations before its adaptations, so a relocalisation never joins a
  batch that already holds an adaptation of its room; the library orders a
  room's batches and adaptations on the device with stream events,
* records per-request latency (completion observed by the host minus arrival).

Results depend only on (room state, frame, request seed), so a request gives
the same result alone and in any mix.
"""
from __future__ import annotations

import collections
import ctypes
import dataclasses
import time

import numpy as np

from . import AdaptRequest


@dataclasses.dataclass
class Request:
    rid: int
    kind: str                 # "relocalise" or "adapt"
    room: object              # paper_1810_12163_amd.Room
    depth: object = None      # torch CUDA tensor (h, w) float32
    rgb: object = None        # torch CUDA tensor (h, w, 3) uint8
    K: tuple = ()
    pose: np.ndarray | None = None       # adapt only
    n_hypotheses: int = 0
    host_depth: object = None  # frame on the host (pinned torch CPU tensors), copied into a frame slot
    host_rgb: object = None
    host_frame: object = None  # or both in one pinned uint8 tensor: h*w*4 depth bytes, then h*w*3 colour
    frame_hw: tuple = ()       # (h, w) of host_frame
    slot: int = -1
    deferred: bool = False     # waited in the backlog for a frame slot
    arrival: float = 0.0
    submitted: float = 0.0
    done: float = 0.0
    result: dict | None = None
    refused: bool = False


def form_batch(pending, max_batch):
    """Scheduling policy (pure).  Walks the pending requests in arrival order.

    Returns (batch, keep):
    * ``batch``: requests to submit now as one batch (at most max_batch),
      in arrival order.  The library runs a batch's relocalisations first and
      its adaptations after them, so a relocalisation may join the batch only
      if no adaptation of its room is already in it (it must see that
      adaptation), and nothing may pass a request of its room left waiting;
    * ``keep``: everything else, still in arrival order."""
    blocked, adapted = set(), set()
    batch, keep = [], collections.deque()
    for q in pending:
        r = id(q.room)
        if len(batch) >= max_batch or r in blocked or (q.kind != "adapt" and r in adapted):
            blocked.add(r)
            keep.append(q)
            continue
        batch.append(q)
        if q.kind == "adapt":
            adapted.add(r)
    return batch, keep


class Ledger:
    """Device-memory budget of a server in bytes (None = unlimited): resident
    rooms, batch contexts and the frame pool are charged against it."""

    def __init__(self, budget=None):
        self.budget = budget
        self.items = {}

    @property
    def used(self) -> int:
        return sum(self.items.values())

    def fits(self, nbytes: int) -> bool:
        return self.budget is None or self.used + nbytes <= self.budget

    def charge(self, key, nbytes: int) -> bool:
        if not self.fits(nbytes):
            return False
        self.items[key] = self.items.get(key, 0) + int(nbytes)
        return True

    def release(self, key):
        self.items.pop(key, None)


class FramePool:
    """Fixed-size frame slots in device memory, each holding the depth and
    colour of the largest frame (depth bytes, then colour bytes); a request's
    frame is copied into a slot and the slot is returned once the request's
    device work has completed."""

    def __init__(self, n_slots, max_width, max_height, device):
        import torch
        self.max_px = max_width * max_height
        self.buf = torch.empty((n_slots, self.max_px * 7), dtype=torch.uint8, device=device)
        self.free = list(range(n_slots - 1, -1, -1))
        self.n_slots = n_slots

    @staticmethod
    def slot_bytes(max_width, max_height) -> int:
        return max_width * max_height * (4 + 3)

    def take(self) -> int:
        return self.free.pop() if self.free else -1

    def give(self, slot: int):
        self.free.append(slot)

    def views(self, slot, h, w):
        import torch
        b = self.buf[slot]
        return b[:4 * h * w].view(torch.float32).view(h, w), b[4 * h * w:7 * h * w].view(h, w, 3)


def pack_host_frame(depth, rgb):
    """One pinned host buffer holding a frame as a frame slot does (depth
    bytes, then colour bytes): one copy per request instead of two."""
    import torch
    d = np.ascontiguousarray(depth, dtype=np.float32)
    c = np.ascontiguousarray(rgb, dtype=np.uint8)
    out = torch.empty(d.nbytes + c.nbytes, dtype=torch.uint8, pin_memory=True)
    out[:d.nbytes].copy_(torch.from_numpy(d.view(np.uint8).reshape(-1)))
    out[d.nbytes:].copy_(torch.from_numpy(c.reshape(-1)))
    return out, d.shape


class Server:
    def __init__(self, max_batch=64, max_width=640, max_height=480, max_hypotheses=1024, max_eta=500,
                 max_rounds=10, n_trees=5, max_modes_per_pixel=50, contexts=2, memory_budget=None,
                 frame_slots=0, max_queue=4096, device=None, use_graph=True):
        """memory_budget: device bytes for the rooms this server creates
        (create_room), its batch contexts and its frame pool (None =
        unlimited).  Contexts beyond the budget are dropped (at least one
        must fit).  frame_slots (0 = none, for requests whose frames already
        live on the device): the pool is created when the first request with
        a host frame arrives, cut to what the budget leaves after the rooms
        created so far; rooms created later are charged against the rest."""
        import torch

        from . import Batch, Result
        self.torch = torch
        self._Result = Result
        self.device = torch.device(device if device is not None else "cuda")
        self.max_width, self.max_height = max_width, max_height
        args = (max_batch, max_width, max_height, max_hypotheses, max_eta, max_rounds, n_trees,
                max_modes_per_pixel)
        self.ledger = Ledger(memory_budget)
        self.per_context_bytes = batch_workspace_bytes(*args)
        n_ctx = 0
        for i in range(contexts):
            if not self.ledger.charge(("context", i), self.per_context_bytes):
                break
            n_ctx += 1
        if n_ctx == 0:
            raise ValueError("the memory budget does not hold one batch context")
        self.ctx = [Batch(*args, device=self.device) for _ in range(n_ctx)]
        self.frame_slots = frame_slots
        self.pool = None                     # created at the first host frame, from what the budget leaves
        self.busy = [None] * n_ctx          # (requests, host buffer, event)
        self.max_batch = max_batch
        self.max_queue = max_queue
        self.use_graph = use_graph
        self.pending = collections.deque()
        self.backlog = collections.deque()   # admitted, waiting for a frame slot
        self.completed = []
        self.refused = []
        self.deferred = 0
        self.max_backlog = 0
        self.batch_sizes = []
        self.rooms = []
        self.host_s = collections.Counter()   # host seconds per phase of the loop
        rs = ctypes.sizeof(Result)
        self._res = [torch.empty(max_batch * rs, dtype=torch.uint8, device=self.device) for _ in range(n_ctx)]
        self._host = [torch.empty(max_batch * rs, dtype=torch.uint8, pin_memory=True) for _ in range(n_ctx)]

    # ---- rooms ----------------------------------------------------------------
    def create_room(self, params: dict, nodes, max_width=None, max_height=None):
        """Creates a resident room if its device state fits the memory budget
        (returns None otherwise)."""
        from . import Room, room_state_bytes
        mw, mh = max_width or self.max_width, max_height or self.max_height
        nb = sum(room_state_bytes(params, mw, mh))
        key = ("room", len(self.rooms))
        if not self.ledger.charge(key, nb):
            return None
        room = Room(params, nodes, mw, mh, device=self.device)
        self.rooms.append(room)
        return room

    # ---- admission ------------------------------------------------------------
    def admit(self, req: Request, now: float) -> bool:
        req.arrival = now
        if len(self.pending) + len(self.backlog) >= self.max_queue:
            req.refused = True
            self.refused.append(req)
            return False
        if req.host_depth is None and req.host_frame is None:
            self.pending.append(req)
            return True
        if self.pool is None:
            self._open_pool()
        t0 = time.perf_counter()
        staged = not self.backlog and self._stage(req)
        self.host_s["admit"] += time.perf_counter() - t0
        if staged:
            self.pending.append(req)
        else:
            req.deferred = True
            self.deferred += 1
            self.backlog.append(req)
            self.max_backlog = max(self.max_backlog, len(self.backlog))
        return True

    def _open_pool(self):
        sb = FramePool.slot_bytes(self.max_width, self.max_height)
        n = self.frame_slots
        if self.ledger.budget is not None:
            n = min(n, max(0, (self.ledger.budget - self.ledger.used) // sb))
        if n <= 0:
            raise ValueError("no frame slot fits the memory budget (frame_slots > 0 needed for host frames)")
        self.ledger.charge("frame_pool", n * sb)
        self.pool = FramePool(n, self.max_width, self.max_height, self.device)

    def _stage(self, req) -> bool:
        """Copies the request's host frame into a free slot (queued on the
        current stream, which batches and rooms wait for)."""
        slot = self.pool.take()
        if slot < 0:
            return False
        if req.host_frame is not None:
            h, w = req.frame_hw
            self.pool.buf[slot, :7 * h * w].copy_(req.host_frame, non_blocking=True)
            d, c = self.pool.views(slot, h, w)
        else:
            h, w = req.host_depth.shape
            d, c = self.pool.views(slot, h, w)
            d.copy_(req.host_depth, non_blocking=True)
            c.copy_(req.host_rgb, non_blocking=True)
        req.depth, req.rgb, req.slot = d, c, slot
        return True

    def _refill(self):
        """Moves waiting requests, in arrival order, into free frame slots."""
        while self.backlog and self._stage(self.backlog[0]):
            self.pending.append(self.backlog.popleft())

    def _release(self, req):
        if req.slot >= 0:
            self.pool.give(req.slot)
            req.slot = -1

    def poll(self, now_fn=time.perf_counter) -> int:
        """Completes finished batches, returns their frame slots, moves waiting
        requests into free slots, issues ready adaptations and fills every
        free context with a new batch.  Returns the number of completions."""
        from . import decode_results
        done = 0
        tp = time.perf_counter()
        for i, b in enumerate(self.busy):
            if b is not None and b[2].query():
                reqs, host, _ = b
                t = now_fn()
                for q, r in zip(reqs, decode_results(host.numpy(), len(reqs))):
                    q.result = r
                    q.done = t
                    self._release(q)
                    self.completed.append(q)
                done += len(reqs)
                self.busy[i] = None
        self._refill()
        self.host_s["complete"] += time.perf_counter() - tp
        while True:
            free = [i for i, b in enumerate(self.busy) if b is None]
            if not free or not self.pending:
                break
            tf = time.perf_counter()
            batch, keep = form_batch(self.pending, self.max_batch)
            self.pending = keep
            t1 = time.perf_counter()
            self.host_s["form"] += t1 - tf
            if not batch:
                break
            self._submit(free[0], batch, now_fn())
            self.host_s["submit"] += time.perf_counter() - t1
        return done

    def _submit(self, i, reqs, t):
        torch = self.torch
        for q in reqs:
            q.submitted = t
        b = self.ctx[i]
        items = [AdaptRequest(q.room, q.depth, q.rgb, q.K, q.pose) if q.kind == "adapt" else
                 (q.room, q.depth, q.rgb, q.K, q.rid, q.n_hypotheses) for q in reqs]
        # frames in the server's slots stay put until the batch has completed
        b.relocalise_async(items, self._res[i], use_graph=self.use_graph, record=any(q.slot < 0 for q in reqs))
        nbytes = len(reqs) * ctypes.sizeof(self._Result)
        with torch.cuda.stream(b.stream):
            self._host[i][:nbytes].copy_(self._res[i][:nbytes], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(b.stream)
        self.busy[i] = (reqs, self._host[i], ev)
        self.batch_sizes.append(len(reqs))

    def reset_stats(self):
        """Forgets completed requests and counters (between measurement windows)."""
        self.completed, self.refused, self.batch_sizes = [], [], []
        self.host_s = collections.Counter()
        self.deferred, self.max_backlog = 0, 0

    def idle(self) -> bool:
        return not self.pending and not self.backlog and all(b is None for b in self.busy)

    def drain(self, now_fn=time.perf_counter):
        while not self.idle():
            self.poll(now_fn)

    def close(self):
        self.drain()
        for b in self.ctx:
            b.close()
        for r in self.rooms:
            r.close()


def batch_workspace_bytes(max_frames, max_width, max_height, max_hypotheses, max_eta, max_rounds,
                          n_trees, max_modes_per_pixel) -> int:
    from . import BatchParams, lib
    bp = BatchParams(max_frames, max_width, max_height, max_hypotheses, max_eta, max_rounds, n_trees,
                     max_modes_per_pixel)
    nb = ctypes.c_size_t()
    if lib().rl_batch_workspace_bytes(ctypes.byref(bp), ctypes.byref(nb)) != 0:
        raise ValueError(lib().rl_last_error().decode())
    return int(nb.value)


def poisson_arrivals(rate: float, duration: float, seed: int) -> np.ndarray:
    """Arrival times (s) of a Poisson process of the given rate."""
    rng = np.random.default_rng(seed)
    n = int(rate * duration * 1.5) + 16
    t = np.cumsum(rng.exponential(1.0 / rate, size=n))
    return t[t < duration]


def run_open_loop(server: Server, requests: list, arrivals, warmup_s: float = 0.0) -> dict:
    """Feeds requests at their arrival times (seconds from start) and runs the
    scheduling loop until all are done.  Statistics cover the relocalisations
    that arrived after ``warmup_s``."""
    t0 = time.perf_counter()
    now = lambda: time.perf_counter() - t0   # noqa: E731
    k, n = 0, len(requests)
    while k < n or not server.idle():
        tnow = now()
        while k < n and arrivals[k] <= tnow:
            server.admit(requests[k], float(arrivals[k]))
            k += 1
        server.poll(now)
        if k < n and server.idle():
            wait = arrivals[k] - now()
            if wait > 0:
                time.sleep(min(wait, 0.0002))
    rel = [q for q in server.completed if q.kind == "relocalise" and q.arrival >= warmup_s]
    lat = np.array([q.done - q.arrival for q in rel]) if rel else np.zeros(1)
    span = (max(q.done for q in rel) - warmup_s) if rel else 1.0
    return dict(relocs_per_s=len(rel) / max(span, 1e-9), p50_ms=float(np.percentile(lat, 50) * 1e3),
                p99_ms=float(np.percentile(lat, 99) * 1e3), n=len(rel), refused=len(server.refused),
                deferred=server.deferred, max_backlog=server.max_backlog,
                host_s={k: round(v, 4) for k, v in getattr(server, "host_s", {}).items()},
                batches=len(server.batch_sizes),
                mean_batch=float(np.mean(server.batch_sizes)) if server.batch_sizes else 0.0,
                offered=n, wall_s=now())
