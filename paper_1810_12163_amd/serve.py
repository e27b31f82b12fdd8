"""Continuous-batching relocalisation server over many resident rooms.

Every room's forest, reservoirs and modes stay resident in device memory.
Requests (relocalise or adapt, any room, any resolution) arrive over time;
the server

* admits them into a bounded queue (refusing when it is full),
* keeps up to ``contexts`` batches in flight at once, each on its own stream
  with its own workspace, their number capped by the device-memory budget,
* whenever a context is free, forms a batch from the pending relocalise
  requests (up to ``max_batch``) and submits it asynchronously, so requests
  that arrive while other batches run overlap with them on the device,
* serves each room's requests in arrival order: a relocalisation sees exactly
  the adaptations of its room that arrived before it.  An adapt is queued on
  its room's stream only once every earlier request of that room has been
  submitted; the library orders a room's batches and adaptations on the
  device with stream events,
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
    arrival: float = 0.0
    submitted: float = 0.0
    done: float = 0.0
    result: dict | None = None
    refused: bool = False


def form_batch(pending, max_batch):
    """Scheduling policy (pure).  Walks the pending requests in arrival order.

    Returns (batch, adapts, keep):
    * ``batch``: relocalisations to submit now (at most max_batch), none of
      them behind a pending adapt of its room;
    * ``adapts``: adaptations to issue now, in arrival order, none of them
      behind a pending or batched relocalisation of its room;
    * ``keep``: everything else, still in arrival order.
    Adaptations are issued before the batch is submitted, which is the
    arrival order for every room involved."""
    blocked, in_batch = set(), set()
    batch, adapts, keep = [], [], collections.deque()
    for q in pending:
        r = id(q.room)
        if q.kind == "adapt":
            if r in blocked or r in in_batch:
                blocked.add(r)
                keep.append(q)
            else:
                adapts.append(q)
        else:
            if r in blocked or len(batch) >= max_batch:
                blocked.add(r)
                keep.append(q)
            else:
                batch.append(q)
                in_batch.add(r)
    return batch, adapts, keep


class Server:
    def __init__(self, max_batch=64, max_width=640, max_height=480, max_hypotheses=1024, max_eta=500,
                 max_rounds=10, n_trees=5, max_modes_per_pixel=50, contexts=2, memory_budget=None,
                 max_queue=4096, device=None, use_graph=True):
        import torch

        from . import Batch, Result
        self.torch = torch
        self._Result = Result
        self.device = torch.device(device if device is not None else "cuda")
        args = (max_batch, max_width, max_height, max_hypotheses, max_eta, max_rounds, n_trees,
                max_modes_per_pixel)
        self.per_context_bytes = batch_workspace_bytes(*args)
        if memory_budget is not None:
            contexts = max(1, min(contexts, int(memory_budget // self.per_context_bytes)))
        self.ctx = [Batch(*args, device=self.device) for _ in range(contexts)]
        self.busy = [None] * contexts          # (requests, host buffer, event)
        self.max_batch = max_batch
        self.max_queue = max_queue
        self.use_graph = use_graph
        self.pending = collections.deque()
        self.completed = []
        self.refused = []
        self.batch_sizes = []
        rs = ctypes.sizeof(Result)
        self._res = [torch.empty(max_batch * rs, dtype=torch.uint8, device=self.device) for _ in range(contexts)]
        self._host = [torch.empty(max_batch * rs, dtype=torch.uint8, pin_memory=True) for _ in range(contexts)]

    def admit(self, req: Request, now: float) -> bool:
        req.arrival = now
        if len(self.pending) >= self.max_queue:
            req.refused = True
            self.refused.append(req)
            return False
        self.pending.append(req)
        return True

    def poll(self, now_fn=time.perf_counter) -> int:
        """Completes finished batches, issues ready adaptations and fills every
        free context with a new batch.  Returns the number of completions."""
        from . import _result
        done = 0
        rs = ctypes.sizeof(self._Result)
        for i, b in enumerate(self.busy):
            if b is not None and b[2].query():
                reqs, host, _ = b
                t = now_fn()
                raw = host.numpy()
                for k, q in enumerate(reqs):
                    q.result = _result(self._Result.from_buffer_copy(raw[k * rs:(k + 1) * rs].tobytes()))
                    q.done = t
                    self.completed.append(q)
                done += len(reqs)
                self.busy[i] = None
        while True:
            free = [i for i, b in enumerate(self.busy) if b is None]
            batch, adapts, keep = form_batch(self.pending, self.max_batch if free else 0)
            self.pending = keep
            t = now_fn()
            for q in adapts:
                q.submitted = t
                q.room.adapt(q.depth, q.rgb, q.K, q.pose)
                q.done = t                    # queued on the device, ordered before later requests
                q.result = {"status": "adapted"}
                self.completed.append(q)
            if not batch:
                break
            self._submit(free[0], batch, t)
            if len(free) == 1:
                break
        return done

    def _submit(self, i, reqs, t):
        torch = self.torch
        for q in reqs:
            q.submitted = t
        b = self.ctx[i]
        items = [(q.room, q.depth, q.rgb, q.K, q.rid, q.n_hypotheses) for q in reqs]
        b.relocalise_async(items, self._res[i], use_graph=self.use_graph)
        nbytes = len(reqs) * ctypes.sizeof(self._Result)
        with torch.cuda.stream(b.stream):
            self._host[i][:nbytes].copy_(self._res[i][:nbytes], non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(b.stream)
        self.busy[i] = (reqs, self._host[i], ev)
        self.batch_sizes.append(len(reqs))

    def idle(self) -> bool:
        return not self.pending and all(b is None for b in self.busy)

    def drain(self, now_fn=time.perf_counter):
        while not self.idle():
            self.poll(now_fn)

    def close(self):
        for b in self.ctx:
            b.close()


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
                batches=len(server.batch_sizes),
                mean_batch=float(np.mean(server.batch_sizes)) if server.batch_sizes else 0.0,
                wall_s=now())
