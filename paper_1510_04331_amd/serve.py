"""Request loop for ADI reductions on one GPU.

Requests (one cube each, with its recentring shifts and parallactic angles)
arrive over time.  A request becomes resident when it is admitted: its cube is
allocated in HBM, filled, reduced in place by ``adi_reduce_batch`` and freed
once its final image is ready.  Admission works under two limits, the HBM
budget (cube bytes plus the reduction's workspace) and the number of execution
slots (HIP streams).  Whenever a slot frees up, the waiting requests at the
head of the queue that fit are admitted at once, as one batched reduction on
that slot's stream, so work that arrives while other reductions run overlaps
with them on the device (continuous batching).  Large requests, which fill
the device by themselves, run one at a time (see ``Admission``).

The scheduling policy (``Admission``) and the loop (``run``) are plain host
code; the device work sits behind an executor with three calls (``launch``,
``done``, ``release``).  ``TorchExecutor`` is the HIP one.
"""

import collections
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    """One reduction request.  ``fill(cube, stream)`` writes the cube's frames
    into the device tensor ``cube`` on ``stream`` (the upload)."""
    rid: int
    arrival: float                 # seconds on the loop's clock
    T: int
    N: int
    dx: np.ndarray
    dy: np.ndarray
    parang: np.ndarray
    fill: object = None
    admitted: float = None         # filled in by the loop
    done: float = None
    final: object = None           # final image (device tensor) once done

    @property
    def cube_bytes(self):
        return self.T * self.N * self.N * 4

    @property
    def latency(self):
        return None if self.done is None else self.done - self.arrival


class Admission:
    """Admission under an HBM budget and a slot count.

    ``group_bytes(list_of_requests)`` is the device memory a batch of requests
    holds while it runs (cubes plus workspace); ``cost(request)`` estimates its
    device time.  A request whose cost reaches ``big_cost`` is "large": large
    requests run alone in their group and one at a time, because a large
    reduction fills the device by itself and two of them sharing it would
    only finish later.  Small requests are admitted first come, first served,
    batched up to ``max_batch`` per group, and may run beside a large one; when
    the head of the queue is a large request that has to wait for another,
    small requests behind it are admitted meanwhile (backfilling).  A small
    request never overtakes a large one that could start.
    """

    def __init__(self, budget_bytes, slots, max_batch, group_bytes, cost=None, big_cost=None):
        if slots < 1 or max_batch < 1 or budget_bytes <= 0:
            raise ValueError("slots, max_batch and budget must be positive")
        self.budget = int(budget_bytes)
        self.slots = int(slots)
        self.max_batch = int(max_batch)
        self.group_bytes = group_bytes
        self.cost = cost
        self.big_cost = big_cost

    def is_big(self, req):
        return self.cost is not None and self.big_cost is not None and self.cost(req) >= self.big_cost

    def check(self, req):
        """Reject a request that could never be admitted."""
        if self.group_bytes([req]) > self.budget:
            raise ValueError("request %d needs %d bytes, above the HBM budget of %d"
                             % (req.rid, self.group_bytes([req]), self.budget))

    def admit(self, waiting, used_bytes, free_slots, big_inflight=0):
        """Take admitted groups out of ``waiting`` (a deque, arrival order).
        Returns a list of (group, bytes, is_big) triples, at most one per free
        slot."""
        out = []
        while free_slots > 0 and waiting:
            head = waiting[0]
            if self.is_big(head) and big_inflight == 0:
                nb = self.group_bytes([head])
                if used_bytes + nb > self.budget:
                    break                       # the large head waits for memory; nothing overtakes it
                waiting.popleft()
                out.append(([head], nb, True))
                used_bytes += nb
                big_inflight += 1
                free_slots -= 1
                continue
            # small requests from the front of the queue, skipping large ones
            # that must wait for the one in flight
            group, gb, picked = [], 0, []
            for i, r in enumerate(waiting):
                if len(group) >= self.max_batch:
                    break
                if self.is_big(r):
                    if big_inflight == 0:
                        break                   # a large request that could start: no overtaking
                    continue
                nb = self.group_bytes(group + [r])
                if used_bytes + nb > self.budget:
                    break
                group.append(r)
                picked.append(i)
                gb = nb
            if not group:
                break
            for i in reversed(picked):
                del waiting[i]
            out.append((group, gb, False))
            used_bytes += gb
            free_slots -= 1
        return out


@dataclass
class Stats:
    n: int = 0
    frames: int = 0
    wall_s: float = 0.0
    latencies_s: list = field(default_factory=list)
    max_inflight: int = 0
    max_used_bytes: int = 0
    groups: int = 0

    def summary(self):
        lat = np.sort(np.asarray(self.latencies_s, dtype=np.float64))

        def pct(q):
            if lat.size == 0:
                return None
            return float(lat[min(lat.size - 1, int(np.ceil(q * lat.size)) - 1)])
        return {"requests": self.n, "frames": self.frames, "wall_s": round(self.wall_s, 4),
                "frames_per_s": round(self.frames / self.wall_s, 1) if self.wall_s > 0 else None,
                "latency_ms": {"p50": None if lat.size == 0 else round(1e3 * pct(0.50), 3),
                               "p99": None if lat.size == 0 else round(1e3 * pct(0.99), 3),
                               "max": None if lat.size == 0 else round(1e3 * float(lat[-1]), 3)},
                "max_inflight_groups": self.max_inflight, "max_used_bytes": self.max_used_bytes,
                "groups": self.groups}


def run(requests, executor, admission, clock=time.perf_counter, sleep=time.sleep, poll_s=2e-4):
    """Serve ``requests`` (any order; sorted by arrival here) to completion.
    Returns Stats; every request gets ``admitted``, ``done`` and ``final``."""
    reqs = sorted(requests, key=lambda r: r.arrival)
    for r in reqs:
        admission.check(r)
    waiting = collections.deque()
    inflight = []            # (slot, group, bytes, is_big, handle)
    free = list(range(admission.slots))[::-1]
    used = 0
    big = 0
    st = Stats(n=len(reqs), frames=sum(r.T for r in reqs))
    nxt = 0
    finished = 0
    t0 = clock()
    while finished < len(reqs):
        now = clock() - t0
        progressed = False
        while nxt < len(reqs) and reqs[nxt].arrival <= now:
            waiting.append(reqs[nxt])
            nxt += 1
            progressed = True
        for item in list(inflight):
            slot, group, nb, is_big, h = item
            if executor.done(h):
                t = clock() - t0
                finals = executor.release(h)
                for r, f in zip(group, finals):
                    r.done = t
                    r.final = f
                    st.latencies_s.append(r.done - r.arrival)
                finished += len(group)
                used -= nb
                big -= int(is_big)
                free.append(slot)
                inflight.remove(item)
                progressed = True
        for group, nb, is_big in admission.admit(waiting, used, len(free), big):
            slot = free.pop()
            t = clock() - t0
            for r in group:
                r.admitted = t
            inflight.append((slot, group, nb, is_big, executor.launch(group, slot)))
            used += nb
            big += int(is_big)
            st.groups += 1
            st.max_used_bytes = max(st.max_used_bytes, used)
            progressed = True
        st.max_inflight = max(st.max_inflight, len(inflight))
        if not progressed:
            wait = poll_s
            if not inflight and not waiting and nxt < len(reqs):
                wait = max(0.0, min(reqs[nxt].arrival - (clock() - t0), 0.05))
            sleep(wait)
    st.wall_s = clock() - t0
    return st


class TorchExecutor:
    """Runs each admitted group as one in-place batched reduction on the
    slot's HIP stream (default priority), allocating the group's cubes and
    workspace from torch's caching allocator on that stream."""

    def __init__(self, device, slots):
        import torch
        from . import ops
        self.torch = torch
        self.ops = ops
        self.device = torch.device(device)
        self.streams = [torch.cuda.Stream(self.device) for _ in range(slots)]

    def group_bytes(self, group):
        """Device bytes a group holds while it runs: its cubes (rounded to the
        allocator's 2 MiB granularity) and the in-place workspace."""
        if not group:
            return 0
        cubes = sum(-(-r.cube_bytes // (2 << 20)) * (2 << 20) for r in group)
        ws = self.ops.batch_workspace_size([_Shape(r.T, r.N) for r in group], inplace=True,
                                           device_index=self.device.index or 0)
        return cubes + ws

    @staticmethod
    def cost(req):
        """Estimated device milliseconds of one reduction (about 40 ps per
        pixel of every frame on MI355X)."""
        return req.T * req.N * req.N * 4e-8

    def launch(self, group, slot):
        torch = self.torch
        s = self.streams[slot]
        with torch.cuda.stream(s):
            cubes = []
            for r in group:
                c = torch.empty((r.T, r.N, r.N), dtype=torch.float32, device=self.device)
                r.fill(c, s)
                cubes.append(c)
            finals = self.ops.adi_reduce_batch(cubes, [r.dx for r in group], [r.dy for r in group],
                                               [r.parang for r in group], inplace=True, stream=s)
            ev = torch.cuda.Event()
            ev.record(s)
        return (ev, cubes, finals)

    def done(self, h):
        return h[0].query()

    def release(self, h):
        ev, cubes, finals = h
        del cubes[:]            # the cube memory returns to the stream's pool
        return finals


class _Shape:
    """Shape-only stand-in for a cube (workspace queries need only shapes)."""

    def __init__(self, T, N):
        self.shape = (T, N, N)
