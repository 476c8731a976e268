"""Serving loop over resident rollouts with continuous batching.

A rollout is one driving scene resident on the GPU (its sim workspace and
its image buffer live in one block of a device arena).  A request to a
rollout carries one action per agent; serving it means one kinematic step of
the rollout followed by a render of every agent's view.  The paper has no
serving loop; this is the batched-environment pattern of App. A
("High-Throughput Batched Rendering") turned into a request loop:

* admission by HBM footprint: a rollout is admitted when its footprint fits
  in the arena (first fit, coalescing free list); otherwise it waits, in
  arrival order, until enough memory is freed;
* requests to one rollout are served in arrival order, at most one in flight
  (the next request of a rollout overwrites its images);
* continuous batching: whenever an execution slot (a stream) is free, every
  rollout with a pending request and nothing in flight joins one batch, which
  runs as one batched step + render launch on that slot's stream;
* latency runs from a request's arrival to the completion of its batch.

The scheduler is host logic and runs against an executor: `GpuExecutor`
drives the HIP library through gp.batch_step_render; tests drive the same
scheduler with a CPU executor under a virtual clock.
"""
from __future__ import annotations

import bisect
import collections
import dataclasses
import math
from typing import Callable, Deque, Dict, List, Optional, Sequence, Tuple

import numpy as np

ALIGN = 256


# ------------------------------------------------------------------ arena

class Arena:
    """First-fit allocator over [0, capacity) in ALIGN-byte units; adjacent
    free blocks are merged on free."""

    def __init__(self, capacity: int, align: int = ALIGN):
        self.align = align
        self.capacity = capacity // align * align
        self._free: List[Tuple[int, int]] = [(0, self.capacity)] if self.capacity else []   # sorted (off, size)
        self._used: Dict[int, int] = {}

    def _round(self, n: int) -> int:
        return max(self.align, (n + self.align - 1) // self.align * self.align)

    def alloc(self, nbytes: int) -> Optional[int]:
        need = self._round(nbytes)
        for i, (off, size) in enumerate(self._free):
            if size >= need:
                if size == need:
                    del self._free[i]
                else:
                    self._free[i] = (off + need, size - need)
                self._used[off] = need
                return off
        return None

    def free(self, off: int):
        size = self._used.pop(off)
        i = bisect.bisect_left(self._free, (off, 0))
        self._free.insert(i, (off, size))
        # merge with the right, then the left neighbour
        if i + 1 < len(self._free) and off + size == self._free[i + 1][0]:
            self._free[i] = (off, size + self._free[i + 1][1])
            del self._free[i + 1]
        if i > 0 and self._free[i - 1][0] + self._free[i - 1][1] == off:
            po, ps = self._free[i - 1]
            self._free[i - 1] = (po, ps + self._free[i][1])
            del self._free[i]

    @property
    def used_bytes(self) -> int:
        return sum(self._used.values())

    @property
    def free_bytes(self) -> int:
        return self.capacity - self.used_bytes

    def largest_free(self) -> int:
        return max((s for _, s in self._free), default=0)


# ------------------------------------------------------------------ requests and rollouts

OK, REJECTED, CANCELLED = "ok", "rejected", "cancelled"


@dataclasses.dataclass
class Request:
    rid: int
    rollout: int
    actions: np.ndarray
    t_arrival: float
    t_done: Optional[float] = None
    status: Optional[str] = None
    batch: Optional[int] = None


@dataclasses.dataclass
class Rollout:
    id: int
    scene: object
    n_agents: int
    n_views: int
    footprint: int
    offset: Optional[int] = None
    handle: object = None
    pending: Deque[Request] = dataclasses.field(default_factory=collections.deque)
    inflight: Optional[Request] = None
    closing: bool = False
    served: int = 0


class ServeError(ValueError):
    pass


# ------------------------------------------------------------------ scheduler

class Server:
    """Admission, per-rollout FIFO queues and continuous batching over the
    executor's slots.  Single-threaded: the caller drives it with pump(now)."""

    def __init__(self, executor, budget_bytes: int, max_batch_rollouts: int = 256,
                 on_complete: Optional[Callable[[Request, Rollout], None]] = None):
        self.ex = executor
        self.arena = Arena(budget_bytes)
        self.max_batch = max_batch_rollouts
        self.on_complete = on_complete
        self.rollouts: Dict[int, Rollout] = {}
        self.waiting: Deque[Rollout] = collections.deque()   # not yet admitted
        self.done: List[Request] = []
        self.batches: Dict[int, Tuple[List[Rollout], List[Request]]] = {}
        self.batch_sizes: List[int] = []
        self._ready: Dict[int, Rollout] = {}      # admitted, a request pending, none in flight
        self._next_rollout = 0
        self._next_request = 0
        self._next_batch = 0

    # -- rollouts
    def open(self, scene) -> int:
        """Register a rollout; it is admitted now if its footprint fits, else
        it waits for memory.  A rollout larger than the whole arena is refused."""
        fp = int(self.ex.footprint(scene))
        if fp > self.arena.capacity:
            raise ServeError(f"rollout footprint {fp} exceeds the arena ({self.arena.capacity} bytes)")
        cap = getattr(self.ex, "max_batch_agents", None)
        if cap is not None and scene.agent_state.shape[0] > cap:
            raise ServeError(f"rollout of {scene.agent_state.shape[0]} agents exceeds the executor's batch "
                             f"({cap} agents)")
        r = Rollout(self._next_rollout, scene, int(scene.agent_state.shape[0]),
                    int(scene.agent_state.shape[0]) * self.ex.n_cams, fp)
        self._next_rollout += 1
        self.rollouts[r.id] = r
        self.waiting.append(r)
        self._admit()
        return r.id

    def admitted(self, rid: int) -> bool:
        return self.rollouts[rid].handle is not None

    def close(self, rid: int):
        """Close after the pending requests are served."""
        r = self.rollouts[rid]
        r.closing = True
        self._maybe_release(r)

    def cancel(self, rid: int):
        """Drop the pending requests (status 'cancelled') and close."""
        r = self.rollouts[rid]
        while r.pending:
            q = r.pending.popleft()
            q.status = CANCELLED
            self.done.append(q)
        self._mark(r)
        self.close(rid)

    def _admit(self):
        while self.waiting:
            r = self.waiting[0]
            off = self.arena.alloc(r.footprint)
            if off is None:
                return
            self.waiting.popleft()
            r.offset = off
            r.handle = self.ex.create(r.scene, off, r.footprint)
            self._mark(r)

    def _mark(self, r: Rollout):
        if r.handle is not None and r.inflight is None and r.pending:
            self._ready[r.id] = r
        else:
            self._ready.pop(r.id, None)

    def _maybe_release(self, r: Rollout):
        if r.closing and not r.pending and r.inflight is None:
            if r.handle is not None:
                self.ex.destroy(r.handle)
                self.arena.free(r.offset)
                r.handle = None
            elif r in self.waiting:
                self.waiting.remove(r)
            del self.rollouts[r.id]
            self._admit()

    # -- requests
    def submit(self, rid: int, actions, now: float) -> Request:
        """Queue one request; an invalid one is returned with status 'rejected'
        and leaves every other request untouched."""
        q = Request(self._next_request, rid, None, now)
        self._next_request += 1
        r = self.rollouts.get(rid)
        a = np.asarray(actions, dtype=np.float32) if actions is not None else None
        if r is None or r.closing:
            q.status = REJECTED
        elif a is None or a.shape != (r.n_agents, 2) or not np.all(np.isfinite(a)):
            q.status = REJECTED
        if q.status == REJECTED:
            q.t_done = now
            self.done.append(q)
            return q
        q.actions = np.ascontiguousarray(a)
        r.pending.append(q)
        self._mark(r)
        return q

    # -- the loop
    def pump(self, now: float) -> int:
        """Retire finished batches, admit waiting rollouts, launch batches while
        slots are free.  Returns the number of batches launched."""
        for token, t_done in self.ex.poll(now):
            rolls, reqs = self.batches.pop(token)
            for r, q in zip(rolls, reqs):
                q.t_done = t_done
                q.status = OK
                r.inflight = None
                r.served += 1
                self.done.append(q)
                if self.on_complete:
                    self.on_complete(q, r)
                self._mark(r)
                self._maybe_release(r)
        self._admit()
        launched = 0
        while self.ex.free_slots() > 0:
            if not self._ready:
                break
            # oldest first, as many rollouts as the executor's batch holds
            cap = getattr(self.ex, "max_batch_agents", None)
            ready, agents = [], 0
            for r in sorted(self._ready.values(), key=lambda r: r.pending[0].t_arrival):
                if len(ready) == self.max_batch:
                    break
                if cap is not None and agents + r.n_agents > cap:
                    continue        # waits for the next batch (open() made sure it fits alone)
                ready.append(r)
                agents += r.n_agents
            reqs = [r.pending.popleft() for r in ready]
            for r in ready:
                del self._ready[r.id]
            token = self._next_batch
            self._next_batch += 1
            for r, q in zip(ready, reqs):
                r.inflight = q
                q.batch = token
            self.batches[token] = (ready, reqs)
            try:
                self.ex.launch(token, [r.handle for r in ready], [q.actions for q in reqs], now)
            except Exception:
                # nothing was queued: put the requests back at the head of
                # their rollouts' queues and leave the server as it was
                del self.batches[token]
                for r, q in zip(ready, reqs):
                    r.inflight = None
                    q.batch = None
                    r.pending.appendleft(q)
                    self._mark(r)
                raise
            self.batch_sizes.append(len(ready))
            launched += 1
        return launched

    def idle(self) -> bool:
        return not self.batches and not any(r.pending for r in self.rollouts.values())

    # -- statistics
    def latencies(self, t0: float = -math.inf) -> np.ndarray:
        return np.array([q.t_done - q.t_arrival for q in self.done if q.status == OK and q.t_arrival >= t0])

    def summary(self, t0: float, t1: float) -> dict:
        lat = self.latencies(t0)
        ok = [q for q in self.done if q.status == OK and t0 <= q.t_arrival]
        views = sum(self.ex.n_cams * q.actions.shape[0] for q in ok)
        span = max(t1 - t0, 1e-9)
        return {
            "completed": len(ok),
            "completed_per_s": len(ok) / span,
            "views_per_s": views / span,
            "p50_ms": float(np.percentile(lat, 50) * 1e3) if lat.size else None,
            "p99_ms": float(np.percentile(lat, 99) * 1e3) if lat.size else None,
            "mean_batch_rollouts": float(np.mean(self.batch_sizes)) if self.batch_sizes else 0.0,
            "rejected": sum(1 for q in self.done if q.status == REJECTED),
        }


# ------------------------------------------------------------------ executors

class GpuExecutor:
    """Rollouts in one device arena; batches on `n_streams` streams, each with
    its own pinned staging buffer and device batch buffer."""

    def __init__(self, camera, palette, budget_bytes: int, n_streams: int = 4, max_batch_agents: int = 65536,
                 max_batch_rollouts: int = 256, launch: Optional[dict] = None, device: str = "cuda:0"):
        import torch
        from . import gp
        self.gp, self.torch = gp, torch
        self.camera, self.palette = camera, palette
        self.n_cams = len(camera.cam_dirs)
        self.device = torch.device(device)
        self.launch_cfg = launch
        self.arena = torch.empty(budget_bytes, dtype=torch.uint8, device=self.device)
        self.img_bytes = camera.width * camera.height * 3
        nb = gp.lib().gp_batch_required_bytes(max_batch_rollouts, max_batch_agents,
                                              max_batch_agents * self.n_cams)
        self.slots = []
        for _ in range(n_streams):
            self.slots.append({
                "stream": torch.cuda.Stream(device=self.device),
                "ws": torch.empty(nb, dtype=torch.uint8, device=self.device),
                "staging": torch.empty(nb, dtype=torch.uint8, pin_memory=True),
                "event": None, "token": None,
            })
        self.max_batch_agents = max_batch_agents
        # optional event pair around every batch (device_spans), for checking
        # that batches of different streams overlapped on the device
        self.record_spans = False
        self.spans = []
        # Creating a sim uploads its scene and waits for that upload.  On a
        # stream of its own (non-blocking, like every torch stream) the wait
        # covers the upload only, not the batches queued on the slots' streams
        # (the legacy default stream would wait for all of them).  A rollout's
        # arena block is reused only after its last batch completed.
        self.upload_stream = torch.cuda.Stream(device=self.device)

    def footprint(self, scene) -> int:
        ws = self.gp.required_bytes([scene], self.camera, self.palette)
        n_views = scene.agent_state.shape[0] * self.n_cams
        return (ws + ALIGN - 1) // ALIGN * ALIGN + n_views * self.img_bytes

    def create(self, scene, offset: int, footprint: int):
        ws_bytes = self.gp.required_bytes([scene], self.camera, self.palette)
        ws_end = offset + (ws_bytes + ALIGN - 1) // ALIGN * ALIGN
        n_views = scene.agent_state.shape[0] * self.n_cams
        sim = self.gp.Sim([scene], self.camera, self.palette, device=str(self.device),
                          workspace=self.arena[offset:offset + ws_bytes], stream=self.upload_stream)
        if self.launch_cfg:
            sim.set_launch(**self.launch_cfg)
        rgb = self.arena[ws_end:ws_end + n_views * self.img_bytes].view(
            n_views, self.camera.height, self.camera.width, 3)
        return {"sim": sim, "rgb": rgb}

    def destroy(self, handle):
        handle["sim"].close()

    def free_slots(self) -> int:
        return sum(1 for s in self.slots if s["token"] is None)

    def launch(self, token, handles, actions, now):
        slot = next(s for s in self.slots if s["token"] is None)
        sims = [h["sim"] for h in handles]
        if sum(x.n_agents for x in sims) > self.max_batch_agents:
            raise ServeError("batch larger than the executor's batch buffer")
        with self.torch.cuda.stream(slot["stream"]):
            t0 = None
            if self.record_spans:
                t0 = self.torch.cuda.Event(enable_timing=True)
                t0.record(slot["stream"])
            self.gp.batch_step_render(sims, actions, [h["rgb"] for h in handles], slot["ws"],
                                      slot["staging"], stream=slot["stream"])
            ev = self.torch.cuda.Event(enable_timing=self.record_spans)
            ev.record(slot["stream"])
        if self.record_spans:
            self.spans.append((t0, ev))
        slot["event"], slot["token"] = ev, token

    def device_spans(self):
        """(start, end) in ms of every recorded batch on the device, relative
        to the first batch's start (needs record_spans; synchronises)."""
        self.torch.cuda.synchronize()
        if not self.spans:
            return []
        base = self.spans[0][0]
        return [(base.elapsed_time(a), base.elapsed_time(b)) for a, b in self.spans]

    def poll(self, now):
        out = []
        for s in self.slots:
            if s["token"] is not None and s["event"].query():
                out.append((s["token"], now))
                s["token"] = None
        return out


class VirtualExecutor:
    """CPU executor for tests: a batch of V views finishes `base + per_view * V`
    seconds after launch on a virtual clock, using `n_slots` slots; the step
    and render are delegated to `run(handle, actions)` (e.g. the oracle)."""

    def __init__(self, n_cams: int = 1, n_slots: int = 2, base: float = 1e-4, per_view: float = 1e-6,
                 footprint_fn: Optional[Callable] = None, run: Optional[Callable] = None,
                 max_batch_agents: Optional[int] = None):
        self.n_cams = n_cams
        self.max_batch_agents = max_batch_agents
        self.n_slots = n_slots
        self.base, self.per_view = base, per_view
        self.footprint_fn = footprint_fn or (lambda sc: 4096 + 64 * sc.agent_state.shape[0] + 32 * sc.road_xy.shape[0])
        self.run = run
        self.busy: Dict[int, float] = {}
        self.created = 0
        self.live = set()

    def footprint(self, scene) -> int:
        return int(self.footprint_fn(scene))

    def create(self, scene, offset, footprint):
        h = {"scene": scene, "offset": offset, "id": self.created}
        self.created += 1
        self.live.add(h["id"])
        return h

    def destroy(self, handle):
        self.live.discard(handle["id"])

    def free_slots(self) -> int:
        return self.n_slots - len(self.busy)

    def launch(self, token, handles, actions, now):
        if self.max_batch_agents is not None and sum(a.shape[0] for a in actions) > self.max_batch_agents:
            raise ServeError("batch larger than the executor's batch buffer")
        views = sum(a.shape[0] * self.n_cams for a in actions)
        self.busy[token] = now + self.base + self.per_view * views
        if self.run:
            for h, a in zip(handles, actions):
                self.run(h, a)

    def poll(self, now):
        out = [(t, d) for t, d in self.busy.items() if d <= now]
        for t, _ in out:
            del self.busy[t]
        return sorted(out, key=lambda x: x[1])


# ------------------------------------------------------------------ Poisson load

def poisson_arrivals(rate: float, duration: float, seed: int) -> np.ndarray:
    """Arrival times of a Poisson process of `rate` per second on [0, duration)."""
    rng = np.random.default_rng(seed)
    n = int(rate * duration * 1.2) + 16
    t = np.cumsum(rng.exponential(1.0 / rate, size=n))
    while t[-1] < duration:
        t = np.concatenate([t, t[-1] + np.cumsum(rng.exponential(1.0 / rate, size=n))])
    return t[t < duration]


def drive(server: Server, arrivals: Sequence[float], pick_rollout: Callable[[int], int],
          actions_for: Callable[[int, int], np.ndarray], clock: Callable[[], float],
          advance: Optional[Callable[[float], None]] = None, drain: bool = True):
    """Feed requests at the given arrival times (relative to the clock at the
    start) and pump the server until every request has finished.  With a
    virtual clock, `advance(t)` moves it to t."""
    t0 = clock()
    i = 0
    n = len(arrivals)
    while i < n or (drain and not server.idle()):
        now = clock() - t0
        while i < n and arrivals[i] <= now:
            rid = pick_rollout(i)
            server.submit(rid, actions_for(i, rid), arrivals[i])
            i += 1
        server.pump(now)
        if advance is not None:
            nxt = [arrivals[i]] if i < n else []
            nxt += list(server.ex.busy.values()) if hasattr(server.ex, "busy") else []
            if not nxt:
                break          # nothing can change any more (idle, or waiting for memory forever)
            advance(t0 + max(min(nxt), now))
    return t0
