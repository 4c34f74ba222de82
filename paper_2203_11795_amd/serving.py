"""Serving a stream of transform requests on one GPU.

A request names a shape (rank 2..4 here, every side split over a 2-processor
cyclic grid, so p_l = 2), a dtype and a direction. Serving one request means:
generate its input on the device (fftu_fill_uniform with key (seed, request
id), so no data crosses PCIe and any result can be reproduced on the host),
transform it in place with an external plan (fftu_plan_external +
fftu_execute_ws: no allocation per request), and report it complete when its
stream passes the event recorded after it. Latency is completion minus arrival,
both on one clock: completion times come from the GPU timestamps of those events,
placed on the host clock through one reference event.

HBM admission: every request needs 2 N b bytes (its buffer and the plan's
workspace). They are carved out of one device arena allocated up front; a
request is admitted, in arrival order, only when both fit, and otherwise waits
for running requests to release theirs. Plans hold no device memory, so the plan
cache is an LRU of host objects.

Three policies over the same arena, plan cache and kernels:
  "continuous"  up to `streams` requests run at once, one per HIP stream (all of
                default priority); a stream that finishes takes the next
                admitted request at once, and no stream waits for the host.
                Requests of at least `large_bytes` go to `large_lanes` streams
                of their own, in arrival order, so a large request shares HBM
                bandwidth only with small ones (two large requests at once would
                each take twice as long), while small requests never queue
                behind a large one. A large lane with no large request waiting
                takes a small one.
  "coalesced"   "continuous", and when a free stream finds the first waiting
                request small (at most `coalesce_bytes`, a shape the persistent
                batch kernel supports: every local side n_l/2 <= 256) with at
                least one more such request of the same dtype and direction
                waiting, it takes up to `coalesce_max` of them and runs them as
                one batch launch (fftu_plan_batch_external: a host-only plan,
                cached per composition; its work list goes over from a
                page-locked staging ring, its workspace comes from the arena). A
                small request that waits alone runs as in "continuous". Members of
                a batch are bitwise the same as in a batch of one, and within the
                dtype's tolerance of the per-request path.
  "fifo"        one request at a time on one stream; the host waits for each to
                finish before it starts the next (the plain baseline).
"""
from __future__ import annotations

import bisect
import collections
import math
import time
from dataclasses import dataclass, field

from . import fftu as _b

ALIGN = 256


@dataclass
class Request:
    rid: int
    arrival: float           # seconds after the start of the run
    shape: tuple
    dtype: str               # "complex64" or "complex128"
    direction: int           # -1 forward, +1 inverse

    @property
    def grid(self):
        return (2,) * len(self.shape)

    @property
    def N(self) -> int:
        return math.prod(self.shape)

    @property
    def esize(self) -> int:
        return 16 if self.dtype == "complex128" else 8


def requests_from_trace(trace, limit_seconds=None):
    """Request objects from synth.serving_trace records (optionally the first seconds only)."""
    import numpy as np
    out = []
    for r in trace:
        if limit_seconds is not None and r["t"] >= limit_seconds:
            break
        dt = "complex128" if np.dtype(r["dtype"]) == np.complex128 else "complex64"
        out.append(Request(int(r["id"]), float(r["t"]), tuple(r["shape"]), dt, int(r["direction"])))
    return out


def request_class(req: Request, lanes: int, large_bytes: int) -> str:
    """'large' when the continuous policy has large lanes and the request's buffer
    is at least large_bytes; else 'small'."""
    return "large" if lanes and req.N * req.esize >= large_bytes else "small"


def next_queue(stream: int, lanes: int, large, small):
    """The queue stream `stream` takes its next request from: the large lanes
    (streams below `lanes`) take large requests first and small ones when no
    large one waits; the other streams take small requests only. None: nothing
    for this stream."""
    if stream < lanes and large:
        return large
    return small if small else None


def fits_arena(req: Request, capacity: int) -> bool:
    """Whether the request's two blocks (buffer and workspace, each rounded up to
    ALIGN) fit an empty arena of `capacity` bytes."""
    block = (req.N * req.esize + ALIGN - 1) // ALIGN * ALIGN
    return 2 * block <= capacity


class Arena:
    """First-fit allocator over [0, capacity) with coalescing (offsets in bytes)."""

    def __init__(self, capacity: int):
        self.capacity = int(capacity)
        self.free = [(0, self.capacity)]        # sorted, non-adjacent
        self.used = 0

    def alloc(self, nbytes: int):
        need = (int(nbytes) + ALIGN - 1) // ALIGN * ALIGN
        for i, (off, size) in enumerate(self.free):
            if size >= need:
                if size == need:
                    self.free.pop(i)
                else:
                    self.free[i] = (off + need, size - need)
                self.used += need
                return off, need
        return None

    def release(self, off: int, need: int):
        i = bisect.bisect_left(self.free, (off, 0))
        self.free.insert(i, (off, need))
        self.used -= need
        # merge with the right, then the left neighbour
        if i + 1 < len(self.free) and self.free[i][0] + self.free[i][1] == self.free[i + 1][0]:
            self.free[i] = (off, self.free[i][1] + self.free[i + 1][1])
            self.free.pop(i + 1)
        if i > 0 and self.free[i - 1][0] + self.free[i - 1][1] == self.free[i][0]:
            self.free[i - 1] = (self.free[i - 1][0], self.free[i - 1][1] + self.free[i][1])
            self.free.pop(i)


class PlanCache:
    """LRU of external plans keyed by (shape, dtype, direction)."""

    def __init__(self, capacity: int = 4096):
        self.capacity = int(capacity)
        self.plans = collections.OrderedDict()
        self.hits = 0
        self.misses = 0

    def get(self, req: Request):
        key = (req.shape, req.dtype, req.direction)
        pl = self.plans.get(key)
        if pl is not None:
            self.plans.move_to_end(key)
            self.hits += 1
            return pl
        self.misses += 1
        pl = _b.Plan(req.shape, req.grid, req.dtype, req.direction, external=True)
        self.plans[key] = pl
        if len(self.plans) > self.capacity:
            _, old = self.plans.popitem(last=False)
            old.close()
        return pl

    def close(self):
        for pl in self.plans.values():
            pl.close()
        self.plans.clear()


@dataclass
class _Running:
    reqs: list               # the requests this launch serves (one, or a coalesced batch)
    blocks: list
    end: object              # torch.cuda.Event
    outs: list               # their buffers (views into the arena)
    slot: int = -1           # staging slot held until `end` (coalesced batches)


@dataclass
class ServeResult:
    policy: str
    latencies: dict = field(default_factory=dict)    # rid -> seconds
    completed: int = 0
    unfinished: int = 0
    wall: float = 0.0
    outputs: dict = field(default_factory=dict)      # rid -> host copy (numpy), for the rids asked for
    plan_hits: int = 0
    plan_misses: int = 0
    peak_arena_bytes: int = 0
    refused: list = field(default_factory=list)      # rids larger than the whole arena (never admissible)
    batches: int = 0                                 # launches of the persistent batch kernel ("coalesced")
    coalesced_requests: int = 0                      # requests served by them
    max_batch: int = 0
    coalesced_rids: set = field(default_factory=set)


class Server:
    """Serves requests with one of the two policies over a shared arena and plan cache."""

    def __init__(self, arena_bytes: int = 16 << 30, streams: int = 4, seed: int = 5, plan_cache: int = 4096,
                 large_bytes: int = 64 << 20, large_lanes: int = 2, coalesce_bytes: int = 4 << 20,
                 coalesce_max: int = 64, staging_slots: int = 16, staging_bytes: int = 2 << 20):
        import torch
        self.torch = torch
        self.dev = torch.device("cuda:0")
        self.arena_bytes = int(arena_bytes)
        self.mem = torch.empty(self.arena_bytes, dtype=torch.uint8, device=self.dev)
        self.seed = int(seed)
        self.nstreams = int(streams)
        self.streams = [torch.cuda.Stream(self.dev) for _ in range(self.nstreams)]   # default priority
        self.plans = PlanCache(plan_cache)
        self.large_bytes = int(large_bytes)
        self.large_lanes = max(1, min(int(large_lanes), self.nstreams))
        self.coalesce_bytes = int(coalesce_bytes)
        self.coalesce_max = max(1, int(coalesce_max))
        # page-locked staging ring for the batch work lists; a slot is free again once
        # the event recorded after its batch has passed
        self.staging = [torch.empty(int(staging_bytes), dtype=torch.uint8, pin_memory=True)
                        for _ in range(int(staging_slots))]
        self.slot_busy = [None] * len(self.staging)
        self._batchable = {}
        self.batch_plans = collections.OrderedDict()     # composition -> external BatchPlan (host-only)
        self.batch_plan_cap = 1024

    def close(self):
        self.plans.close()
        for bp in self.batch_plans.values():
            bp.close()
        self.batch_plans.clear()
        self.mem = None
        self.staging = []

    def _batch_plan(self, group):
        key = (tuple(r.shape for r in group), group[0].dtype, group[0].direction)
        bp = self.batch_plans.get(key)
        if bp is not None:
            self.batch_plans.move_to_end(key)
            return bp
        bp = _b.BatchPlan([r.shape for r in group], [r.grid for r in group], group[0].dtype, group[0].direction,
                          external=True)
        self.batch_plans[key] = bp
        if len(self.batch_plans) > self.batch_plan_cap:
            _, old = self.batch_plans.popitem(last=False)
            old.close()                       # host-only: enqueued work does not refer to it
        return bp

    def batchable(self, req: Request) -> bool:
        """Whether the coalesced policy runs this request through the batch kernel:
        at most coalesce_bytes, a shape the persistent kernel supports, and a work
        list that fits one staging slot on its own."""
        if req.N * req.esize > self.coalesce_bytes or not self.staging:
            return False
        key = (req.shape, req.dtype)
        ok = self._batchable.get(key)
        if ok is None:
            try:
                bp = _b.BatchPlan([req.shape], [req.grid], req.dtype, req.direction, external=True)
                ok = bp.staging_bytes <= self.staging[0].numel()
                bp.close()
            except _b.FftuError:
                ok = False
            self._batchable[key] = ok
        return ok

    def _free_slot(self):
        for i, ev in enumerate(self.slot_busy):
            if ev is None or ev.query():
                self.slot_busy[i] = None
                return i
        return -1

    def _view(self, off: int, req: Request):
        t = self.torch.complex128 if req.dtype == "complex128" else self.torch.complex64
        return self.mem[off:off + req.N * req.esize].view(t)

    def _launch(self, req: Request, arena: Arena, stream):
        nbytes = req.N * req.esize
        a = arena.alloc(nbytes)
        if a is None:
            return None
        b = arena.alloc(nbytes)
        if b is None:
            arena.release(*a)
            return None
        plan = self.plans.get(req)
        buf = self._view(a[0], req)
        ws = self._view(b[0], req)
        _b.fill_uniform(buf, self.seed, req.rid, 0, stream=stream)
        plan(buf, buf, stream=stream, workspace=ws)
        end = self.torch.cuda.Event(enable_timing=True)
        end.record(stream)
        return _Running([req], [a, b], end, [buf])

    def _launch_batch(self, group, arena: Arena, stream):
        """One persistent launch for the requests in `group` (same dtype and
        direction): their buffers and the batch workspace from the arena, the work
        list through a free staging slot. None when memory or a slot is lacking."""
        slot = self._free_slot()
        if slot < 0:
            return None
        bp = self._batch_plan(group)
        if bp.staging_bytes > self.staging[slot].numel():
            return None
        blocks = []
        for r in group:
            a = arena.alloc(r.N * r.esize)
            if a is None:
                break
            blocks.append(a)
        w = arena.alloc(bp.workspace_bytes) if len(blocks) == len(group) else None
        if w is None:
            for blk in blocks:
                arena.release(*blk)
            return None
        bufs = [self._view(a[0], r) for a, r in zip(blocks, group)]
        for r, buf in zip(group, bufs):
            _b.fill_uniform(buf, self.seed, r.rid, 0, stream=stream)
        bp.execute_ws_ptrs([b.data_ptr() for b in bufs], [b.data_ptr() for b in bufs],
                           self.mem.data_ptr() + w[0], self.staging[slot].data_ptr(), int(stream.cuda_stream))
        end = self.torch.cuda.Event(enable_timing=True)
        end.record(stream)
        self.slot_busy[slot] = end
        return _Running(list(group), blocks + [w], end, bufs, slot)

    def warmup(self, requests, count: int = 8):
        """Run the largest few requests untimed (first-use costs: the shared twiddle
        tables, the kernels' first launches), and one small batch of each dtype."""
        arena = Arena(self.arena_bytes)
        for r in sorted(requests, key=lambda r: -r.N)[:count]:
            run = self._launch(r, arena, self.streams[0])
            run.end.synchronize()
            for blk in run.blocks:
                arena.release(*blk)
        for dt in ("complex64", "complex128"):
            group = [r for r in requests if r.dtype == dt and self.batchable(r)][:4]
            group = [q for q in group if q.direction == group[0].direction] if group else []
            if group:
                run = self._launch_batch(group, arena, self.streams[0])
                if run is not None:
                    run.end.synchronize()
                    for blk in run.blocks:
                        arena.release(*blk)
        self.torch.cuda.synchronize()

    def serve(self, requests, policy: str = "continuous", keep=(), time_limit: float = None) -> ServeResult:
        """Serve `requests` (sorted by arrival) in real time. keep: rids whose outputs
        are copied to the host. time_limit: stop admitting after this many seconds
        (requests not done by then count as unfinished)."""
        torch = self.torch
        if policy not in ("continuous", "coalesced", "fifo"):
            raise ValueError(policy)
        reqs = sorted(requests, key=lambda r: r.arrival)
        keep = set(keep)
        nstreams = 1 if policy == "fifo" else self.nstreams
        coalesce = policy == "coalesced"
        arena = Arena(self.arena_bytes)
        res = ServeResult(policy)
        hits0, miss0 = self.plans.hits, self.plans.misses

        torch.cuda.synchronize()
        ref = torch.cuda.Event(enable_timing=True)
        ref.record(self.streams[0])
        ref.synchronize()
        t0 = time.perf_counter()                  # host time of the reference event (to ~10 us)

        def finish(run: _Running):
            done = ref.elapsed_time(run.end) * 1e-3
            for r, buf in zip(run.reqs, run.outs):
                res.latencies[r.rid] = done - r.arrival
                res.completed += 1
                if r.rid in keep:
                    res.outputs[r.rid] = buf.cpu().numpy()
            for blk in run.blocks:
                arena.release(*blk)

        def take(q, s):
            """Launch the head of q on stream s (with its coalescing partners); None if
            memory or a staging slot is lacking."""
            head = q[0]
            group, idx = [head], [0]
            if coalesce and self.batchable(head):
                for j in range(1, min(len(q), 4 * self.coalesce_max)):
                    if len(group) >= self.coalesce_max:
                        break
                    r = q[j]
                    if r.dtype == head.dtype and r.direction == head.direction and self.batchable(r):
                        group.append(r)
                        idx.append(j)
            run = self._launch_batch(group, arena, self.streams[s]) if len(group) > 1 else None
            if run is None:
                # nothing to coalesce with (or no memory or staging slot for the group now):
                # the head alone, by the per-request path
                run = self._launch(head, arena, self.streams[s])
                if run is not None:
                    q.popleft()
                return run
            for j in reversed(idx):
                del q[j]
            res.batches += 1
            res.coalesced_requests += len(group)
            res.max_batch = max(res.max_batch, len(group))
            res.coalesced_rids.update(r.rid for r in group)
            return run

        # continuous / coalesced: streams [0, large_lanes) serve the large class first; fifo: one queue
        small = collections.deque()
        large = collections.deque()
        lanes = 0 if policy == "fifo" else self.large_lanes
        running = [None] * nstreams
        i = 0
        n = len(reqs)

        while True:
            now = time.perf_counter() - t0
            if time_limit is not None and now > time_limit:
                break
            while i < n and reqs[i].arrival <= now:
                r = reqs[i]
                i += 1
                if not fits_arena(r, self.arena_bytes):
                    res.refused.append(r.rid)     # would wait forever for memory that never frees
                    continue
                (large if request_class(r, lanes, self.large_bytes) == "large" else small).append(r)
            progressed = False
            for s in range(nstreams):
                run = running[s]
                if run is not None and run.end.query():
                    finish(run)
                    running[s] = None
                    progressed = True
            blocked = False
            for s in range(nstreams):
                if running[s] is not None or blocked:
                    continue
                q = next_queue(s, lanes, large, small)
                if q is None:
                    continue
                run = take(q, s)
                if run is None:
                    if all(r is None for r in running):
                        # nothing runs, so nothing will free memory or a staging slot: this
                        # request can never start
                        res.refused.append(q.popleft().rid)
                        continue
                    blocked = True                # HBM admission: wait for running requests
                    continue
                res.peak_arena_bytes = max(res.peak_arena_bytes, arena.used)
                running[s] = run
                progressed = True
                if policy == "fifo":
                    run.end.synchronize()         # the host waits for each request
            if i >= n and not small and not large and all(r is None for r in running):
                break
            if not progressed:
                if all(r is None for r in running) and not small and not large and i < n:
                    time.sleep(max(0.0, min(reqs[i].arrival - (time.perf_counter() - t0), 1e-3)))
                else:
                    time.sleep(2e-5)
        for s in range(nstreams):
            if running[s] is not None:
                running[s].end.synchronize()
                finish(running[s])
        torch.cuda.synchronize()
        res.wall = time.perf_counter() - t0
        res.unfinished = len(reqs) - res.completed - len(res.refused)
        res.plan_hits = self.plans.hits - hits0
        res.plan_misses = self.plans.misses - miss0
        return res


def precision_errors(server: "Server", requests) -> dict:
    """The error of every complex64 request's result, stated per result: the
    request's own input (Philox, key (seed, rid)) transformed by its complex64
    plan, against the complex128 transform of the same values promoted exactly;
    rel-L2 = ||y32 - y64|| / ||y64||, computed on the device. Returns rid -> error."""
    torch = server.torch
    out = {}
    stream = server.streams[0]
    with torch.cuda.stream(stream):
        for r in requests:
            if r.dtype != "complex64":
                continue
            p32 = server.plans.get(r)
            r64 = Request(r.rid, r.arrival, r.shape, "complex128", r.direction)
            p64 = server.plans.get(r64)
            x32 = torch.empty(r.N, dtype=torch.complex64, device=server.dev)
            _b.fill_uniform(x32, server.seed, r.rid, 0, stream=stream)
            x64 = x32.to(torch.complex128)
            ws32 = torch.empty_like(x32)
            ws64 = torch.empty_like(x64)
            p32(x32, x32, stream=stream, workspace=ws32)
            p64(x64, x64, stream=stream, workspace=ws64)
            num = torch.linalg.vector_norm(x32.to(torch.complex128) - x64)
            den = torch.linalg.vector_norm(x64)
            out[r.rid] = (num / den).item()
    return out


def summarize(res: ServeResult, requests) -> dict:
    """p50/p99 latency, offered and achieved rates and GFLOP/s (5 N log2 N) of a run."""
    import numpy as np
    byid = {r.rid: r for r in requests}
    lat = np.array(sorted(res.latencies.values())) if res.latencies else np.array([float("nan")])
    flops = sum(5.0 * byid[k].N * math.log2(byid[k].N) for k in res.latencies)
    span = max(r.arrival for r in requests) if requests else 0.0
    return {
        "policy": res.policy, "requests": len(requests), "completed": res.completed, "unfinished": res.unfinished,
        "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 3), "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 3),
        "mean_ms": round(float(lat.mean()) * 1e3, 3), "max_ms": round(float(lat.max()) * 1e3, 3),
        "offered_rps": round(len(requests) / span, 1) if span > 0 else None,
        "achieved_rps": round(res.completed / res.wall, 1) if res.wall > 0 else None,
        "GFLOPs": round(flops / res.wall / 1e9, 1) if res.wall > 0 else None,
        "wall_s": round(res.wall, 3), "plan_hits": res.plan_hits, "plan_misses": res.plan_misses,
        "peak_arena_GiB": round(res.peak_arena_bytes / 2 ** 30, 3), "refused": len(res.refused),
        "batches": res.batches, "coalesced_requests": res.coalesced_requests, "max_batch": res.max_batch,
    }
