"""Continuous-batching reconstruction server on one GPU.

Requests (a scan geometry, a voxel grid and a device-resident sinogram) arrive over time.
The server

* builds the float64 plan of each new geometry on worker threads (on the GPU, straight into
  device tables; plans are cached by the exact geometry/grid tuple, least recently used
  ones dropped beyond a table budget once no request in flight holds them),
* admits ready requests first-come-first-served while their device footprint (sinogram
  copy, filter workspace, g^F, volume) gets a contiguous block of the server's HBM arena
  (one buffer of the budget's size, first-fit), otherwise they wait until earlier requests
  finish and free their blocks,
* launches every admitted group as the per-request filter kernels followed by one grouped
  backprojection (``katsevich_backproject_batch``: the tiles of all the group's requests in
  one grid, so small reconstructions fill the GPU together), alternating between two streams
  so that a new group's filtering overlaps the previous group's backprojection; a group is
  closed once its backprojection work (voxel-view updates) reaches ``group_work``, which
  bounds the latency a request waits for its group-mates,
* records per-request latency (completion event time - arrival) and throughput.

Every reconstruction step runs in libkatsevich; this module only schedules.  The packed
launch computes each tile exactly as the one-request kernel does, so a request's volume is
bit-identical alone and in the mix.
"""
from __future__ import annotations

import collections
import threading
import time
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

from . import katsevich as K


def plan_key(geom: dict, grid: dict, n_psi: int = 0, bp_slices: int = 0):
    return (tuple(sorted((k, float(v)) for k, v in geom.items())),
            tuple(sorted((k, float(v)) for k, v in grid.items())), int(n_psi), int(bp_slices))


@dataclass
class Request:
    rid: int
    arrival: float               # seconds after the trace start
    geom: dict
    grid: dict
    sino: object                 # device tensor [n_views, rows, cols] (read only)
    # event recorded on the stream that wrote sino (None: sino was complete before run());
    # the serving stream waits for it before reading the sinogram
    ready: object = None
    # filled by the server
    t_plan_ready: float = float("nan")
    t_admit: float = float("nan")
    t_done: float = float("nan")
    cache_hit: bool = False
    plan_seconds: float = 0.0
    footprint: int = 0
    valid_voxels: int = 0        # voxels the plan reconstructs (the rest of the grid is 0)
    plan_key: object = None
    offset: int = 0              # arena byte offset while in flight
    volume: object = None
    error: str = ""              # non-empty: rejected (plan failed or footprint too large)

    @property
    def latency(self):
        return self.t_done - self.arrival


class PlanFailed(RuntimeError):
    """The plan of a request's geometry could not be built."""


class PlanCache:
    """Plans keyed by geometry; built on worker threads, each on its own stream (on the GPU
    by default: katsevich_plan_device writes the tables straight into device memory, so the
    serving streams never wait for a table upload).  Cached plans are kept while their tables
    fit table_budget bytes; beyond it the least recently used plans that no request in
    flight holds (acquire / release) are dropped."""

    def __init__(self, device, workers=2, n_psi=0, bp_slices=0, gpu_plan=True,
                 table_budget: float = 32e9):
        self.device = device
        self.n_psi, self.bp_slices = n_psi, bp_slices
        self.gpu_plan = gpu_plan                   # plans built on the GPU (katsevich_plan_device)
        self.table_budget = float(table_budget)
        self.plans = collections.OrderedDict()     # least recently used first
        self.pending = {}
        self.failed = {}
        self.build_seconds = {}
        self.inuse = collections.Counter()
        self.hits = self.misses = self.evicted = 0
        self.table_bytes = 0
        self._lock = threading.Lock()
        self._pool = ThreadPoolExecutor(max_workers=workers)
        self._streams = {}

    def acquire(self, key):
        """A request in flight holds the plan of key (it is not evicted meanwhile)."""
        with self._lock:
            self.inuse[key] += 1
            if key in self.plans:
                self.plans.move_to_end(key)

    def release(self, key):
        with self._lock:
            self.inuse[key] -= 1
            if self.inuse[key] <= 0:
                del self.inuse[key]
            self._evict()

    def _evict(self):
        # caller holds the lock
        if self.table_bytes <= self.table_budget:
            return
        for key in list(self.plans):
            if self.table_bytes <= self.table_budget:
                break
            if self.inuse.get(key, 0) > 0:
                continue
            plan = self.plans.pop(key)
            self.table_bytes -= int(plan.info["table_bytes"])
            self.evicted += 1

    def _build(self, geom, grid):
        import torch
        t0 = time.perf_counter()
        tid = threading.get_ident()
        with self._lock:
            s = self._streams.get(tid)
            if s is None:
                s = self._streams[tid] = torch.cuda.Stream(device=self.device)
        index = self.device.index if hasattr(self.device, "index") else self.device
        with torch.cuda.stream(s):
            # a device-built plan is bound to the table buffer it was built in
            plan = K.Plan(geom, grid, n_psi=self.n_psi, bind=False, bp_slices=self.bp_slices,
                          gpu_plan=self.gpu_plan, device=index)
            if plan.tables is None:
                plan.bind(index)
        return plan, time.perf_counter() - t0

    def request(self, geom, grid):
        """(key, cache_hit); starts a background build on a miss."""
        key = plan_key(geom, grid, self.n_psi, self.bp_slices)
        with self._lock:
            if key in self.plans:
                self.hits += 1
                self.plans.move_to_end(key)
                return key, True
            self.misses += 1
            if key not in self.pending:
                self.pending[key] = self._pool.submit(self._build, geom, grid)
            return key, False

    def poll(self, key):
        """Plan of key if built (moving it into the cache), else None; raises
        PlanFailed if its build failed (every later poll of that key raises too)."""
        with self._lock:
            if key in self.plans:
                return self.plans[key]
            if key in self.failed:
                raise PlanFailed(self.failed[key])
            fut = self.pending.get(key)
        if fut is None or not fut.done():
            return None
        try:
            plan, secs = fut.result()
        except Exception as exc:                      # a geometry the library rejects
            with self._lock:
                self.failed[key] = f"plan build failed: {exc}"
                self.pending.pop(key, None)
            raise PlanFailed(self.failed[key]) from exc
        with self._lock:
            if key not in self.plans:
                self.plans[key] = plan
                self.build_seconds[key] = secs
                self.table_bytes += int(plan.info["table_bytes"])
                self.pending.pop(key, None)
                self._evict()
            return plan

    def get_blocking(self, geom, grid):
        """Plan of (geom, grid), waiting for its build (raises PlanFailed)."""
        key, _ = self.request(geom, grid)
        while True:
            p = self.poll(key)
            if p is not None:
                return p
            time.sleep(0.0005)

    def close(self):
        self._pool.shutdown(wait=True)


_ALIGN = 256


def _up(n: int) -> int:
    return (int(n) + _ALIGN - 1) // _ALIGN * _ALIGN


def layout(plan: K.Plan):
    """Byte offsets of a request's device buffers inside its arena block: sinogram copy,
    filter workspace, g^F, volume (each 256-byte aligned); returns (offsets, total)."""
    g, gr = plan.geom, plan.grid
    sizes = (int(g["n_views"]) * int(g["det_rows"]) * int(g["det_cols"]) * 4,
             max(int(plan.info["workspace_bytes_filter"]), _ALIGN),
             int(plan.info["filtered_bytes"]),
             int(gr["nx"]) * int(gr["ny"]) * int(gr["nz"]) * 4)
    offs, o = [], 0
    for n in sizes:
        offs.append(o)
        o += _up(n)
    return offs, o


def footprint(plan: K.Plan) -> int:
    """Device bytes a request holds while in flight."""
    return layout(plan)[1]


class Arena:
    """First-fit allocation of 256-byte-aligned ranges of one device buffer (host-side
    bookkeeping; the admission test of the server).  A request is admitted when its whole
    footprint gets one contiguous range, so admitted work never waits on the framework's
    allocator and the budget is exact."""

    def __init__(self, nbytes: int):
        self.size = int(nbytes) // _ALIGN * _ALIGN
        self.free = [(0, self.size)] if self.size else []     # sorted, coalesced
        self.used = 0

    def alloc(self, nbytes: int):
        n = _up(nbytes)
        if n > self.size:
            raise ValueError(f"request footprint {n} B exceeds the whole budget {self.size} B")
        for i, (o, sz) in enumerate(self.free):
            if sz >= n:
                if sz == n:
                    del self.free[i]
                else:
                    self.free[i] = (o + n, sz - n)
                self.used += n
                return o
        return None

    def release(self, offset: int, nbytes: int):
        n = _up(nbytes)
        self.used -= n
        assert self.used >= 0
        i = 0
        while i < len(self.free) and self.free[i][0] < offset:
            i += 1
        self.free.insert(i, (offset, n))
        # coalesce with the right, then the left neighbour
        if i + 1 < len(self.free) and self.free[i][0] + self.free[i][1] == self.free[i + 1][0]:
            self.free[i] = (self.free[i][0], self.free[i][1] + self.free[i + 1][1])
            del self.free[i + 1]
        if i > 0 and self.free[i - 1][0] + self.free[i - 1][1] == self.free[i][0]:
            self.free[i - 1] = (self.free[i - 1][0], self.free[i - 1][1] + self.free[i][1])
            del self.free[i]


# Backprojection work (voxel-view updates) after which a group is closed: ~2 ms of the
# backprojector, short enough that a request rarely waits long for its group-mates and
# long enough that small reconstructions share launches.
GROUP_WORK = 3.0e9


class Server:
    """Continuous-batching server.  All request buffers live in one device arena of
    budget_bytes (allocated on the first run, kept across runs, freed by close())."""

    def __init__(self, plan_cache: PlanCache, budget_bytes: float = 200e9, max_batch: int = 32,
                 keep_volumes: bool = False, n_streams: int = 2, group_work: float = GROUP_WORK):
        import torch
        self.cache = plan_cache
        self.device = plan_cache.device
        self.arena = Arena(int(budget_bytes))
        self._buf = None
        self.max_batch = max_batch
        self.group_work = float(group_work)
        self.keep_volumes = keep_volumes
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(n_streams)]

    def close(self):
        self._buf = None

    def _views(self, r, plan):
        """Tensors of request r inside its arena block."""
        import torch
        offs, _ = layout(plan)
        g, gr = plan.geom, plan.grid
        base = r.offset

        def view(i, shape, dtype):
            n = int(np.prod(shape)) * (4 if dtype == torch.float32 else 1)
            return self._buf[base + offs[i]: base + offs[i] + n].view(dtype).view(shape)
        sino = view(0, (int(g["n_views"]), int(g["det_rows"]), int(g["det_cols"])), torch.float32)
        ws = view(1, (max(int(plan.info["workspace_bytes_filter"]), _ALIGN),), torch.uint8)
        gF = view(2, K.filtered_shape(plan), torch.float32)
        vol = view(3, K._vol_shape(plan), torch.float32)
        return sino, ws, gF, vol

    def _launch(self, si, batch):
        import torch
        s = self.streams[si]
        plans, gFs, vols = [], [], []
        with torch.cuda.stream(s):
            for r, plan in batch:
                sino, ws, gF, vol = self._views(r, plan)
                if r.ready is not None:                    # the producer's writes first
                    s.wait_event(r.ready)
                r.sino.record_stream(s)                    # read here: keep it alive for s
                sino.copy_(r.sino)                         # D2D copy into the request's slot
                K.filter_views(plan, sino, out=gF, ws=ws)
                plans.append(plan)
                gFs.append(gF)
                vols.append(vol)
            K.backproject_batch(plans, gFs, vols)
            ev = torch.cuda.Event()
            ev.record(s)
        return ev, vols

    def _reject(self, r, why, t0, done):
        """Complete request r with an error; the loop goes on with the others."""
        r.error = why
        r.t_done = time.perf_counter() - t0
        self.cache.release(r.plan_key)
        done.append(r)

    def run(self, requests, clock_start=None):
        """Serve requests (sorted by arrival); returns them with timings filled in."""
        import torch
        if self._buf is None:
            self._buf = torch.empty(self.arena.size, dtype=torch.uint8, device=self.device)
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        waiting = []                                   # arrived, plan maybe not ready
        inflight = [None] * len(self.streams)          # (event, batch, vols)
        t0 = time.perf_counter() if clock_start is None else clock_start
        done = []
        n = len(pending)
        while len(done) < n:
            now = time.perf_counter() - t0
            while pending and pending[0].arrival <= now:
                r = pending.popleft()
                key, hit = self.cache.request(r.geom, r.grid)
                self.cache.acquire(key)                # held until the request completes
                r.cache_hit = hit
                r.plan_key = key
                waiting.append((r, key))
            # completions: the group's stream has finished, its arena blocks are free again
            for si, item in enumerate(inflight):
                if item is not None and item[0].query():
                    tdone = time.perf_counter() - t0
                    _, batch, vols = item
                    for (r, plan), v in zip(batch, vols):
                        r.t_done = tdone
                        if self.keep_volumes:
                            r.volume = v.clone()
                            torch.cuda.current_stream(self.device).synchronize()
                        self.arena.release(r.offset, r.footprint)
                        self.cache.release(r.plan_key)
                        done.append(r)
                    inflight[si] = None
            # admission into a free stream (first come, first served)
            free = [si for si, item in enumerate(inflight) if item is None]
            launched = False
            if free and waiting:
                batch, rest = [], []
                blocked = False
                work = 0.0
                for r, key in waiting:
                    try:
                        plan = self.cache.poll(key)
                    except PlanFailed as exc:
                        self._reject(r, str(exc), t0, done)
                        continue
                    if plan is None:
                        rest.append((r, key))
                        continue
                    if r.t_plan_ready != r.t_plan_ready:     # nan: first time seen ready
                        r.t_plan_ready = time.perf_counter() - t0
                        r.plan_seconds = self.cache.build_seconds.get(key, 0.0)
                        r.footprint = footprint(plan)
                        r.valid_voxels = int(plan.info["n_valid_voxels"])
                        if r.footprint > self.arena.size:
                            self._reject(r, f"footprint {r.footprint} B exceeds the budget "
                                            f"{self.arena.size} B", t0, done)
                            continue
                    off = None
                    if not blocked and len(batch) < self.max_batch and \
                            (not batch or work < self.group_work):
                        off = self.arena.alloc(r.footprint)
                    if off is not None:
                        r.offset = off
                        r.t_admit = time.perf_counter() - t0
                        batch.append((r, plan))
                        work += float(plan.info["n_vv"])
                    else:
                        blocked = True                       # keep arrival order
                        rest.append((r, key))
                waiting = rest
                if batch:
                    si = free[0]
                    ev, vols = self._launch(si, batch)
                    inflight[si] = (ev, batch, vols)
                    launched = True
            if not launched:
                time.sleep(0.0002)
        return done


def serve_sequential(plan_cache: PlanCache, requests, keep_volumes=False):
    """Baseline: one request at a time in arrival order with the single-call
    katsevich_recon (plan from the same cache, synchronised after every request)."""
    import torch
    reqs = sorted(requests, key=lambda r: r.arrival)
    t0 = time.perf_counter()
    for r in reqs:
        while time.perf_counter() - t0 < r.arrival:
            time.sleep(0.0002)
        key, hit = plan_cache.request(r.geom, r.grid)
        plan_cache.acquire(key)
        r.cache_hit = hit
        r.plan_key = key
        try:
            plan = plan_cache.get_blocking(r.geom, r.grid)
        except PlanFailed as exc:
            r.error = str(exc)
            r.t_done = time.perf_counter() - t0
            plan_cache.release(key)
            continue
        r.t_plan_ready = r.t_admit = time.perf_counter() - t0
        r.plan_seconds = plan_cache.build_seconds.get(key, 0.0)
        r.valid_voxels = int(plan.info["n_valid_voxels"])
        if r.ready is not None:
            torch.cuda.current_stream(r.sino.device).wait_event(r.ready)
        sino = r.sino.clone()
        vol = K.recon(plan, sino)
        torch.cuda.current_stream(sino.device).synchronize()
        r.t_done = time.perf_counter() - t0
        r.volume = vol if keep_volumes else None
        del sino
        plan.release_workspace()
        plan_cache.release(key)
    return reqs


def summarize(reqs):
    rejected = [r for r in reqs if r.error]
    reqs = [r for r in reqs if not r.error]
    lat = np.array([r.latency for r in reqs])
    first = min(r.arrival for r in reqs)
    last = max(r.t_done for r in reqs)
    plan_s = np.array([r.plan_seconds for r in reqs if not r.cache_hit] or [0.0])
    return {"requests": len(reqs), "p50_latency_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_latency_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_latency_ms": float(lat.mean() * 1e3), "makespan_s": float(last - first),
            "volumes_per_s": float(len(reqs) / max(last - first, 1e-9)),
            "cache_hits": int(sum(r.cache_hit for r in reqs)),
            "cache_hit_rate": float(np.mean([r.cache_hit for r in reqs])),
            "plan_build_ms_mean": float(plan_s.mean() * 1e3),
            "plan_build_ms_max": float(plan_s.max() * 1e3), "rejected": len(rejected),
            "valid_voxel_fraction": float(sum(r.valid_voxels for r in reqs) /
                                          max(1, sum(int(r.grid["nx"]) * int(r.grid["ny"]) *
                                                     int(r.grid["nz"]) for r in reqs)))}
