"""Serving front end: Helmholtz solve requests over resident set-up contexts, continuously batched.

A request names a problem key and carries nrhs right-hand sides (already in device memory).  The
context cache keeps set-up contexts (local inverses, coarse basis, B_0^{-1}) resident by key, so
later requests for the same problem reuse them.  A miss is set up on a side thread with its own
HIP stream while the live set keeps iterating; the cache evicts least-recently-used idle contexts
when its byte budget would be exceeded, and a setup waits until room frees up.  Ready requests go
to the C++ server (``hkgeneo_server_*``), which admits them by Krylov-workspace budget at iteration
boundaries and steps every live request in the same launches.

Every numerical step runs in the HIP library; this module only schedules.  Latency of a request is
measured from its arrival to the poll that returns it, so it includes queueing and, on a cache
miss, the setup.
"""
from __future__ import annotations

import collections
import dataclasses
import queue
import threading
import time

import numpy as np

from . import hkgeneo as H


@dataclasses.dataclass
class Request:
    tag: int
    arrival: float              # seconds from the start of the run
    key: tuple                  # problem key (hashable)
    f: object                   # (nrhs, n) float64 tensor on the GPU
    t_submit: float = -1.0
    t_done: float = -1.0
    cache_hit: bool = False
    info: list | None = None
    status: int = 0
    u: object = None


def footprint_estimate(problem, local_prec: int = 32, nev: int = 12) -> int:
    """Device bytes a set-up context will hold, from the host partition alone: local inverses,
    coarse basis (twice: both layouts), dense B_0^{-1}, CSR and index data."""
    nI, _, _, _, _, _ = H.partition(problem)
    m0 = int(len(nI)) * (nev + 4)
    s = 4 if local_prec == 32 else 8
    return int(s * np.sum(np.asarray(nI, np.int64) ** 2) + 16 * np.sum(nI) * (nev + 4) + 8 * m0 * m0
               + 32 * len(problem.col_idx) + 64 * problem.n_dof)


class ContextCache:
    """Resident contexts by key with least-recently-used eviction of idle entries."""

    def __init__(self, budget_bytes: int):
        self.budget = int(budget_bytes)
        self._items: collections.OrderedDict = collections.OrderedDict()   # key -> [solver, bytes, refs]
        self.hits = 0
        self.misses = 0
        self.evictions = 0

    @property
    def bytes(self) -> int:
        return sum(v[1] for v in self._items.values())

    def __contains__(self, key):
        return key in self._items

    def acquire(self, key):
        v = self._items[key]
        self._items.move_to_end(key)
        v[2] += 1
        return v[0]

    def release(self, key):
        self._items[key][2] -= 1

    def make_room(self, need: int) -> bool:
        """Evict idle contexts (least recently used first) until `need` more bytes fit."""
        while self.bytes + need > self.budget:
            idle = [k for k, v in self._items.items() if v[2] == 0]
            if not idle:
                return False
            solver = self._items.pop(idle[0])[0]
            solver.close()
            self.evictions += 1
        return True

    def insert(self, key, solver):
        self._items[key] = [solver, int(solver.stats()["device_bytes"]), 0]

    def close(self):
        for v in self._items.values():
            v[0].close()
        self._items.clear()


class _SetupWorker(threading.Thread):
    """Sets up contexts on its own HIP stream (the ctypes calls release the interpreter lock)."""

    def __init__(self, make_solver):
        super().__init__(daemon=True)
        self.make_solver = make_solver
        self.jobs: queue.Queue = queue.Queue()
        self.results: queue.Queue = queue.Queue()

    def run(self):
        import torch
        stream = torch.cuda.Stream()
        while True:
            key = self.jobs.get()
            if key is None:
                return
            t = time.perf_counter()
            try:
                solver = self.make_solver(key, stream)
                stream.synchronize()
                self.results.put((key, solver, time.perf_counter() - t, None))
            except Exception as e:   # reported by the serving loop
                self.results.put((key, None, time.perf_counter() - t, e))


def run_stream(requests, make_solver, estimate, *, ctx_budget: int, workspace_budget: int, max_requests: int = 64,
               max_nrhs: int = 8, restart: int = 50, periods: int = 1, cache: ContextCache | None = None):
    """Serve `requests` (sorted by arrival) in real time and return (requests, summary).

    make_solver(key, stream) sets up a context; estimate(key) is its footprint before setup.  The
    cache may be passed in to start warm (and is then left open); otherwise it is closed at the end.
    """
    import torch
    own_cache = cache is None
    cache = cache or ContextCache(ctx_budget)
    worker = _SetupWorker(make_solver)
    worker.start()
    waiting: dict = collections.defaultdict(list)     # key -> requests waiting for its setup
    blocked: collections.deque = collections.deque()    # keys whose setup waits for cache room
    in_setup: set = set()
    by_tag = {r.tag: r for r in requests}
    setup_times = []
    hbm_peak = 0
    srv = H.Server(workspace_budget, max_requests=max_requests, max_nrhs=max_nrhs, restart=restart)
    counts0 = (cache.hits, cache.misses, cache.evictions)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nxt, done = 0, 0

    def now():
        return time.perf_counter() - t0

    def submit(r):
        r.t_submit = now()
        srv.submit(cache.acquire(r.key), r.f, r.tag)

    def try_setups():
        while blocked:
            key = blocked[0]
            if not cache.make_room(estimate(key)):
                return
            blocked.popleft()
            in_setup.add(key)
            worker.jobs.put(key)

    try:
        while done < len(requests):
            t = now()
            while nxt < len(requests) and requests[nxt].arrival <= t:
                r = requests[nxt]
                nxt += 1
                if r.key in cache:
                    r.cache_hit = True
                    cache.hits += 1
                    submit(r)
                else:
                    cache.misses += 1
                    waiting[r.key].append(r)
                    if r.key not in in_setup and r.key not in blocked:
                        blocked.append(r.key)
            try_setups()
            while True:
                try:
                    key, solver, dt, err = worker.results.get_nowait()
                except queue.Empty:
                    break
                if err is not None:
                    raise err
                in_setup.discard(key)
                setup_times.append(dt)
                cache.insert(key, solver)
                for r in waiting.pop(key, []):
                    submit(r)
            st = srv.stats()
            if st["live"] + st["queued"] > 0:
                srv.pump(periods)
            for tag, u, info, status in srv.poll():
                r = by_tag[tag]
                r.t_done = now()
                r.u, r.info, r.status = u, info, status
                cache.release(r.key)
                done += 1
            hbm_peak = max(hbm_peak, cache.bytes + srv.stats()["device_bytes"])
            if srv.stats()["live"] == 0 and nxt < len(requests) and not in_setup:
                dt = requests[nxt].arrival - now()
                if dt > 0:
                    time.sleep(min(dt, 2e-3))
        wall = max(r.t_done for r in requests) - min(r.arrival for r in requests)
        stats = srv.stats()
    finally:
        worker.jobs.put(None)
        srv.close()
        if own_cache:
            cache.close()
    lat = np.array([r.t_done - r.arrival for r in requests])
    nrhs = sum(int(r.f.shape[0]) for r in requests)
    summary = dict(requests=len(requests), rhs=nrhs, wall_s=wall, solves_per_s=nrhs / wall,
                   p50_ms=float(np.percentile(lat, 50) * 1e3), p99_ms=float(np.percentile(lat, 99) * 1e3),
                   mean_ms=float(lat.mean() * 1e3), hits=cache.hits - counts0[0], misses=cache.misses - counts0[1],
                   evictions=cache.evictions - counts0[2],
                   setups=len(setup_times), setup_ms_mean=float(np.mean(setup_times) * 1e3) if setup_times else 0.0,
                   hbm_peak_bytes=int(hbm_peak), iterations=stats["iterations"], captures=stats["captures"],
                   converged=all(i["converged"] for r in requests for i in r.info))
    return requests, summary
