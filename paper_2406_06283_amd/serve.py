"""Serving front end: Helmholtz solve requests over resident set-up contexts, continuously batched.

A request names a problem key and carries nrhs right-hand sides (already in device memory).  The
context cache keeps set-up contexts (local inverses, coarse basis, B_0^{-1}) resident by key, so
later requests for the same problem reuse them.  A miss is set up on a side thread with its own
HIP stream while the live set keeps iterating; the cache evicts least-recently-used idle contexts
when its byte budget would be exceeded, and a setup is dispatched only once a reservation of its
estimated peak footprint fits (the reservation becomes the context's measured bytes when it ends).
Ready requests go to the C++ server (``hkgeneo_server_*``), which admits them by Krylov-workspace budget at iteration
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


def footprint_estimate(problem, local_prec: int = 32, m_per_sub: int = 64) -> int:
    """Upper bound on the device bytes of a context at its peak (setup workspace included), from the
    host partition alone, when no subdomain keeps more than m_per_sub eigenvectors (pass the options'
    max_eig_per_sub: setup fails beyond it).  Resident: the local inverses (leading dimension padded
    to 32), the coarse basis in both layouts, the dense B_0^{-1}, CSR and index data.  Workspace: seven
    float64 blocks per subdomain of the size of B_D (its LU, the Schur complement and its product,
    C_II, the padded tridiagonalisation copy, the staging of the inverse and of its float32 copy), the
    Gamma blocks, and six m0 x m0 arrays for B_0 (assembly, a copy, the inverse and the work of the
    banded-LU fallback).  Measured on the serving keys and the named workloads: peak <= bound."""
    nI, nG, _, _, _, _ = H.partition(problem)
    nI = np.asarray(nI, np.int64)
    nG = np.asarray(nG, np.int64)
    m0 = int(len(nI)) * int(m_per_sub)
    s = 4 if local_prec == 32 else 8
    ld = (nI + 31) // 32 * 32
    resident = (s * np.sum(ld * nI) + 16 * np.sum(nI) * m_per_sub + 8 * m0 * m0
                + 32 * len(problem.col_idx) + 64 * problem.n_dof)
    work = 8 * np.sum(7 * (ld + 32) * nI + nG * nG + 2 * nG * nI) + 6 * 8 * m0 * m0
    return int(resident + work)


class ContextCache:
    """Resident contexts by key with least-recently-used eviction of idle entries.

    Bytes are counted against the budget in two ways: a resident context by its measured
    device_bytes, a context being set up by the reservation made when its setup was dispatched (an
    estimate of its peak).  When the setup ends the reservation is replaced by the real bytes and
    idle contexts are evicted if that overshoots the budget."""

    def __init__(self, budget_bytes: int):
        self.budget = int(budget_bytes)
        self._items: collections.OrderedDict = collections.OrderedDict()   # key -> [solver, bytes, refs]
        self._pending: dict = {}                                           # key -> reserved bytes
        self.hits = 0
        self.misses = 0
        self.evictions = 0
        self.overshoots = 0           # setups whose real peak exceeded the reservation
        self.over_budget = 0          # inserts that left the cache above budget (no idle context left)

    @property
    def bytes(self) -> int:
        return sum(v[1] for v in self._items.values()) + sum(self._pending.values())

    def __contains__(self, key):
        return key in self._items

    def acquire(self, key):
        v = self._items[key]
        self._items.move_to_end(key)
        v[2] += 1
        return v[0]

    def release(self, key):
        self._items[key][2] -= 1

    def make_room(self, need: int, keep=None) -> bool:
        """Evict idle contexts (least recently used first, never `keep`) until `need` more bytes fit."""
        while self.bytes + need > self.budget:
            idle = [k for k, v in self._items.items() if v[2] == 0 and k != keep]
            if not idle:
                return False
            solver = self._items.pop(idle[0])[0]
            solver.close()
            self.evictions += 1
        return True

    def reserve(self, key, nbytes: int) -> bool:
        """Make room for and reserve `nbytes` for the setup of `key`; False if it does not fit yet."""
        if not self.make_room(int(nbytes)):
            return False
        self._pending[key] = int(nbytes)
        return True

    def cancel(self, key):
        self._pending.pop(key, None)

    def insert(self, key, solver):
        """A finished setup: its reservation becomes the context's measured device bytes."""
        reserved = self._pending.pop(key, None)
        st = solver.stats()
        if reserved is not None and st.get("peak_device_bytes", 0) > reserved:
            self.overshoots += 1
        self._items[key] = [solver, int(st["device_bytes"]), 0]
        if not self.make_room(0, keep=key):
            self.over_budget += 1

    def close(self):
        for v in self._items.values():
            v[0].close()
        self._items.clear()
        self._pending.clear()


class SetupAdmission:
    """Admission of setups by HBM footprint: keys missing from the cache queue up in arrival order,
    and the head is dispatched (``dispatch(key)``) only once the cache can reserve ``estimate(key)``
    bytes for it, evicting idle contexts if needed.  Keys stay queued in order while the head does not
    fit (no overtaking, so a large setup is not starved by small ones).  At most ``max_in_flight``
    setups are dispatched at a time: the worker runs them one after the other anyway, and a longer
    queue would only hold reservations (upper bounds) that evict resident contexts."""

    def __init__(self, cache: ContextCache, estimate, dispatch, max_in_flight: int = 2):
        self.cache = cache
        self.estimate = estimate
        self.dispatch = dispatch
        self.max_in_flight = int(max_in_flight)
        self.blocked: collections.deque = collections.deque()
        self.in_setup: set = set()

    def request(self, key):
        if key not in self.cache and key not in self.in_setup and key not in self.blocked:
            self.blocked.append(key)

    def pump(self) -> int:
        n = 0
        while self.blocked and len(self.in_setup) < self.max_in_flight:
            key = self.blocked[0]
            need = int(self.estimate(key))
            if need > self.cache.budget:
                raise ValueError(f"setup of {key!r} needs {need} bytes, above the whole budget {self.cache.budget}")
            if not self.cache.reserve(key, need):
                break
            self.blocked.popleft()
            self.in_setup.add(key)
            self.dispatch(key)
            n += 1
        return n

    def finished(self, key, solver):
        self.in_setup.discard(key)
        self.cache.insert(key, solver)

    def failed(self, key):
        self.in_setup.discard(key)
        self.cache.cancel(key)


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
    adm = SetupAdmission(cache, estimate, worker.jobs.put)
    by_tag = {r.tag: r for r in requests}
    setup_times = []
    hbm_peak = 0
    srv = H.Server(workspace_budget, max_requests=max_requests, max_nrhs=max_nrhs, restart=restart)
    counts0 = (cache.hits, cache.misses, cache.evictions, cache.overshoots, cache.over_budget)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nxt, done = 0, 0

    def now():
        return time.perf_counter() - t0

    def submit(r):
        r.t_submit = now()
        srv.submit(cache.acquire(r.key), r.f, r.tag)

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
                    adm.request(r.key)
            adm.pump()
            while True:
                try:
                    key, solver, dt, err = worker.results.get_nowait()
                except queue.Empty:
                    break
                if err is not None:
                    adm.failed(key)
                    raise err
                setup_times.append(dt)
                adm.finished(key, solver)
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
            if srv.stats()["live"] == 0 and nxt < len(requests) and not adm.in_setup:
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
                   evictions=cache.evictions - counts0[2], reservation_overshoots=cache.overshoots - counts0[3],
                   over_budget_inserts=cache.over_budget - counts0[4],
                   setups=len(setup_times), setup_ms_mean=float(np.mean(setup_times) * 1e3) if setup_times else 0.0,
                   hbm_peak_bytes=int(hbm_peak), iterations=stats["iterations"], captures=stats["captures"],
                   converged=all(i["converged"] for r in requests for i in r.info))
    return requests, summary
