"""Serving loop: Kemeny queries and edge-update batches on resident graphs.

Each graph keeps its CSR, tau0 and a resident sample set on the device
(``kc_samples_init``).  A query answers the estimate of Theorem 3.3 over the
graph's current trees (``kc_samples_query``); an update batch applies basic
(section 4.1, Algorithm 2) or improved (section 4.2, Algorithm 3) sample
maintenance (``kc_apply_updates``).

Scheduling (continuous batching): every graph has its own HIP stream and one
worker thread that takes that graph's requests in arrival order, so requests
on different graphs run on the device at the same time and a request is
started as soon as its graph is free and the HBM it may need is available.
Requests on one graph run in arrival order, so every graph's results are the
same alone and in any mix.  For comparison, ``one_at_a_time`` serves every
request in one worker, one after another (the plain form); ``set_schedule``
switches between the two on the same resident graphs.

Admission is by HBM footprint, against one device budget:
  - a resident graph holds, for as long as it is resident, its graph arrays
    (``kc_graph_info.device_bytes``), its trees (4 n bytes each) and their f
    values (16 bytes each), and the workspace the library may keep for it
    (its ``KC_OPT_MEM_BUDGET``: at most ``workspace_share``, and no more than
    its trees' worth of samples in flight, ``sample_bytes`` each);
  - an update additionally holds, while it runs, the temporary buffers the
    library allocates for it (at most two parent arrays per resident tree);
  - a query allocates nothing.
A graph is admitted only while the resident footprints, its own included,
leave room for the largest update of any resident graph: the bytes outside
the resident graphs then always hold that update, so an update waits at most
for the requests and initial draws running before it, never for good.  A
graph whose footprint can never fit is refused with KC_ERR_NOMEM; one that
does not fit now waits until removed graphs free memory (or is refused after
``timeout``).

This module only orchestrates calls into the HIP library; every step of the
estimator and of the maintenance runs in the library's kernels.
"""
from __future__ import annotations

import collections
import queue
import threading
import time
from dataclasses import dataclass, field

import numpy as np

from . import Graph, KC_OPT_MEM_BUDGET, KC_OPT_MAINTENANCE, KC_MAINT_BASIC, KcError


@dataclass
class Request:
    gid: int
    kind: str                      # "query" or "update"
    edges: list = field(default_factory=list)  # update: [(u, v), ...]
    insert: bool = False           # update: insert the edges (else delete them)
    t_arrive: float = 0.0
    t_start: float = 0.0
    t_done: float = 0.0
    result: object = None          # query: Estimate; update: trees replaced
    error: str = ""


class _Budget:
    """Device bytes held by resident graphs and by the requests in flight.

    free: bytes nothing holds now.  resident: the steady-state bytes of the
    admitted graphs.  reserves: the temporary bytes one update of each
    admitted graph may need; resident + max(reserves) never exceeds total."""

    def __init__(self, total: int):
        self.total = total
        self.free = total
        self.resident = 0
        self.reserves = collections.Counter()
        self.cv = threading.Condition()

    def largest_reserve(self) -> int:
        return max(self.reserves, default=0)

    def acquire(self, nbytes: int, timeout: float = None, hopeless=None, taken=None,
                steady: int = 0, reserve: int = 0) -> bool:
        """Take nbytes once they are free.  For a graph being admitted, steady
        is what it keeps resident and reserve what one of its updates may
        need: it also waits until the resident bytes with steady added still
        leave room for the largest reserve.  False after `timeout` seconds, at
        once if it could not fit even alone, or as soon as hopeless() says
        that nothing held now will be released; taken() runs under the same
        lock once the bytes are taken."""
        if nbytes > self.total or steady + reserve > self.total:
            return False
        end = None if timeout is None else time.perf_counter() + timeout

        def fits():
            if self.free < nbytes:
                return False
            return steady == 0 or self.resident + steady + max(self.largest_reserve(), reserve) <= self.total

        with self.cv:
            while not fits():
                left = None if end is None else end - time.perf_counter()
                if left is not None and left <= 0:
                    return False
                if hopeless is not None and hopeless():
                    return False
                self.cv.wait(left if hopeless is None else min(1.0, left) if left is not None else 1.0)
            self.free -= nbytes
            if steady:
                self.resident += steady
                self.reserves[reserve] += 1
            if taken is not None:
                taken()
        return True

    def release(self, nbytes: int, steady: int = 0, reserve: int = 0, then=None):
        """Return nbytes (for a graph leaving: also its steady bytes and its
        reserve); then() runs under the same lock, before the waiters wake."""
        with self.cv:
            self.free += nbytes
            if steady:
                self.resident -= steady
                self.reserves[reserve] -= 1
                if self.reserves[reserve] == 0:
                    del self.reserves[reserve]
            if then is not None:
                then()
            self.cv.notify_all()


def resident_bytes(info: dict, samples: int, workspace: int) -> int:
    """Device bytes a resident graph holds: graph arrays, `samples` parent
    arrays of 4 n bytes, their f (8 bytes, and 8 more for its recomputation
    buffer) and the workspace cap."""
    return int(info["device_bytes"]) + samples * (4 * int(info["n"]) + 16) + workspace


def update_bytes(info: dict, samples: int) -> int:
    """Temporary device bytes an update may allocate: replacement trees and the
    saved rows of transformed trees, each at most one parent array per tree."""
    return 2 * samples * 4 * int(info["n"])


class Server:
    """Resident graphs and their request workers."""

    def __init__(self, budget_bytes: int, workspace_share: int, maintenance: int = KC_MAINT_BASIC,
                 one_at_a_time: bool = False, init_share: int = 0):
        """budget_bytes: device bytes the server may hold in all; workspace_share:
        the most workspace one graph's estimates and updates may keep
        (KC_OPT_MEM_BUDGET); init_share: the workspace a graph may use while its
        resident trees are first drawn (freed afterwards; 0: workspace_share);
        one_at_a_time: the plain form for comparison, one worker for all graphs,
        so requests run strictly one after another."""
        self.one_at_a_time = one_at_a_time
        self.init_share = init_share
        self.budget = _Budget(budget_bytes)
        self.workspace_share = workspace_share
        self.maintenance = maintenance     # KC_MAINT_BASIC (Algorithm 2) or KC_MAINT_IMPROVED (Algorithm 3)
        self.graphs = {}
        self.held = {}       # gid -> resident bytes charged
        self.tmp = {}        # gid -> bytes an update of it charges
        self.queues = {}
        self.threads = {}
        self.streams = {}
        self.done = []
        self.done_cv = threading.Condition()
        self.submitted = 0
        self.solo_q = queue.Queue()    # the one queue of the plain form
        self.solo_t = None
        self.drawing = 0               # graphs drawing their resident trees now

    def add_graph(self, gid: int, g, seed: int, samples: int, timeout: float = None, hopeless=None):
        """Make g resident with `samples` trees once its footprint fits the
        budget (KcError KC_ERR_NOMEM if it never can, not within `timeout`, or
        once hopeless() is true while it waits)."""
        import torch
        stream = torch.cuda.Stream()
        G = Graph.from_graph(g, stream=stream)
        info = G.info
        workspace = min(self.workspace_share, samples * int(info["sample_bytes"]))
        init_ws = max(workspace, min(self.init_share, samples * int(info["sample_bytes"])))
        need = resident_bytes(info, samples, workspace)
        need_init = resident_bytes(info, samples, init_ws)

        tmp = update_bytes(info, samples)

        def drawing_starts():
            self.drawing += 1

        def drawing_ends():
            self.drawing -= 1

        if not self.budget.acquire(need_init, timeout, hopeless, taken=drawing_starts, steady=need, reserve=tmp):
            G.close()
            raise KcError(3, "graph %s needs %d device bytes resident and %d for an update; %d of %d are free, "
                          "%d held resident" % (gid, need_init, tmp, self.budget.free, self.budget.total,
                                                self.budget.resident))
        try:
            G.set_option(KC_OPT_MEM_BUDGET, init_ws)
            G.set_option(KC_OPT_MAINTENANCE, self.maintenance)
            G.samples_init(seed, samples, stream=stream)
            if init_ws > workspace:
                # keep only the steady-state workspace: the rest returns to the budget
                G.trim(stream)
                G.set_option(KC_OPT_MEM_BUDGET, workspace)
        except Exception:
            G.close()
            self.budget.release(need_init, steady=need, reserve=tmp, then=drawing_ends)
            raise
        # the end of the draw and the bytes it returns are seen together
        self.budget.release(need_init - need, then=drawing_ends)
        with self.done_cv:
            self.graphs[gid] = G
            self.held[gid] = need
            self.tmp[gid] = tmp
            self.streams[gid] = stream
            q = queue.Queue()
            self.queues[gid] = q
            t = threading.Thread(target=self._worker, args=(q,), daemon=True)
            self.threads[gid] = t
        t.start()

    def add_graphs(self, items, workers: int = 8, on_added=None):
        """add_graph for many (gid, g, seed, samples) at once, `workers` at a
        time: their resident trees are drawn concurrently, each on its own
        stream.  on_added(gid, seconds, error) is called as each one ends.
        Returns {gid: error message} for the graphs refused."""
        from concurrent.futures import ThreadPoolExecutor
        errors = {}

        def one(item):
            gid, g, seed, samples = item
            t0 = time.perf_counter()
            err = None
            try:
                # a graph waits for memory only while another one is drawing its trees
                # (which then returns its extra workspace)
                self.add_graph(gid, g, seed=seed, samples=samples, hopeless=lambda: self.drawing == 0)
            except KcError as exc:
                err = errors[gid] = str(exc)
            if on_added:
                on_added(gid, time.perf_counter() - t0, err)

        with ThreadPoolExecutor(max_workers=max(1, workers)) as pool:
            list(pool.map(one, items))
        return errors

    def set_schedule(self, one_at_a_time: bool):
        """Switch between per-graph workers (continuous batching) and the plain
        form; requests already submitted finish under the old schedule first."""
        self.drain()
        self.one_at_a_time = one_at_a_time

    def remove_graph(self, gid: int):
        """Free a resident graph once every request submitted so far (on any
        graph) is done; its bytes and its update reserve return to the budget
        and its worker ends."""
        self.drain()
        with self.done_cv:
            q = self.queues.pop(gid)
            t = self.threads.pop(gid)
        q.put(None)
        t.join()
        G = self.graphs.pop(gid)
        G.close()
        self.streams.pop(gid, None)
        held = self.held.pop(gid)
        self.budget.release(held, steady=held, reserve=self.tmp.pop(gid))

    def submit(self, req: Request):
        with self.done_cv:
            self.submitted += 1
        req.t_arrive = time.perf_counter()
        if self.one_at_a_time:
            if self.solo_t is None:
                self.solo_t = threading.Thread(target=self._worker, args=(self.solo_q,), daemon=True)
                self.solo_t.start()
            self.solo_q.put(req)
        else:
            self.queues[req.gid].put(req)

    def _worker(self, q):
        while True:
            req = q.get()
            if req is None:
                return
            G = self.graphs[req.gid]
            stream = self.streams[req.gid]
            held = 0
            try:
                if req.kind == "update":
                    held = self.tmp[req.gid]
                    if not self.budget.acquire(held):
                        held = 0
                        raise KcError(3, "an update of graph %s needs %d temporary device bytes, more than "
                                      "the whole budget" % (req.gid, self.tmp[req.gid]))
                req.t_start = time.perf_counter()
                if req.kind == "query":
                    req.result = G.samples_query(stream=stream)
                else:
                    req.result = G.apply_updates([a for a, _ in req.edges], [b for _, b in req.edges],
                                                 [1 if req.insert else 0] * len(req.edges), stream=stream)
            except KcError as exc:
                req.error = str(exc)
            finally:
                if held:
                    self.budget.release(held)
            req.t_done = time.perf_counter()
            with self.done_cv:
                self.done.append(req)
                self.done_cv.notify_all()

    def drain(self, timeout: float = None) -> int:
        """Wait until every submitted request has finished (or `timeout` seconds
        pass); returns how many have finished."""
        end = None if timeout is None else time.perf_counter() + timeout
        with self.done_cv:
            while len(self.done) < self.submitted:
                left = None if end is None else end - time.perf_counter()
                if left is not None and left <= 0:
                    break
                self.done_cv.wait(left)
            return len(self.done)

    def close(self):
        for q in list(self.queues.values()) + [self.solo_q]:
            q.put(None)
        for t in list(self.threads.values()) + ([self.solo_t] if self.solo_t else []):
            t.join()
        for gid, G in self.graphs.items():
            G.close()
            held = self.held.get(gid, 0)
            self.budget.release(held, steady=held, reserve=self.tmp.get(gid, 0))
        self.graphs.clear()
        self.held.clear()
        self.tmp.clear()


def latency_stats(reqs, kind: str):
    lat = np.array([(r.t_done - r.t_arrive) * 1e3 for r in reqs if r.kind == kind and not r.error])
    if lat.size == 0:
        return None
    return {"count": int(lat.size), "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean())}
