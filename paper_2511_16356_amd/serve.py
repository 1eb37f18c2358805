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
Admission is by HBM footprint: an update may allocate at most its share of
the device budget (``KC_OPT_MEM_BUDGET``), and it starts only when that
share is free; queries need no workspace.  Requests on one graph run in
arrival order, so every graph's results are the same alone and in any mix.
For comparison, ``one_at_a_time`` serves every request in one worker, one
after another (the plain form).

This module only orchestrates calls into the HIP library; every step of the
estimator and of the maintenance runs in the library's kernels.
"""
from __future__ import annotations

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
    """Device bytes shared by the requests in flight."""

    def __init__(self, total: int):
        self.total = total
        self.free = total
        self.cv = threading.Condition()

    def acquire(self, nbytes: int):
        nbytes = min(nbytes, self.total)
        with self.cv:
            while self.free < nbytes:
                self.cv.wait()
            self.free -= nbytes
        return nbytes

    def release(self, nbytes: int):
        with self.cv:
            self.free += nbytes
            self.cv.notify_all()


class Server:
    """Resident graphs and their request workers."""

    def __init__(self, budget_bytes: int, update_share: int, maintenance: int = KC_MAINT_BASIC,
                 one_at_a_time: bool = False):
        """one_at_a_time: the plain form for comparison, one worker for all
        graphs, so requests run strictly one after another in arrival order."""
        self.one_at_a_time = one_at_a_time
        self.budget = _Budget(budget_bytes)
        self.update_share = update_share   # device bytes one update may use
        self.maintenance = maintenance     # KC_MAINT_BASIC (Algorithm 2) or KC_MAINT_IMPROVED (Algorithm 3)
        self.graphs = {}
        self.queues = {}
        self.threads = {}
        self.streams = {}
        self.done = []
        self.done_cv = threading.Condition()
        self.submitted = 0

    def add_graph(self, gid: int, g, seed: int, samples: int):
        import torch
        stream = torch.cuda.Stream()
        G = Graph.from_graph(g, stream=stream)
        G.set_option(KC_OPT_MEM_BUDGET, self.update_share)
        G.set_option(KC_OPT_MAINTENANCE, self.maintenance)
        G.samples_init(seed, samples, stream=stream)
        self.graphs[gid] = G
        self.streams[gid] = stream
        if self.one_at_a_time and self.threads:
            self.queues[gid] = next(iter(self.queues.values()))
            return
        q = queue.Queue()
        self.queues[gid] = q
        t = threading.Thread(target=self._worker, args=(q,), daemon=True)
        self.threads[gid] = t
        t.start()

    def submit(self, req: Request):
        with self.done_cv:
            self.submitted += 1
        req.t_arrive = time.perf_counter()
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
                    held = self.budget.acquire(self.update_share)
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
        for q in {id(q): q for q in self.queues.values()}.values():
            q.put(None)
        for t in self.threads.values():
            t.join()
        for G in self.graphs.values():
            G.close()
        self.graphs.clear()


def latency_stats(reqs, kind: str):
    lat = np.array([(r.t_done - r.t_arrive) * 1e3 for r in reqs if r.kind == kind and not r.error])
    if lat.size == 0:
        return None
    return {"count": int(lat.size), "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean())}
