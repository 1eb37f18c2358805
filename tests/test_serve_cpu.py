"""Host logic of the serving loop (paper_2511_16356_amd.serve), on the CPU:
the graphs and streams are replaced by stand-ins that record what runs when,
so the scheduling rules can be checked without a device.  Also the
benchmark's host helpers: exact kappa against closed forms, the serving
mix's request plans, the algorithmic byte count, the oracle leg's record,
and the refusal of more than one GPU."""
import threading
import time

import pytest


class _FakeStream:
    cuda_stream = 0


def _opt_mem_budget():
    from paper_2511_16356_amd import KC_OPT_MEM_BUDGET
    return KC_OPT_MEM_BUDGET


class _FakeGraph:
    """Records (gid, kind, start, end) of every call; updates take longer."""
    log = []
    lock = threading.Lock()
    running = 0
    max_running = 0

    info = {"n": 1024, "device_bytes": 100000, "sample_bytes": 100}

    def __init__(self, gid):
        self.gid = gid
        self.options = {}
        self.inits = 0
        self.closed = False

    @classmethod
    def from_graph(cls, g, stream=None):
        return cls(g)

    def set_option(self, opt, value):
        self.options[opt] = value

    def samples_init(self, seed, count, stream=None):
        self.inits += 1
        self.init_budget = self.options.get(_opt_mem_budget())

    def trim(self, stream=None):
        self.trimmed = True

    def _run(self, kind, seconds):
        with _FakeGraph.lock:
            _FakeGraph.running += 1
            _FakeGraph.max_running = max(_FakeGraph.max_running, _FakeGraph.running)
            t0 = time.perf_counter()
        time.sleep(seconds)
        with _FakeGraph.lock:
            _FakeGraph.running -= 1
            _FakeGraph.log.append((self.gid, kind, t0, time.perf_counter()))

    def samples_query(self, stream=None):
        self._run("query", 0.01)
        return "estimate"

    def apply_updates(self, u, v, is_insert, stream=None):
        if u and u[0] < 0:
            from paper_2511_16356_amd import KcError
            raise KcError(1, "bad edge")
        self._run("update", 0.05)
        return len(u)

    def close(self):
        self.closed = True


@pytest.fixture
def serve(monkeypatch):
    import torch
    import paper_2511_16356_amd.serve as serve
    monkeypatch.setattr(serve, "Graph", _FakeGraph)
    monkeypatch.setattr(torch.cuda, "Stream", lambda *a, **k: _FakeStream())
    _FakeGraph.log = []
    _FakeGraph.running = 0
    _FakeGraph.max_running = 0
    return serve


def _submit_all(srv, serve, plan):
    reqs = []
    for gid, kind in plan:
        r = serve.Request(gid, kind, [(1, 2)] if kind == "update" else [])
        reqs.append(r)
        srv.submit(r)
    assert srv.drain(timeout=30.0) == len(reqs)
    return reqs


def test_requests_on_one_graph_keep_their_order(serve):
    srv = serve.Server(budget_bytes=1 << 30, workspace_share=1 << 20)
    try:
        for gid in range(3):
            srv.add_graph(gid, gid, seed=gid, samples=8)
        plan = [(k % 3, "update" if k % 4 == 1 else "query") for k in range(24)]
        reqs = _submit_all(srv, serve, plan)
        assert all(not r.error for r in reqs)
        for gid in range(3):
            mine = [r for r in reqs if r.gid == gid]
            starts = [r.t_start for r in mine]
            assert starts == sorted(starts)
            for a, b in zip(mine, mine[1:]):
                assert a.t_done <= b.t_start + 1e-6  # one after another on a graph
        # different graphs overlap
        assert _FakeGraph.max_running > 1
    finally:
        srv.close()


def _resident(serve, samples=8, share=1 << 20):
    info = _FakeGraph.info
    return serve.resident_bytes(info, samples, min(share, samples * info["sample_bytes"]))


def test_update_budget_admits_one_update_at_a_time(serve):
    # a budget that holds the four resident graphs and exactly one update's
    # temporaries: updates never overlap
    tmp = serve.update_bytes(_FakeGraph.info, 8)
    srv = serve.Server(budget_bytes=4 * _resident(serve) + tmp, workspace_share=1 << 20)
    try:
        for gid in range(4):
            srv.add_graph(gid, gid, seed=gid, samples=8)
        reqs = _submit_all(srv, serve, [(gid, "update") for gid in range(4)] * 2)
        ups = sorted((s, e) for g, k, s, e in _FakeGraph.log if k == "update")
        assert len(ups) == 8
        for (s0, e0), (s1, e1) in zip(ups, ups[1:]):
            assert e0 <= s1 + 1e-6
        assert srv.budget.free == srv.budget.total - 4 * _resident(serve)
        assert all(r.result == 1 for r in reqs)
    finally:
        srv.close()


def test_one_at_a_time_runs_in_arrival_order(serve):
    srv = serve.Server(budget_bytes=1 << 30, workspace_share=1 << 20, one_at_a_time=True)
    try:
        for gid in range(3):
            srv.add_graph(gid, gid, seed=gid, samples=8)
        plan = [(k % 3, "update" if k % 3 == 0 else "query") for k in range(12)]
        reqs = _submit_all(srv, serve, plan)
        assert srv.solo_t is not None
        assert _FakeGraph.max_running == 1
        for a, b in zip(reqs, reqs[1:]):
            assert a.t_done <= b.t_start + 1e-6
    finally:
        srv.close()


def test_schedule_switches_on_the_same_graphs(serve):
    """The plain form and continuous batching on the same resident graphs:
    one request at a time, then requests on different graphs overlapping."""
    srv = serve.Server(budget_bytes=1 << 30, workspace_share=1 << 20)
    try:
        errors = srv.add_graphs([(gid, gid, gid, 8) for gid in range(4)], workers=4)
        assert errors == {} and sorted(srv.graphs) == [0, 1, 2, 3]
        srv.set_schedule(True)
        _submit_all(srv, serve, [(gid, "update") for gid in range(4)])
        assert _FakeGraph.max_running == 1
        srv.set_schedule(False)
        for gid in range(4):
            srv.submit(serve.Request(gid, "update", [(1, 2)]))
        assert srv.drain(timeout=30.0) == 8
        assert _FakeGraph.max_running > 1
    finally:
        srv.close()


def test_concurrent_admission_refuses_what_cannot_fit(serve):
    """Graphs admitted together wait for memory only while another graph is
    drawing its trees: one that cannot fit beside the resident ones is refused
    as soon as nothing is left to free, instead of waiting forever."""
    one = _resident(serve)
    srv = serve.Server(budget_bytes=int(2.5 * one), workspace_share=1 << 20)
    try:
        t0 = time.perf_counter()
        errors = srv.add_graphs([(gid, gid, gid, 8) for gid in range(3)], workers=3)
        assert time.perf_counter() - t0 < 10.0
        assert len(srv.graphs) == 2 and len(errors) == 1
        assert all("KC_ERR_NOMEM" in e or "needs" in e for e in errors.values())
        assert srv.budget.free == srv.budget.total - 2 * one
    finally:
        srv.close()


def test_init_share_is_returned_after_the_trees_are_drawn(serve):
    """A graph may draw its resident trees with a larger workspace than it
    keeps: the difference is charged while the trees are drawn, then trimmed
    and returned to the budget."""
    srv = serve.Server(budget_bytes=1 << 30, workspace_share=300, init_share=1 << 20)
    try:
        srv.add_graph(0, 0, seed=0, samples=8)
        G = srv.graphs[0]
        assert G.init_budget == 8 * 100 and getattr(G, "trimmed", False)
        assert G.options[serve.KC_OPT_MEM_BUDGET] == 300
        assert srv.budget.free == srv.budget.total - _resident(serve, share=300)
    finally:
        srv.close()


def test_errors_are_reported_and_release_the_budget(serve):
    srv = serve.Server(budget_bytes=_resident(serve) + serve.update_bytes(_FakeGraph.info, 8),
                       workspace_share=1 << 20)
    try:
        srv.add_graph(0, 0, seed=0, samples=8)
        bad = serve.Request(0, "update", [(-1, 2)])
        good = serve.Request(0, "update", [(1, 2)])
        srv.submit(bad)
        srv.submit(good)
        assert srv.drain(timeout=30.0) == 2
        assert "KC_ERR_INVALID" in bad.error and good.error == "" and good.result == 1
        assert srv.budget.free == srv.budget.total - _resident(serve)
    finally:
        srv.close()


def test_maintenance_option_reaches_every_graph(serve):
    from paper_2511_16356_amd import KC_OPT_MAINTENANCE, KC_MAINT_IMPROVED
    srv = serve.Server(budget_bytes=1 << 30, workspace_share=1 << 20, maintenance=KC_MAINT_IMPROVED)
    try:
        for gid in range(2):
            srv.add_graph(gid, gid, seed=gid, samples=8)
        for G in srv.graphs.values():
            assert G.options[KC_OPT_MAINTENANCE] == KC_MAINT_IMPROVED and G.inits == 1
    finally:
        srv.close()


def test_admission_by_resident_footprint(serve):
    """Each resident graph holds its graph arrays, trees, f and workspace cap for
    as long as it is resident: a graph that does not fit waits, and is refused
    with KC_ERR_NOMEM after its timeout; removing a graph frees its bytes; a
    graph larger than the whole budget is refused at once."""
    from paper_2511_16356_amd import KcError
    one = _resident(serve)
    assert one == 100000 + 8 * (4 * 1024 + 16) + 8 * 100
    srv = serve.Server(budget_bytes=2 * one + serve.update_bytes(_FakeGraph.info, 8), workspace_share=1 << 20)
    try:
        srv.add_graph(0, 0, seed=0, samples=8)
        srv.add_graph(1, 1, seed=1, samples=8)
        assert srv.graphs[0].options[serve.KC_OPT_MEM_BUDGET] == 8 * 100  # workspace cap: its samples
        t0 = time.perf_counter()
        with pytest.raises(KcError) as ei:
            srv.add_graph(2, 2, seed=2, samples=8, timeout=0.2)
        assert ei.value.status == 3 and time.perf_counter() - t0 >= 0.19
        # an update's temporaries still fit beside the two graphs
        reqs = _submit_all(srv, serve, [(0, "update"), (1, "update"), (1, "query")])
        assert all(not r.error for r in reqs)
        srv.remove_graph(0)
        srv.add_graph(2, 2, seed=2, samples=8, timeout=0.2)
        assert srv.budget.free == srv.budget.total - 2 * one
        with pytest.raises(KcError) as ei:
            srv.add_graph(3, 3, seed=3, samples=10 ** 6, timeout=None)  # never fits: refused at once
        assert ei.value.status == 3
    finally:
        srv.close()
    assert srv.budget.free == srv.budget.total


def test_admission_keeps_room_for_an_update(serve):
    """A budget that would hold two resident graphs but not, beside them, the
    temporaries of one update: the second graph is refused, so the first
    graph's updates still run instead of waiting for good.  The reserve goes
    when its graph does."""
    from paper_2511_16356_amd import KcError
    one = _resident(serve)
    tmp = serve.update_bytes(_FakeGraph.info, 8)
    srv = serve.Server(budget_bytes=2 * one + tmp // 2, workspace_share=1 << 20)
    try:
        srv.add_graph(0, 0, seed=0, samples=8)
        assert srv.budget.resident == one and srv.budget.largest_reserve() == tmp
        with pytest.raises(KcError) as ei:
            srv.add_graph(1, 1, seed=1, samples=8, timeout=0.2)
        assert ei.value.status == 3 and "for an update" in str(ei.value)
        reqs = _submit_all(srv, serve, [(0, "update"), (0, "query"), (0, "update")])
        assert all(not r.error for r in reqs) and [r.result for r in reqs] == [1, "estimate", 1]
        # a smaller graph whose own update fits beside the first graph's reserve is admitted
        small = dict(_FakeGraph.info, n=16, device_bytes=1000)
        need = serve.resident_bytes(small, 8, 8 * 100)
        assert one + need + tmp <= srv.budget.total
        orig = _FakeGraph.info
        _FakeGraph.info = small
        try:
            srv.add_graph(2, 2, seed=2, samples=8, timeout=0.2)
        finally:
            _FakeGraph.info = orig
        assert srv.budget.resident == one + need and srv.budget.largest_reserve() == tmp
        srv.remove_graph(0)
        assert srv.budget.resident == need and srv.budget.largest_reserve() == serve.update_bytes(small, 8)
    finally:
        srv.close()
    assert srv.budget.free == srv.budget.total and srv.budget.resident == 0 and srv.budget.largest_reserve() == 0


def test_bench_exact_kemeny_closed_forms(gen):
    import bench
    for n in (3, 5, 9):
        g = gen.complete(n)
        assert bench.exact_kemeny(g.offsets, g.indices) == pytest.approx((n - 1) ** 2 / n, rel=1e-12)
    for n in (5, 8, 13):
        g = gen.cycle(n)
        assert bench.exact_kemeny(g.offsets, g.indices) == pytest.approx((n * n - 1) / 6, rel=1e-12)
    from oracle import exact as E
    g = gen.grid(32, 32)
    assert bench.exact_kemeny(g.offsets, g.indices) == pytest.approx(E.kemeny_exact(g.offsets, g.indices), rel=1e-12)


def test_bench_request_plans(gen):
    """The serving mix's request plans: the same seed gives the same plan,
    about 80% queries and 20% update batches, deletions of at most 1,000 and
    insertions of at most 10 edges, arrival times increasing at the offered
    rate (all at zero when saturated), and each update applied to the
    planned graph so that later updates see it."""
    import numpy as np
    import bench
    import graphgen
    base = [graphgen.road_like(3000, seed=1), gen.grid(12, 12)]
    plans = []
    for _ in range(2):
        cur = list(base)
        plans.append(bench.plan_requests(cur, 200, 50.0, np.random.default_rng(5)))
    a, b = plans
    assert [(t, g, k, len(e), i) for t, g, k, e, i in a] == [(t, g, k, len(e), i) for t, g, k, e, i in b]
    kinds = [k for _, _, k, _, _ in a]
    assert 0.7 < kinds.count("query") / len(kinds) < 0.9
    times = [t for t, _, _, _, _ in a]
    assert all(x < y for x, y in zip(times, times[1:]))
    assert 2.0 < times[-1] < 6.0  # 200 requests at 50 per second
    ups = [(e, ins) for _, _, kind, e, ins in a if kind == "update"]
    # a deletion batch that would disconnect the graph is halved, possibly to nothing
    assert all(len(e) <= (10 if ins else 1000) for e, ins in ups)
    assert sum(1 for e, _ in ups if e) >= len(ups) // 2
    cur = list(base)
    sat = bench.plan_requests(cur, 40, 1.0, np.random.default_rng(6), saturate=True)
    assert all(t == 0.0 for t, _, _, _, _ in sat)
    removed = sum(len(e) for _, _, k, e, ins in sat if k == "update" and not ins)
    added = sum(len(e) for _, _, k, e, ins in sat if k == "update" and ins)
    assert sum(g.two_m for g in cur) == sum(g.two_m for g in base) - 2 * removed + 2 * added


def test_bench_algorithmic_bytes():
    import bench
    # one sector per draw, per vertex (joining the tree), and per path-mapping term
    assert bench.algorithmic_bytes(draws=100, n=8, two_m=20, depth0=2, samples=3) == 64 * (100 + 3 * (8 + 8 * 2))
    assert bench.algorithmic_bytes(draws=0, n=1024, two_m=3968, depth0=60, samples=1) == 64 * (1024 + 1024 * 10)
    # a CSR larger than the last-level cache adds its offset and neighbour sectors to every draw
    n, two_m = 3_000_000, 227_000_000
    assert bench.algorithmic_bytes(draws=100, n=n, two_m=two_m, depth0=3, samples=1) == 64 * (300 + n + 3 * n)


def test_bench_refuses_more_than_one_gpu():
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_bench_cpu_baseline_record(gen):
    """The oracle leg of the benchmark on a tiny graph: a positive rate over
    exactly threads x per_thread samples when that pass is long enough, and
    the host it ran on; a pass shorter than min_s is followed by the next ids,
    in whole rounds of the thread count, up to about target_s of work."""
    import bench
    g = gen.grid(6, 6)
    rec = bench.cpu_baseline(g, seed=3, first=10, threads=2, per_thread=3, what="the 6x6 grid", min_s=0.0)
    assert rec["kind"] == "oracle" and rec["unit"] == "samples/s" and rec["cores"] == 2
    assert rec["value"] > 0 and rec["nproc"] >= 1
    assert rec["sample"].startswith("samples 10..15 of the 6x6 grid (6 on 2 threads)")
    rec = bench.cpu_baseline(g, seed=3, first=10, threads=2, per_thread=3, what="the 6x6 grid",
                             min_s=0.05, target_s=0.1)
    first, last = (int(x) for x in rec["sample"].split()[1].split(".."))
    count = last - first + 1
    assert first == 10 and count > 6 and count % 2 == 0 and count <= 6 + 2 * 64 * 3
    assert "(%d on 2 threads)" % count in rec["sample"]
