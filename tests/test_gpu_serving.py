"""Serving loop: every graph's results are the same alone and in a mix of
graphs served at the same time (requests on one graph keep their order;
requests on different graphs overlap on the device)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def kc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2511_16356_amd as kc
    kc.library()
    return kc


def _ops(gen, g, seed, rounds):
    """A fixed request sequence for one graph: query, update (a deletion batch
    or an insertion batch), query, ..."""
    rng = np.random.default_rng(seed)
    ops = [("query", None, False)]
    for k in range(rounds):
        if k % 2 == 0:
            batch = gen.deletion_batch(g, [1, 7, 60][k % 3], rng)
            g = gen.remove_edges(g, batch)
            ops += [("update", batch, False), ("query", None, False)]
        else:
            batch = gen.insertion_batch(g, 2, rng)
            g = gen.add_edges(g, batch)
            ops += [("update", batch, True), ("query", None, False)]
    return ops


def _serve(kc, graphs, ops, order, maintenance=0, one_at_a_time=False):
    from paper_2511_16356_amd.serve import Server, Request
    srv = Server(budget_bytes=8 << 30, workspace_share=2 << 30, maintenance=maintenance, one_at_a_time=one_at_a_time)
    try:
        for gid in graphs:
            srv.add_graph(gid, graphs[gid], seed=100 + gid, samples=128)
        reqs = []
        for gid, k in order:
            kind, batch, ins = ops[gid][k]
            r = Request(gid, kind, batch or [], insert=ins)
            reqs.append(r)
            srv.submit(r)
        srv.drain()
        for r in reqs:
            assert not r.error, r.error
        out = {gid: [] for gid in graphs}
        for r in reqs:
            if r.kind == "query":
                out[r.gid].append((r.result.kappa, r.result.sum_f, r.result.sum_f2))
            else:
                out[r.gid].append(r.result)
        return out
    finally:
        srv.close()


@pytest.mark.parametrize("maintenance", [0, 1], ids=["basic", "improved"])
def test_same_alone_and_in_the_mix(kc, gen, maintenance):
    graphs = {0: gen.grid(40, 40), 1: gen.road_like(3000, seed=4), 2: gen.chung_lu(2000, 2.2, 10.0, 200.0, seed=6)}
    ops = {gid: _ops(gen, graphs[gid], 10 + gid, 4) for gid in graphs}
    # interleaved arrival across graphs (round robin), all submitted at once
    steps = max(len(v) for v in ops.values())
    mixed_order = [(gid, k) for k in range(steps) for gid in graphs if k < len(ops[gid])]
    _say("mix", len(mixed_order), "requests")
    mixed = _serve(kc, graphs, ops, mixed_order, maintenance)
    _say("one at a time", len(mixed_order), "requests")
    assert _serve(kc, graphs, ops, mixed_order, maintenance, one_at_a_time=True) == mixed
    for gid in graphs:
        _say("alone", gid)
        alone = _serve(kc, {gid: graphs[gid]}, ops, [(gid, k) for k in range(len(ops[gid]))], maintenance)
        assert alone[gid] == mixed[gid]
