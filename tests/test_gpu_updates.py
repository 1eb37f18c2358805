"""GPU parity of basic sample maintenance (section 4.1, Algorithm 2, deletion
case) against the oracle: after every batch of edge deletions the resident
trees, their sample indices, their f on the new graph and the estimate are
identical to the oracle's."""
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


def deletion_batches(gen, g, sizes, seed):
    """Seeded batches of distinct edges whose removal keeps the graph connected:
    candidates in a seeded random order, each kept if the graph stays connected."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import connected_components
    rng = np.random.default_rng(seed)
    out = []
    for size in sizes:
        src = np.repeat(np.arange(g.n), np.diff(g.offsets))
        mask = src < g.indices
        eu, ev = src[mask], g.indices[mask]
        batch = []
        for i in rng.permutation(eu.shape[0]):
            trial = batch + [(int(eu[i]), int(ev[i]))]
            g2 = gen.remove_edges(g, trial)
            a = csr_matrix((np.ones(g2.indices.shape[0]), g2.indices, g2.offsets), shape=(g2.n, g2.n))
            if connected_components(a, directed=False)[0] == 1:
                batch = trial
                if len(batch) == size:
                    break
        assert len(batch) == size
        out.append(batch)
        g = gen.remove_edges(g, batch)
    return out


def _compare(G, S, two_m):
    par, f, ids = G.samples_get()
    assert np.array_equal(ids, S.ids)
    assert np.array_equal(par.cpu().numpy(), S.parents)
    assert np.array_equal(f.cpu().numpy(), S.f)
    assert G.two_m == two_m


@pytest.mark.parametrize("name", ["grid32", "road3k", "social3k"])
def test_bsm_deletions_match_oracle(kc, oracle_lib, gen, name):
    from test_gpu_parity import small_graphs
    g = small_graphs(gen)[name]
    count = 64
    S = oracle_lib.samples_init(g.offsets, g.indices, seed=11, count=count)
    with kc.Graph.from_graph(g) as G:
        G.samples_init(11, count)
        _compare(G, S, g.two_m)
        for batch in deletion_batches(gen, g, [1, 5, 40], seed=3):
            _say(name, "delete", len(batch))
            g = gen.remove_edges(g, batch)
            S, ref_k = oracle_lib.bsm_delete(S, g.offsets, g.indices, batch)
            k = G.apply_updates([a for a, _ in batch], [b for _, b in batch])
            assert k == ref_k
            _compare(G, S, g.two_m)
            est = G.samples_query()
            K, se, s1, s2 = oracle_lib.reduce_estimate(S.f, g.two_m)
            assert est.sum_f == s1 and est.sum_f2 == s2
            assert est.kappa == K and est.std_error == se


def test_rejected_updates_change_nothing(kc, gen):
    from test_gpu_parity import small_graphs
    g = small_graphs(gen)["road3k"]
    deg = np.diff(g.offsets)
    leaf = int(np.nonzero(deg == 1)[0][0])
    nb = int(g.indices[g.offsets[leaf]])
    with kc.Graph.from_graph(g) as G:
        G.samples_init(2, 16)
        par0, f0, ids0 = G.samples_get()
        with pytest.raises(kc.KcError) as ei:   # a bridge: G' would be disconnected
            G.apply_updates([leaf], [nb])
        assert ei.value.status == 2
        with pytest.raises(kc.KcError) as ei:   # not an edge
            G.apply_updates([0], [g.n - 1] if g.n - 1 not in g.indices[g.offsets[0]:g.offsets[1]] else [0])
        assert ei.value.status == 1
        with pytest.raises(kc.KcError) as ei:   # inserting an existing edge
            G.apply_updates([leaf], [nb], is_insert=[1])
        assert ei.value.status == 1
        par1, f1, ids1 = G.samples_get()
        assert np.array_equal(par0.cpu().numpy(), par1.cpu().numpy())
        assert np.array_equal(f0.cpu().numpy(), f1.cpu().numpy())
        assert np.array_equal(ids0, ids1) and G.two_m == g.two_m


def test_update_failing_after_the_switch_changes_nothing(kc, oracle_lib, gen):
    """A deletion whose replacement trees hit the step limit (forced from the
    host: a limit of 50 sampler rounds) fails after the graph was switched;
    the graph, the trees and their f are then as before, and the same update
    succeeds once the limit is lifted.  Earlier updates of the same call stay
    applied."""
    from test_gpu_parity import small_graphs
    g = small_graphs(gen)["road3k"]
    count = 32
    S = oracle_lib.samples_init(g.offsets, g.indices, seed=4, count=count)
    b1, b2 = deletion_batches(gen, g, [3, 40], seed=12)
    with kc.Graph.from_graph(g) as G:
        G.samples_init(4, count)
        G.set_option(kc.KC_OPT_STEP_LIMIT, 50)
        with pytest.raises(kc.KcError) as ei:
            G.apply_updates([a for a, _ in b1], [b for _, b in b1])
        assert ei.value.status == 6
        _compare(G, S, g.two_m)
        # lifted: the same run applies; then a failing run after a good one
        G.set_option(kc.KC_OPT_STEP_LIMIT, 0)
        G.apply_updates([a for a, _ in b1], [b for _, b in b1])
        g = gen.remove_edges(g, b1)
        S, _ = oracle_lib.bsm_delete(S, g.offsets, g.indices, b1)
        _compare(G, S, g.two_m)
        G.set_option(kc.KC_OPT_STEP_LIMIT, 50)
        with pytest.raises(kc.KcError) as ei:
            G.apply_updates([a for a, _ in b2], [b for _, b in b2])
        assert ei.value.status == 6
        _compare(G, S, g.two_m)
        est = G.samples_query()
        K, se, s1, s2 = oracle_lib.reduce_estimate(S.f, g.two_m)
        assert est.sum_f == s1 and est.kappa == K
        G.set_option(kc.KC_OPT_STEP_LIMIT, 0)


def _mixed_plan(gen, g, seed, steps):
    """A seeded list of updates: runs of deletions (that keep the graph connected)
    and single insertions of new edges."""
    rng = np.random.default_rng(seed)
    plan = []
    for k in range(steps):
        if k % 2 == 0:
            while True:
                a, b = (int(x) for x in rng.integers(0, g.n, size=2))
                if a != b and b not in g.indices[g.offsets[a]:g.offsets[a + 1]]:
                    break
            plan.append(("add", [(a, b)]))
            g = gen.add_edges(g, [(a, b)])
        else:
            batch = gen.deletion_batch(g, [3, 20][(k // 2) % 2], rng)
            plan.append(("del", batch))
            g = gen.remove_edges(g, batch)
    return plan


@pytest.mark.parametrize("name", ["grid32", "road3k", "social3k"])
def test_bsm_insertions_and_deletions_match_oracle(kc, oracle_lib, gen, name):
    from test_gpu_parity import small_graphs
    g = small_graphs(gen)[name]
    count = 64
    S = oracle_lib.samples_init(g.offsets, g.indices, seed=17, count=count)
    serial = 0
    with kc.Graph.from_graph(g) as G:
        G.samples_init(17, count)
        for kind, edges in _mixed_plan(gen, g, 5, 8):
            _say(name, kind, len(edges))
            if kind == "add":
                (a, b), = edges
                g = gen.add_edges(g, edges)
                S, ref_k, _ = oracle_lib.bsm_insert(S, g.offsets, g.indices, a, b, serial)
                serial += 1
                k = G.apply_updates([a], [b], is_insert=[1])
            else:
                g = gen.remove_edges(g, edges)
                S, ref_k = oracle_lib.bsm_delete(S, g.offsets, g.indices, edges)
                k = G.apply_updates([a for a, _ in edges], [b for _, b in edges])
            assert k == ref_k
            _compare(G, S, g.two_m)
        est = G.samples_query()
        K, se, s1, s2 = oracle_lib.reduce_estimate(S.f, g.two_m)
        assert est.sum_f == s1 and est.kappa == K and est.std_error == se


def test_one_call_runs_in_order(kc, oracle_lib, gen):
    """A single call with insertions and deletions equals applying, in order,
    each insertion alone and each run of consecutive deletions at once."""
    from test_gpu_parity import small_graphs
    g = small_graphs(gen)["grid32"]
    ups = [(5, 900, 1), (0, 1, 0), (1, 2, 0), (40, 75, 1), (2, 34, 0)]
    groups = [[ups[0]], [ups[1], ups[2]], [ups[3]], [ups[4]]]
    with kc.Graph.from_graph(g) as G1, kc.Graph.from_graph(g) as G2:
        G1.samples_init(3, 32)
        G2.samples_init(3, 32)
        k1 = G1.apply_updates([a for a, _, _ in ups], [b for _, b, _ in ups], [i for _, _, i in ups])
        k2 = 0
        for grp in groups:
            k2 += G2.apply_updates([a for a, _, _ in grp], [b for _, b, _ in grp], [i for _, _, i in grp])
        p1, f1, i1 = G1.samples_get()
        p2, f2, i2 = G2.samples_get()
        assert k1 == k2
        assert np.array_equal(f1.cpu().numpy(), f2.cpu().numpy())
        assert np.array_equal(p1.cpu().numpy(), p2.cpu().numpy()) and np.array_equal(i1, i2)


def test_failed_refresh_is_never_queried(kc, oracle_lib, gen):
    """f is recomputed once at the end of an update call.  When that fails
    (forced from the host: a memory budget of exactly one sample's workspace
    before the insertion, so the sweep's larger Fenwick tree no longer fits),
    the call reports it, and queries report it too instead of reducing the f
    of the previous graph; once the budget is lifted the query recomputes f
    and equals the oracle's result for the updated set (Theorem 4.1)."""
    from test_gpu_parity import small_graphs
    g = small_graphs(gen)["grid32"]
    count = 16
    S = oracle_lib.samples_init(g.offsets, g.indices, seed=23, count=count)
    a, b = 5, 900
    g2 = gen.add_edges(g, [(a, b)])
    S2, _, _ = oracle_lib.bsm_insert(S, g2.offsets, g2.indices, a, b, 0)
    with kc.Graph.from_graph(g) as G:
        G.set_option(kc.KC_OPT_SLOTS, 1)
        G.set_option(kc.KC_OPT_TRAVERSAL, kc.KC_TRAV_SWEEP)
        G.samples_init(23, count)
        G.set_option(kc.KC_OPT_MEM_BUDGET, G.info["sample_bytes"])
        with pytest.raises(kc.KcError) as ei:
            G.apply_updates([a], [b], is_insert=[1])
        assert ei.value.status == 3
        assert G.two_m == g2.two_m  # the insertion itself is in place
        with pytest.raises(kc.KcError) as ei:
            G.samples_query()
        assert ei.value.status == 3
        G.set_option(kc.KC_OPT_MEM_BUDGET, 0)
        est = G.samples_query()
        K, se, s1, _ = oracle_lib.reduce_estimate(S2.f, g2.two_m)
        assert est.sum_f == s1 and est.kappa == K
        _compare(G, S2, g2.two_m)

