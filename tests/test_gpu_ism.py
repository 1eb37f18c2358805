"""GPU parity of improved sample maintenance (section 4.2, Algorithm 3)
against the oracle: after every insertion (link-cut) and deletion (cut-link)
the resident trees, their f on the new graph and their weights equal the
oracle's, and so does the weighted estimate."""
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


def _compare(G, W, two_m, oracle_lib):
    par, f, ids = G.samples_get()
    assert np.array_equal(par.cpu().numpy(), W.S.parents)
    assert np.array_equal(f.cpu().numpy(), W.S.f)
    assert np.array_equal(ids, W.S.ids)
    assert G.two_m == two_m
    w = G.samples_weights()
    assert np.allclose(w, W.w, rtol=1e-12, atol=0)
    assert abs(w.sum() - 1.0) < 1e-12
    est = G.samples_query()
    k_ref, se_ref = oracle_lib.weighted_estimate(W)
    assert est.kappa == pytest.approx(k_ref, rel=1e-12)
    assert est.std_error == pytest.approx(se_ref, rel=1e-9)


@pytest.mark.parametrize("name", ["grid32", "road3k", "social3k"])
def test_ism_matches_oracle(kc, oracle_lib, gen, name):
    from test_gpu_parity import small_graphs
    from test_gpu_updates import deletion_batches
    g = small_graphs(gen)[name]
    count = 48
    W = oracle_lib.ism_init(g.offsets, g.indices, seed=13, count=count)
    with kc.Graph.from_graph(g) as G:
        G.set_option(kc.KC_OPT_MAINTENANCE, kc.KC_MAINT_IMPROVED)
        G.samples_init(13, count)
        _compare(G, W, g.two_m, oracle_lib)
        # equal weights: the maintenance may still change (and change back)
        G.set_option(kc.KC_OPT_MAINTENANCE, kc.KC_MAINT_BASIC)
        G.set_option(kc.KC_OPT_MAINTENANCE, kc.KC_MAINT_IMPROVED)
        rng = np.random.default_rng(5)
        for u, v in gen.insertion_batch(g, 3, rng):
            _say(name, "insert", u, v)
            g = gen.add_edges(g, [(u, v)])
            W, k_ref = oracle_lib.ism_insert(W, g.offsets, g.indices, u, v)
            assert G.apply_updates([u], [v], [1]) == k_ref
            _compare(G, W, g.two_m, oracle_lib)
        if len(set(G.samples_weights().tolist())) > 1:
            with pytest.raises(kc.KcError):   # weighted trees are not a uniform set
                G.set_option(kc.KC_OPT_MAINTENANCE, kc.KC_MAINT_BASIC)
        batch = deletion_batches(gen, g, [4], seed=9)[0]
        _say(name, "delete", batch)
        k_ref = 0
        for a, b in batch:
            g = gen.remove_edges(g, [(a, b)])
            W, k = oracle_lib.ism_delete(W, g.offsets, g.indices, a, b)
            k_ref += k
        assert G.apply_updates([a for a, _ in batch], [b for _, b in batch]) == k_ref
        _compare(G, W, g.two_m, oracle_lib)
        # mixed, in one call: an insertion between two deletions
        (a1, b1), (a2, b2) = deletion_batches(gen, g, [2], seed=10)[0]
        (u, v), = gen.insertion_batch(gen.remove_edges(g, [(a1, b1)]), 1, rng)
        _say(name, "mixed", (a1, b1), (u, v), (a2, b2))
        k_ref = 0
        g = gen.remove_edges(g, [(a1, b1)])
        W, k = oracle_lib.ism_delete(W, g.offsets, g.indices, a1, b1)
        k_ref += k
        g = gen.add_edges(g, [(u, v)])
        W, k = oracle_lib.ism_insert(W, g.offsets, g.indices, u, v)
        k_ref += k
        g = gen.remove_edges(g, [(a2, b2)])
        W, k = oracle_lib.ism_delete(W, g.offsets, g.indices, a2, b2)
        k_ref += k
        assert G.apply_updates([a1, u, a2], [b1, v, b2], [0, 1, 0]) == k_ref
        _compare(G, W, g.two_m, oracle_lib)


def test_ism_deletion_of_every_tree_edge_of_a_cycle(kc, oracle_lib, gen):
    """A cycle plus one chord: deleting a cycle edge hits most trees, and the
    cut-link choice has few candidates (edge cases of the draw and the path
    reversal at the root)."""
    g = gen.add_edges(gen.cycle(12), [(0, 6)])
    count = 16
    W = oracle_lib.ism_init(g.offsets, g.indices, seed=3, count=count)
    with kc.Graph.from_graph(g) as G:
        G.set_option(kc.KC_OPT_MAINTENANCE, kc.KC_MAINT_IMPROVED)
        G.samples_init(3, count)
        for a, b in [(2, 3), (8, 9)]:
            g = gen.remove_edges(g, [(a, b)])
            W, k_ref = oracle_lib.ism_delete(W, g.offsets, g.indices, a, b)
            assert G.apply_updates([a], [b]) == k_ref
            _compare(G, W, g.two_m, oracle_lib)
        # now a tree: every further insertion makes one cycle
        for u, v in [(1, 4), (3, 11)]:
            g = gen.add_edges(g, [(u, v)])
            W, k_ref = oracle_lib.ism_insert(W, g.offsets, g.indices, u, v)
            assert G.apply_updates([u], [v], [1]) == k_ref
            _compare(G, W, g.two_m, oracle_lib)
