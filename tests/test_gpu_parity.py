"""GPU parity: the HIP path against the CPU oracle, through the C ABI.

Bars (exact integer work, so exactness everywhere):
  - sampled parent arrays and per-vertex draw counts bit-identical;
  - per-tree f identical as int64;
  - K-hat and its standard error bit-identical (both computed from the same
    exact integer sums with the same double formula);
  - results independent of walkers per sample, samples in flight, batch
    split and traversal variant.
"""
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
    kc.library()  # raises if the HIP library is missing: no fallback
    return kc


def double_star(gen, leaves):
    """Two hubs joined by an edge, each with `leaves` leaves: the non-root hub
    draws from a row far longer than the inline neighbours."""
    eu = [0] + [0] * leaves + [1] * leaves
    ev = [1] + list(range(2, 2 + leaves)) + list(range(2 + leaves, 2 + 2 * leaves))
    return gen.from_edges("double_star(%d)" % leaves, 2 + 2 * leaves, eu, ev)


def small_graphs(gen):
    return {
        "K2": gen.complete(2), "P300": gen.path(300), "dstar": double_star(gen, 300),
        "K3": gen.complete(3), "K5": gen.complete(5), "C7": gen.cycle(7), "P6": gen.path(6),
        "star9": gen.star(9), "petersen": gen.petersen(), "grid8": gen.grid(8, 8),
        "grid32": gen.grid(32, 32), "ba200": gen.barabasi_albert(200, 3, 1),
        "gnm300": gen.largest_component(gen.gnm(300, 700, 5)),
        "torus12": gen.torus(12, 12), "Q7": gen.hypercube(7),
        "road3k": gen.road_like(3000, seed=4), "social3k": gen.chung_lu(3000, 2.2, 10.0, 300.0, seed=6),
    }


@pytest.fixture(scope="module")
def graphs(gen):
    return small_graphs(gen)


@pytest.mark.parametrize("name", ["K2", "K3", "K5", "C7", "P6", "P300", "star9", "dstar", "petersen",
                                  "grid8", "grid32", "ba200", "gnm300", "torus12", "Q7", "road3k",
                                  "social3k"])
def test_sampled_trees_bit_exact(kc, oracle_lib, graphs, name):
    g = graphs[name]
    _say("sample parity", name, g.n)
    P = oracle_lib.prepare_graph(g)
    count = 48
    ref_par, ref_cnt, ref_steps = oracle_lib.sample(P, seed=77, s0=5, count=count, threads=8)
    with kc.Graph.from_graph(g) as G:
        assert G.root == P.root
        par, cnt, stp = G.sample_trees(77, 5, count)
        assert np.array_equal(par.cpu().numpy(), ref_par)
        assert np.array_equal(cnt.cpu().numpy().astype(np.uint32), ref_cnt)
        assert np.array_equal(stp.cpu().numpy(), ref_steps)


@pytest.mark.parametrize("walkers,slots", [(1, 1), (2, 3), (7, 64), (64, 5), (64, 0)])
def test_launch_shape_invariance(kc, oracle_lib, graphs, walkers, slots):
    for name in ("grid32", "road3k", "social3k"):
        g = graphs[name]
        _say("invariance", name, walkers, slots)
        P = oracle_lib.prepare_graph(g)
        ref_par, ref_cnt, _ = oracle_lib.sample(P, seed=3, s0=100, count=20, threads=8)
        with kc.Graph.from_graph(g) as G:
            G.set_option(kc.KC_OPT_WALKERS, walkers)
            G.set_option(kc.KC_OPT_SLOTS, slots)
            par, cnt, _ = G.sample_trees(3, 100, 20)
            assert np.array_equal(par.cpu().numpy(), ref_par)
            assert np.array_equal(cnt.cpu().numpy().astype(np.uint32), ref_cnt)


@pytest.mark.parametrize("order", [0, 1, 2])
def test_start_order_invariance(kc, oracle_lib, graphs, order):
    """Walk start order changes nothing: trees and draw counts stay bit-exact."""
    for name in ("grid32", "road3k", "social3k", "torus12"):
        g = graphs[name]
        P = oracle_lib.prepare_graph(g)
        ref_par, ref_cnt, _ = oracle_lib.sample(P, seed=8, s0=40, count=16, threads=8)
        with kc.Graph.from_graph(g) as G:
            G.set_option(kc.KC_OPT_START_ORDER, order)
            par, cnt, _ = G.sample_trees(8, 40, 16)
            assert np.array_equal(par.cpu().numpy(), ref_par)
            assert np.array_equal(cnt.cpu().numpy().astype(np.uint32), ref_cnt)


@pytest.mark.parametrize("chains", [2048])
def test_chain_table_size_invariance(kc, oracle_lib, graphs, chains):
    """The chain-table size changes nothing: trees, draw counts and f stay exact."""
    for name in ("K5", "petersen", "grid32", "road3k", "social3k", "torus12"):
        g = graphs[name]
        _say("chains", chains, name)
        P = oracle_lib.prepare_graph(g)
        ref_par, ref_cnt, ref_steps = oracle_lib.sample(P, seed=31, s0=200, count=20, threads=8)
        ref_f = np.array([oracle_lib.f_of_tree(P, t) for t in ref_par], np.int64)
        with kc.Graph.from_graph(g) as G:
            G.set_option(kc.KC_OPT_CHAINS, chains)
            par, cnt, stp = G.sample_trees(31, 200, 20)
            assert np.array_equal(par.cpu().numpy(), ref_par)
            assert np.array_equal(cnt.cpu().numpy().astype(np.uint32), ref_cnt)
            assert np.array_equal(stp.cpu().numpy(), ref_steps)
            _, f, _ = G.estimate(31, 200, 20, per_sample=True)
            assert np.array_equal(f.cpu().numpy(), ref_f)
            assert G.progress() == 20


@pytest.mark.parametrize("lean", [1, 2])
def test_lean_looks_change_nothing(kc, oracle_lib, graphs, lean):
    """A walk's look at its next vertex as the claim alone, with the claimed
    vertex's words read in the next round, or as one full round (either way on
    every graph, whatever the mean-degree default), changes nothing: trees,
    draw counts and f stay exact, also with more samples than slots."""
    for name in ("K5", "petersen", "grid32", "road3k", "social3k", "torus12", "gnm300"):
        g = graphs[name]
        _say("lean", lean, name)
        P = oracle_lib.prepare_graph(g)
        ref_par, ref_cnt, ref_steps = oracle_lib.sample(P, seed=37, s0=300, count=24, threads=8)
        ref_f = np.array([oracle_lib.f_of_tree(P, t) for t in ref_par], np.int64)
        with kc.Graph.from_graph(g) as G:
            G.set_option(kc.KC_OPT_LEAN_LOOKS, lean)
            par, cnt, stp = G.sample_trees(37, 300, 24)
            assert np.array_equal(par.cpu().numpy(), ref_par)
            assert np.array_equal(cnt.cpu().numpy().astype(np.uint32), ref_cnt)
            assert np.array_equal(stp.cpu().numpy(), ref_steps)
            G.set_option(kc.KC_OPT_SLOTS, 5)
            _, f, _ = G.estimate(37, 300, 24, per_sample=True)
            assert np.array_equal(f.cpu().numpy(), ref_f)


def test_lean_looks_with_the_large_chain_table(kc, oracle_lib, graphs):
    """Lean looks together with the 2,048-chain table (kernel variants of
    their own, in the persistent launch and in a captured batch): trees, draw
    counts and f stay exact, also with more samples than slots."""
    for name in ("K5", "grid32", "road3k", "social3k"):
        g = graphs[name]
        _say("lean + 2048 chains", name)
        P = oracle_lib.prepare_graph(g)
        ref_par, ref_cnt, ref_steps = oracle_lib.sample(P, seed=43, s0=600, count=24, threads=8)
        ref_f = np.array([oracle_lib.f_of_tree(P, t) for t in ref_par], np.int64)
        with kc.Graph.from_graph(g) as G:
            G.set_option(kc.KC_OPT_CHAINS, 2048)
            G.set_option(kc.KC_OPT_LEAN_LOOKS, 2)
            par, cnt, stp = G.sample_trees(43, 600, 24)
            assert np.array_equal(par.cpu().numpy(), ref_par)
            assert np.array_equal(cnt.cpu().numpy().astype(np.uint32), ref_cnt)
            assert np.array_equal(stp.cpu().numpy(), ref_steps)
            G.set_option(kc.KC_OPT_SLOTS, 5)
            _, f, _ = G.estimate(43, 600, 24, per_sample=True)
            assert np.array_equal(f.cpu().numpy(), ref_f)
            with kc.Batch([G], [43], [600], [24]) as B:
                B.launch()
                B.results()
                assert np.array_equal(B.f(0).cpu().numpy(), ref_f)


def test_batch_split_invariance(kc, graphs):
    g = graphs["road3k"]
    with kc.Graph.from_graph(g) as G:
        whole, _, _ = G.sample_trees(9, 0, 30)
        a, _, _ = G.sample_trees(9, 0, 11)
        b, _, _ = G.sample_trees(9, 11, 19)
        one, _, _ = G.sample_trees(9, 17, 1)
        w = whole.cpu().numpy()
        assert np.array_equal(w[:11], a.cpu().numpy())
        assert np.array_equal(w[11:], b.cpu().numpy())
        assert np.array_equal(w[17], one.cpu().numpy()[0])


@pytest.mark.parametrize("trav", [1, 2])
@pytest.mark.parametrize("name", ["K3", "petersen", "grid8", "grid32", "ba200", "gnm300",
                                  "torus12", "road3k", "social3k"])
def test_tree_values_exact(kc, oracle_lib, graphs, name, trav):
    """f(tau) of oracle-sampled trees, evaluated on the GPU (both traversals)."""
    import torch
    g = graphs[name]
    _say("f parity", name, trav)
    P = oracle_lib.prepare_graph(g)
    par, _, _ = oracle_lib.sample(P, seed=21, s0=0, count=24, threads=8)
    ref = np.array([oracle_lib.f_of_tree(P, t) for t in par], np.int64)
    with kc.Graph.from_graph(g) as G:
        G.set_option(kc.KC_OPT_TRAVERSAL, trav)
        f = G.evaluate_trees(torch.from_numpy(par).cuda())
        assert np.array_equal(f.cpu().numpy(), ref)


@pytest.mark.parametrize("trav", [1, 2])
@pytest.mark.parametrize("name", ["K2", "K5", "P300", "dstar", "grid32", "ba200", "road3k", "social3k",
                                  "Q7"])
def test_estimate_exact(kc, oracle_lib, graphs, name, trav):
    g = graphs[name]
    _say("estimate parity", name, trav)
    P = oracle_lib.prepare_graph(g)
    count = 64
    ref_f, ref_steps = oracle_lib.estimate_f(P, seed=1234, s0=7, count=count, threads=8)
    K, se, s1, s2 = oracle_lib.reduce_estimate(ref_f, g.two_m)
    with kc.Graph.from_graph(g) as G:
        G.set_option(kc.KC_OPT_TRAVERSAL, trav)
        est, f, stp = G.estimate(1234, 7, count, per_sample=True)
        assert np.array_equal(f.cpu().numpy(), ref_f)
        assert np.array_equal(stp.cpu().numpy(), ref_steps)
        assert est.sum_f == s1 and est.sum_f2 == s2
        assert est.kappa == K  # bit-identical
        assert est.std_error == se
        assert est.total_steps == int(ref_steps.sum())


@pytest.mark.parametrize("trav", [1, 2])
@pytest.mark.parametrize("name", ["petersen", "grid32", "road3k", "social3k"])
def test_more_samples_than_slots(kc, oracle_lib, graphs, name, trav):
    """Five slots serve forty samples, so every slot is reused about eight
    times within one launch: its sampler state, numbering arrays and (sweep)
    Fenwick tree must return to their start state between trees.  Estimate,
    evaluation of given trees and a resident set, each against the oracle."""
    import torch
    g = graphs[name]
    _say("slots < count", name, trav)
    P = oracle_lib.prepare_graph(g)
    ref_f, ref_steps = oracle_lib.estimate_f(P, seed=41, s0=300, count=40, threads=8)
    ref_par, _, _ = oracle_lib.sample(P, seed=41, s0=300, count=40, threads=8)
    K, se, s1, s2 = oracle_lib.reduce_estimate(ref_f, g.two_m)
    with kc.Graph.from_graph(g) as G:
        G.set_option(kc.KC_OPT_SLOTS, 5)
        G.set_option(kc.KC_OPT_TRAVERSAL, trav)
        est, f, stp = G.estimate(41, 300, 40, per_sample=True)
        assert np.array_equal(f.cpu().numpy(), ref_f)
        assert np.array_equal(stp.cpu().numpy(), ref_steps)
        assert est.kappa == K and est.std_error == se and est.sum_f == s1
        fe = G.evaluate_trees(torch.from_numpy(ref_par).cuda())
        assert np.array_equal(fe.cpu().numpy(), ref_f)
        G.samples_init(41, 40)
        S = oracle_lib.samples_init(g.offsets, g.indices, seed=41, count=40)
        par, fr, ids = G.samples_get()
        assert np.array_equal(par.cpu().numpy(), S.parents)
        assert np.array_equal(fr.cpu().numpy(), S.f)


def test_grid32_eps_at_95(kc, oracle_lib, gen):
    """The 32x32 grid with 8,192 samples from seed 0 (the first 8,192 sample
    ids): every f equals the oracle's, and K-hat lies within eps = 0.01 of the
    exact Kemeny constant (Eq. 1, dense eigensolve), with the 95% interval
    (reading A10: 1.96 standard errors) also narrower than eps."""
    from oracle import exact as E
    g = gen.grid(32, 32)
    P = oracle_lib.prepare_graph(g)
    ref_f, _ = oracle_lib.estimate_f(P, seed=0, s0=0, count=8192, threads=8)
    K, se, _, _ = oracle_lib.reduce_estimate(ref_f, g.two_m)
    Kx = E.kemeny_exact(g.offsets, g.indices)
    with kc.Graph.from_graph(g) as G:
        est, f, _ = G.estimate(0, 0, 8192, per_sample=True)
        assert np.array_equal(f.cpu().numpy(), ref_f)
        assert est.kappa == K and est.std_error == se
    assert abs(est.kappa / Kx - 1.0) <= 0.01
    assert 1.959963984540054 * est.std_error / Kx <= 0.01


def test_combine_results_pools_exact_sums(kc, oracle_lib, graphs):
    """Estimates of consecutive sample ranges, pooled by the library, equal one
    estimate over the whole range bit for bit."""
    g = graphs["road3k"]
    with kc.Graph.from_graph(g) as G:
        whole = G.estimate(6, 0, 30)
        parts = [G.estimate(6, 0, 7), G.estimate(6, 7, 1), G.estimate(6, 8, 22)]
        pooled = G.combine(parts)
        assert pooled.sum_f == whole.sum_f and pooled.sum_f2 == whole.sum_f2
        assert pooled.kappa == whole.kappa and pooled.std_error == whole.std_error
        assert pooled.count == 30 and pooled.total_steps == whole.total_steps


def test_grid32_full_config(kc, oracle_lib, gen):
    """32x32 grid, 2,000 samples from seed 0: every f equal to the oracle's,
    and K-hat within 4.5 standard errors of the exact Kemeny constant."""
    from oracle import exact as E
    g = gen.grid(32, 32)
    P = oracle_lib.prepare_graph(g)
    ref_f, _ = oracle_lib.estimate_f(P, seed=0, s0=0, count=2000, threads=8)
    K, se, _, _ = oracle_lib.reduce_estimate(ref_f, g.two_m)
    with kc.Graph.from_graph(g) as G:
        est, f, _ = G.estimate(0, 0, 2000, per_sample=True)
        assert np.array_equal(f.cpu().numpy(), ref_f)
        assert est.kappa == K and est.std_error == se
    Kx = E.kemeny_exact(g.offsets, g.indices)
    assert abs(est.kappa - Kx) < 4.5 * est.std_error


def test_reserve_then_estimate(kc, oracle_lib, graphs):
    """Workspace reserved ahead of time gives the same results."""
    g = graphs["road3k"]
    P = oracle_lib.prepare_graph(g)
    ref_f, _ = oracle_lib.estimate_f(P, seed=5, s0=0, count=16, threads=8)
    with kc.Graph.from_graph(g) as G:
        G.reserve(16)
        est, f, _ = G.estimate(5, 0, 16, per_sample=True)
        assert np.array_equal(f.cpu().numpy(), ref_f)
        with pytest.raises(kc.KcError):
            G.reserve(0)


def test_empty_batches(kc, graphs):
    """count 0 samples nothing and succeeds; an estimate needs at least one sample."""
    g = graphs["grid8"]
    with kc.Graph.from_graph(g) as G:
        par, cnt, stp = G.sample_trees(1, 0, 0)
        assert par.shape == (0, g.n)
        with pytest.raises(kc.KcError) as ei:
            G.estimate(1, 0, 0)
        assert ei.value.status == 1


def test_step_limit_reports_error(kc, graphs):
    g = graphs["grid32"]
    with kc.Graph.from_graph(g) as G:
        G.set_option(kc.KC_OPT_STEP_LIMIT, 50)
        with pytest.raises(kc.KcError) as ei:
            G.sample_trees(0, 0, 4)
        assert ei.value.status == 6
        G.set_option(kc.KC_OPT_STEP_LIMIT, 0)
        par, _, _ = G.sample_trees(0, 0, 4)  # usable again afterwards
        assert par.shape == (4, g.n)


def test_evaluate_rejects_non_tree(kc, graphs):
    import torch
    g = graphs["grid8"]
    with kc.Graph.from_graph(g) as G:
        par, _, _ = G.sample_trees(1, 0, 2)
        bad = par.clone()
        v = 1 if G.root != 1 else 2
        bad[0, v] = g.n + 5  # out of range parent
        with pytest.raises(kc.KcError) as ei:
            G.evaluate_trees(bad)
        assert ei.value.status == 1
