"""The high words of the arrow generator on the GPU, against the CPU oracle.

Each arrow is Philox4x32-10 with counter (k, v, s_lo, s_hi) and key
(seed_lo, seed_hi).  Here every seed has a non-zero high word and the sample
ids run across 2^32 (s_lo wrapping, s_hi changing), so a path that dropped or
swapped a high word would draw different trees.  Checked through every entry
point that draws trees: kc_sample_trees (parents, draw counts, totals),
kc_estimate under both traversals, kc_estimate_static, and replays of a
captured batch whose later launches cross 2^32.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

SEED = 0xDEADBEEF12345678          # seed_hi = 0xDEADBEEF
SEED2 = (1 << 63) | 0x0000000100000003
EDGE = (1 << 32) - 20              # ids EDGE .. EDGE + 39 cross 2^32


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


@pytest.fixture(scope="module")
def graphs(gen):
    from test_gpu_parity import small_graphs
    return small_graphs(gen)


@pytest.mark.parametrize("name", ["K5", "grid8", "road3k", "social3k"])
def test_sample_trees_across_two_to_the_32(kc, oracle_lib, graphs, name):
    g = graphs[name]
    _say("counter words: sample_trees", name, g.n)
    P = oracle_lib.prepare_graph(g)
    ref_par, ref_cnt, ref_steps = oracle_lib.sample(P, seed=SEED, s0=EDGE, count=40, threads=8)
    # the high words matter: the same ids with the seed's high word cleared give other trees
    other, _, _ = oracle_lib.sample(P, seed=SEED & 0xFFFFFFFF, s0=EDGE, count=40, threads=8)
    assert not np.array_equal(other, ref_par)
    with kc.Graph.from_graph(g) as G:
        par, cnt, stp = G.sample_trees(SEED, EDGE, 40)
        assert np.array_equal(par.cpu().numpy(), ref_par)
        assert np.array_equal(cnt.cpu().numpy().astype(np.uint32), ref_cnt)
        assert np.array_equal(stp.cpu().numpy(), ref_steps)


@pytest.mark.parametrize("trav", [1, 2])
@pytest.mark.parametrize("name", ["grid32", "road3k", "social3k"])
def test_estimate_across_two_to_the_32(kc, oracle_lib, graphs, name, trav):
    g = graphs[name]
    _say("counter words: estimate", name, "traversal", trav)
    P = oracle_lib.prepare_graph(g)
    ref_f, ref_steps = oracle_lib.estimate_f(P, seed=SEED2, s0=EDGE, count=40, threads=8)
    K, se, sum_f, sum_f2 = oracle_lib.reduce_estimate(ref_f, g.two_m)
    with kc.Graph.from_graph(g) as G:
        G.set_option(kc.KC_OPT_TRAVERSAL, trav)
        est, f, stp = G.estimate(SEED2, EDGE, 40, per_sample=True)
        assert np.array_equal(f.cpu().numpy(), ref_f)
        assert np.array_equal(stp.cpu().numpy(), ref_steps)
        assert est.sum_f == sum_f and est.sum_f2 == sum_f2
        assert est.kappa == K and est.std_error == se
        est_s, f_s = G.estimate_static(SEED2, EDGE, 40, per_sample=True)
        assert np.array_equal(f_s.cpu().numpy(), ref_f)
        assert est_s.kappa == K and est_s.sum_f == sum_f


def test_batch_replays_cross_two_to_the_32(kc, oracle_lib, graphs):
    """Launch L of the batch draws ids first + L * count ..: with first just
    below 2^32 the second launch lies across it and the third above it."""
    names = ["road3k", "social3k"]
    seeds = [SEED, SEED2]
    counts = [16, 24]
    firsts = [(1 << 32) - 24, (1 << 32) - 30]
    Ps = [oracle_lib.prepare_graph(graphs[nm]) for nm in names]
    Gs = [kc.Graph.from_graph(graphs[nm]) for nm in names]
    try:
        with kc.Batch(Gs, seeds, firsts, counts) as B:
            for L in range(3):
                _say("counter words: batch launch", L)
                B.launch()
                ests, launches = B.results()
                assert launches == L + 1
                for j in range(len(names)):
                    s0 = firsts[j] + L * counts[j]
                    ref_f, _ = oracle_lib.estimate_f(Ps[j], seed=seeds[j], s0=s0, count=counts[j], threads=8)
                    assert np.array_equal(B.f(j).cpu().numpy(), ref_f), (names[j], L)
                    K, se, sum_f, _ = oracle_lib.reduce_estimate(ref_f, Ps[j].two_m)
                    assert ests[j].sum_f == sum_f and ests[j].kappa == K and ests[j].std_error == se
    finally:
        for G in Gs:
            G.close()
