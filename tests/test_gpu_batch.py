"""Batching invariance on the GPU, through the C ABI.

The paper parallelises across samples (section 5, Exp-VI); here samples of
several graphs share one persistent launch, captured once as a HIP graph and
replayed.  For the same (seed, s) every tree, and so every f, draw count and
exact sum, must be what a direct kc_estimate gives:
  - replay after replay of a captured one-graph batch;
  - one launch over graphs of uneven size against per-graph launches;
  - with the options the autotuner picks.
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
    kc.library()
    return kc


@pytest.fixture(scope="module")
def graphs(gen):
    from test_gpu_parity import small_graphs
    return small_graphs(gen)


def _same(est, ref):
    assert est.sum_f == ref.sum_f and est.sum_f2 == ref.sum_f2
    assert est.kappa == ref.kappa and est.std_error == ref.std_error
    assert est.count == ref.count and est.total_steps == ref.total_steps


@pytest.mark.parametrize("name", ["road3k", "social3k", "grid32"])
def test_graph_replay_equals_direct_launch(kc, oracle_lib, graphs, name):
    g = graphs[name]
    _say("replay", name)
    P = oracle_lib.prepare_graph(g)
    ref_f0, _ = oracle_lib.estimate_f(P, seed=13, s0=100, count=48, threads=8)
    with kc.Graph.from_graph(g) as G:
        with kc.Batch([G], [13], [100], [48]) as B:
            for L in range(3):
                B.launch()
                (est,), launches = B.results()
                assert launches == L + 1
                ref, fref, _ = G.estimate(13, 100 + 48 * L, 48, per_sample=True)
                f = B.f(0).cpu().numpy()
                assert np.array_equal(f, fref.cpu().numpy())
                _same(est, ref)
                if L == 0:
                    assert np.array_equal(f, ref_f0)


def test_multi_graph_launch_equals_per_graph(kc, graphs):
    names = ["K5", "grid32", "road3k", "social3k", "petersen", "P300"]
    counts = [7, 40, 25, 33, 3, 12]
    seeds = [1, 2, 3, 4, 5, 6]
    firsts = [0, 10, 500, 7, 1 << 33, 3]
    Gs = [kc.Graph.from_graph(graphs[nm]) for nm in names]
    try:
        with kc.Batch(Gs, seeds, firsts, counts) as B:
            for L in range(2):
                _say("multi-graph launch", L)
                B.launch()
                ests, launches = B.results()
                assert launches == L + 1
                for j, G in enumerate(Gs):
                    ref, fref, _ = G.estimate(seeds[j], firsts[j] + L * counts[j], counts[j], per_sample=True)
                    assert np.array_equal(B.f(j).cpu().numpy(), fref.cpu().numpy()), names[j]
                    _same(ests[j], ref)
    finally:
        for G in Gs:
            G.close()


def test_batch_status_is_read_from_the_device(kc, graphs):
    """A sample over the step limit (forced from the host: 50 rounds) is reported
    by kc_batch_results; the next launch of a batch without the limit works."""
    g = graphs["grid32"]
    with kc.Graph.from_graph(g) as G:
        G.set_option(kc.KC_OPT_STEP_LIMIT, 50)
        with kc.Batch([G], [0], [0], [4]) as B:
            B.launch()
            with pytest.raises(kc.KcError) as ei:
                B.results()
            assert ei.value.status == 6
        G.set_option(kc.KC_OPT_STEP_LIMIT, 0)
        with kc.Batch([G], [0], [0], [4]) as B:
            B.launch()
            (est,), _ = B.results()
            _same(est, G.estimate(0, 0, 4))


def test_autotuned_options_give_identical_results(kc, graphs, tmp_path):
    g = graphs["social3k"]
    cache = str(tmp_path / "tune.jsonl")
    with kc.Graph.from_graph(g) as G:
        ref, fref, _ = G.estimate(21, 0, 300, per_sample=True)
        tune = G.autotune(300, cache_path=cache)
        _say("tuned", tune)
        assert tune["from_cache"] == 0 and tune["trials"] >= 2
        est, f, _ = G.estimate(21, 0, 300, per_sample=True)
        assert np.array_equal(f.cpu().numpy(), fref.cpu().numpy())
        _same(est, ref)
    with kc.Graph.from_graph(g) as G2:
        again = G2.autotune(300, cache_path=cache)
        assert again["from_cache"] == 1
        for key in ("chains", "slots", "walkers", "traversal"):
            assert again[key] == tune[key]
        est2 = G2.estimate(21, 0, 300)
        _same(est2, ref)
