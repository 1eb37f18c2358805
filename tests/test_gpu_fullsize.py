"""GPU parity at the benchmark workloads' full sizes, in the launch
configuration bench.py times (default options, seed 0, sample ids from 0).

Samples are compared one by one with the oracle: per-tree f and draw counts
exactly, and one whole tree (parents and per-vertex draw counts).  The
oracle finishes these few samples in seconds; the rest of a batch is covered
by the invariance tests (results do not depend on the batch or the launch
shape)."""
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


def _check_prefix(kc, oracle_lib, g, count, tree_id):
    P = oracle_lib.prepare_graph(g)
    _say("oracle", g.name, g.n, g.two_m, "count", count)
    ref_f, ref_steps = oracle_lib.estimate_f(P, seed=0, s0=0, count=count, threads=8)
    K, se, s1, s2 = oracle_lib.reduce_estimate(ref_f, g.two_m)
    with kc.Graph.from_graph(g) as G:
        assert G.root == P.root
        # large sparse graphs get the 2,048-entry chain table by default, the others 1,024
        assert G.info["chains"] == (2048 if g.n >= 100_000 and g.two_m < 4 * g.n else 1024)
        _say("gpu estimate")
        est, f, st = G.estimate(0, 0, count, per_sample=True)
        assert np.array_equal(f.cpu().numpy(), ref_f)
        assert np.array_equal(st.cpu().numpy(), ref_steps)
        assert est.sum_f == s1 and est.sum_f2 == s2
        assert est.kappa == K and est.std_error == se
        _say("gpu tree", tree_id)
        par, cnt, _ = G.sample_trees(0, tree_id, 1)
    ref_par, ref_cnt, _ = oracle_lib.sample(P, seed=0, s0=tree_id, count=1)
    assert np.array_equal(par.cpu().numpy(), ref_par)
    assert np.array_equal(cnt.cpu().numpy().astype(np.uint32), ref_cnt)


def _check_random_ids(kc, oracle_lib, g, batch, first, nids, seed_ids):
    """The benchmark's launch shape (default options, `batch` samples from
    `first`), compared with the oracle on a seeded random subset of `nids`
    sample ids of the batch, each computed by the oracle on its own."""
    P = oracle_lib.prepare_graph(g)
    rng = np.random.default_rng(seed_ids)
    pos = np.sort(rng.choice(batch, size=nids, replace=False))
    ids = first + pos
    _say("oracle", g.name, g.n, "ids", nids, "of", batch)
    ref_f, ref_steps = oracle_lib.estimate_ids(P, 0, ids, threads=16)
    with kc.Graph.from_graph(g) as G:
        assert G.root == P.root
        _say("gpu batch", batch, "from", first)
        G.reserve(batch)
        est, f, st = G.estimate(0, first, batch, per_sample=True)
        f = f.cpu().numpy()
        st = st.cpu().numpy()
    assert np.array_equal(f[pos], ref_f)
    assert np.array_equal(st[pos], ref_steps)
    assert est.count == batch and est.sum_f == int(f.astype(object).sum())


def test_dense_power_law_random_ids(kc, oracle_lib):
    """The headline workload (Chung-Lu 3x10^6 vertices, mean degree 76): one
    4,096-sample launch of the third benchmark step (ids 8,192..12,287), as
    bench.py times it, with slots reused across waves; 64 seeded random ids
    checked against the oracle."""
    import graphgen
    _check_random_ids(kc, oracle_lib, graphgen.workload("dense"), 4096, 2 * 4096, 64, 5)


def test_road_like_random_ids(kc, oracle_lib):
    """Road-like 10^6 points: a 256-sample launch in the benchmark's launch
    options, 64 seeded random ids against the oracle."""
    import graphgen
    _check_random_ids(kc, oracle_lib, graphgen.workload("road"), 256, 4096, 64, 6)


def test_road_like_full_size(kc, oracle_lib):
    """Road-like: 10^6 points, thinned RGG, LCC n = 792,324 (the bench workload)."""
    import graphgen
    _check_prefix(kc, oracle_lib, graphgen.workload("road"), 8, 3)


def test_social_full_size(kc, oracle_lib):
    """Chung-Lu 10^6 vertices, exponent 2.2, mean 10, cap 5000."""
    import graphgen
    _check_prefix(kc, oracle_lib, graphgen.workload("social"), 32, 5)


def test_dense_power_law_full_size(kc, oracle_lib):
    """Chung-Lu 3x10^6 vertices, mean degree 76 (about 1.1x10^8 edges), cap 30,000:
    int64 offsets on input, 2m below 2^31."""
    import graphgen
    g = graphgen.workload("dense")
    assert g.offsets.dtype == np.int64
    _check_prefix(kc, oracle_lib, g, 4, 2)
