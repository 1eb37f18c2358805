"""The allocation-free estimate (kc_estimate_static) against kc_estimate,
through the C ABI: per-tree f, the exact sums, kappa and its standard error
bit for bit, on two calls in a row, the second on a smaller input.  The first
graph is deep enough for the sweep traversal, whose Fenwick trees the static
workspace must clear; the second call reuses the workspace the first one left
behind."""
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


def test_static_workspace_matches_estimate(kc, gen):
    cases = [("road-like 20k points", gen.road_like(20000, seed=3), 7, 1000, 300),
             ("grid 16x16", gen.grid(16, 16), 9, 5, 40)]
    for name, g, seed, first, count in cases:
        _say("static workspace:", name, g.n, "samples", count)
        with kc.Graph.from_graph(g) as G:
            ref, fref, _ = G.estimate(seed, first, count, per_sample=True)
            est, f = G.estimate_static(seed, first, count, per_sample=True)
            assert np.array_equal(f.cpu().numpy(), fref.cpu().numpy())
            assert est.sum_f == ref.sum_f and est.sum_f2 == ref.sum_f2
            assert est.kappa == ref.kappa and est.std_error == ref.std_error
            assert est.count == count and est.total_steps == ref.total_steps
            # without f_out the per-tree values live in the static workspace too
            est2 = G.estimate_static(seed, first, count)
            assert est2.sum_f == ref.sum_f and est2.kappa == ref.kappa


def test_static_workspace_rejects_what_does_not_fit(kc, gen):
    with kc.Graph.from_graph(gen.grid(8, 8)) as G:
        with pytest.raises(kc.KcError) as ei:
            G.estimate_static(0, 0, 12_000_000)  # 24 bytes per sample exceed the 256 MiB
        assert ei.value.status == 3
