"""Pins of the CPU oracle to the paper and to mathematics (no GPU).

Each test checks the oracle against something other than itself: an
independent Philox implementation, closed forms, the hitting-time definition
of the Kemeny constant, exhaustive spanning-tree enumeration, the paper's
worked triangle example, the cycle-popping order-independence theorem, and
chi-square uniformity of the sampled trees.
"""
import json
import math
import os
import shutil
import subprocess
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

HERE = os.path.dirname(os.path.abspath(__file__))


# ------------------------------------------------------------------ Philox

@pytest.fixture(scope="module")
def rocrand_probe(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("probe") / "philox_probe")
    subprocess.check_call([hipcc, "-O1", "-o", exe, os.path.join(HERE, "rocrand_philox_probe.cpp")],
                          cwd=str(tmp_path_factory.getbasetemp()))
    return exe


def test_philox_matches_rocrand(oracle_lib, rocrand_probe):
    rng = np.random.default_rng(7)
    cases = [[0] * 6, [0xFFFFFFFF] * 6, [1, 2, 3, 4, 5, 6]]
    cases += rng.integers(0, 2 ** 32, size=(200, 6), dtype=np.uint64).tolist()
    inp = "\n".join(" ".join(str(int(x)) for x in c) for c in cases) + "\n"
    out = subprocess.run([rocrand_probe], input=inp, capture_output=True, text=True, check=True).stdout
    ref = [list(map(int, line.split())) for line in out.strip().splitlines()]
    assert len(ref) == len(cases)
    for c, r in zip(cases, ref):
        got = oracle_lib.philox4x32_10(c[:4], c[4:])
        assert got.tolist() == r, (c, got, r)


def test_arrow_counter_layout_with_high_words(oracle_lib):
    """The arrow of (seed, s, v, k) is the Philox block (checked against
    rocRAND above) at counter (k, v, s_lo, s_hi) and key (seed_lo, seed_hi),
    mapped to floor(x deg / 2^64) with x = o0 | o1 << 32, also when the high
    words of the seed and of the sample id are not zero."""
    rng = np.random.default_rng(11)
    for _ in range(300):
        seed = int(rng.integers(0, 2 ** 63)) * 2 + int(rng.integers(0, 2))
        s = int(rng.integers(0, 2 ** 40))
        v, k = int(rng.integers(0, 2 ** 31)), int(rng.integers(0, 2 ** 20))
        deg = int(rng.integers(1, 1 << 20))
        o = oracle_lib.philox4x32_10([k, v, s & 0xFFFFFFFF, s >> 32], [seed & 0xFFFFFFFF, seed >> 32])
        x = int(o[0]) | (int(o[1]) << 32)
        assert oracle_lib.arrow(seed, s, v, k, deg) == (x * deg) >> 64


def test_arrow_slots_uniform(oracle_lib):
    """Slots drawn for fixed degree are uniform (chi-square) and in range."""
    for deg in (2, 3, 7, 13):
        counts = np.zeros(deg, np.int64)
        for v in range(400):
            for k in range(25):
                j = oracle_lib.arrow(12345, 3, v, k, deg)
                assert 0 <= j < deg
                counts[j] += 1
        p = stats.chisquare(counts).pvalue
        assert p > 1e-4, (deg, counts)


# ------------------------------------------------- exact-K checker pins

def test_closed_forms_match_eigensolve(gen):
    from oracle import exact as E
    for n in range(2, 9):
        g = gen.complete(n)
        assert E.kemeny_exact(g.offsets, g.indices) == pytest.approx(float(E.kemeny_complete(n)), rel=1e-12)
    for n in range(3, 12):
        g = gen.cycle(n)
        assert E.kemeny_exact(g.offsets, g.indices) == pytest.approx(float(E.kemeny_cycle(n)), rel=1e-12)
    for n in range(2, 12):
        g = gen.path(n)
        assert E.kemeny_exact(g.offsets, g.indices) == pytest.approx(float(E.kemeny_path(n)), rel=1e-12)
    for n in range(3, 12):
        g = gen.star(n)
        assert E.kemeny_exact(g.offsets, g.indices) == pytest.approx(float(E.kemeny_star(n)), rel=1e-12)
    for a, b in ((6, 8), (5, 7), (3, 3)):
        g = gen.torus(a, b)
        assert E.kemeny_exact(g.offsets, g.indices) == pytest.approx(E.kemeny_torus(a, b), rel=1e-12)
    for d in (3, 5, 8):
        g = gen.hypercube(d)
        assert E.kemeny_exact(g.offsets, g.indices) == pytest.approx(float(E.kemeny_hypercube(d)), rel=1e-11)


def test_kemeny_equals_hitting_time_definition(gen):
    """kappa = sum_j pi_j H(i, j) for every start i (the definition), against
    the spectral form of Eq. (1)."""
    from oracle import exact as E
    for g in (gen.gnm(12, 25, 3), gen.barabasi_albert(15, 2, 1), gen.grid(3, 4)):
        a = g.dense_adjacency()
        d = a.sum(1)
        p = a / d[:, None]
        n = g.n
        pi = d / d.sum()
        h = np.zeros((n, n))
        for j in range(n):
            keep = [i for i in range(n) if i != j]
            m = np.eye(n - 1) - p[np.ix_(keep, keep)]
            h[keep, j] = np.linalg.solve(m, np.ones(n - 1))
        kem = h @ pi
        assert np.allclose(kem, kem[0], rtol=1e-10)
        assert kem[0] == pytest.approx(E.kemeny_exact(g.offsets, g.indices), rel=1e-10)


# ------------------------------------------------------- f(tau) pins

def _tiny_graphs(gen):
    return [gen.complete(3), gen.complete(4), gen.complete(5), gen.cycle(5), gen.cycle(6),
            gen.path(5), gen.grid(3, 3), gen.grid(2, 4), gen.petersen(), gen.gnm(7, 11, 1)]


def test_enumeration_mean_equals_exact_kemeny(gen, oracle_lib):
    """Theorem 3.3 exactly: the mean of f/2m over ALL spanning trees is kappa;
    the enumerated tree count matches the matrix-tree theorem."""
    from oracle import exact as E
    for g in _tiny_graphs(gen):
        P = oracle_lib.prepare_graph(g)
        trees = E.spanning_trees(g.offsets, g.indices, P.root)
        assert len(trees) == E.tree_count(g.offsets, g.indices)
        for form in ("naive", "peredge", "walk"):
            fs = [oracle_lib.f_of_tree(P, t, form) for t in trees]
            mean = Fraction(sum(fs), len(fs) * g.two_m)
            assert float(mean) == pytest.approx(E.kemeny_exact(g.offsets, g.indices), rel=1e-12), (g.name, form)


def test_enumeration_with_non_bfs_tau0(gen, oracle_lib):
    """Theorems 3.2-3.4 hold for any fixed spanning tree tau0, not only BFS."""
    from oracle import exact as E
    for g in (gen.grid(3, 3), gen.petersen(), gen.gnm(7, 11, 1)):
        P = oracle_lib.prepare_graph(g)
        trees = E.spanning_trees(g.offsets, g.indices, P.root)
        K = E.kemeny_exact(g.offsets, g.indices)
        dfs = oracle_lib.dfs_tree(g.offsets, g.indices, P.root)
        for t0 in (trees[0], trees[len(trees) // 2], trees[-1], dfs):
            Q = oracle_lib.with_tau0(P, t0)
            for form in ("naive", "peredge", "walk"):
                fs = [oracle_lib.f_of_tree(Q, t, form) for t in trees]
                assert sum(fs) / (len(fs) * g.two_m) == pytest.approx(K, rel=1e-12)


def test_worked_triangle_example(gen, oracle_lib):
    ex = json.load(open(os.path.join(HERE, "golden", "k3_worked_example.json")))
    g = gen.complete(3)
    P = oracle_lib.prepare_graph(g)
    assert P.root == ex["root"]
    for key, fval in ex["bfs_tau0"]["f"].items():
        parent = np.array([int(x) for x in key.split(",")], np.int32)
        for form in ("naive", "peredge", "walk"):
            assert oracle_lib.f_of_tree(P, parent, form) == fval
    num, den = ex["bfs_tau0"]["kappa"]
    assert Fraction(sum(ex["bfs_tau0"]["f"].values()), 3 * g.two_m) == Fraction(num, den)
    Q = oracle_lib.with_tau0(P, ex["path_tau0"]["p0"])
    tot = 0
    for key, fval in ex["path_tau0"]["f"].items():
        parent = np.array([int(x) for x in key.split(",")], np.int32)
        for form in ("naive", "peredge", "walk"):
            assert oracle_lib.f_of_tree(Q, parent, form) == fval
        tot += fval
    assert tot == ex["path_tau0"]["sum_f_equals_2m_trees_kappa"]
    # the 2-forest side of the same example: sum_u d(u) sum vol(T1) = 2m |trees| kappa
    tf = ex["two_forests"]
    s = sum(2 * tf[F]["vol_T1"] for u, Fs in tf["separating"].items() for F in Fs)
    assert s == tot


@pytest.mark.parametrize("name", ["grid8", "grid12", "gnm60", "ba80"])
def test_forms_agree_on_sampled_trees(gen, oracle_lib, name):
    g = {"grid8": lambda: gen.grid(8, 8), "grid12": lambda: gen.grid(12, 12),
         "gnm60": lambda: gen.largest_component(gen.gnm(60, 150, 2)),
         "ba80": lambda: gen.barabasi_albert(80, 2, 5)}[name]()
    P = oracle_lib.prepare_graph(g)
    parents, _, _ = oracle_lib.sample(P, seed=11, s0=0, count=40)
    for t in parents:
        vals = {form: oracle_lib.f_of_tree(P, t, form) for form in ("naive", "peredge", "walk")}
        assert len(set(vals.values())) == 1, vals
        assert vals["naive"] > 0


def _exact_spread(oracle_lib, P, trees, two_m):
    """Exact mean, variance and fourth central moment of X = f(tau)/2m over
    uniform spanning trees, from the list of all of them (rationals)."""
    xs = [Fraction(oracle_lib.f_of_tree(P, t), two_m) for t in trees]
    N = len(xs)
    mu = sum(xs) / N
    var = sum((x - mu) ** 2 for x in xs) / N
    m4 = sum((x - mu) ** 4 for x in xs) / N
    return mu, var, m4


@pytest.mark.parametrize("name", ["grid3", "petersen"])
def test_standard_error_matches_exact_spread(gen, oracle_lib, name):
    """Theorem 3.3's estimate is the mean of omega i.i.d. values f(tau)/2m, so
    its standard error is their standard deviation over sqrt(omega).  The
    oracle's se times sqrt(omega) is checked against the exact standard
    deviation over ALL spanning trees (enumeration: 192 trees of the 3x3 grid,
    2,000 of the Petersen graph).  The tolerance is 4.5 sampling standard
    deviations of a sample variance, sqrt((mu4 - var^2) / omega), from the
    exact fourth moment."""
    from oracle import exact as E
    g = gen.grid(3, 3) if name == "grid3" else gen.petersen()
    P = oracle_lib.prepare_graph(g)
    trees = E.spanning_trees(g.offsets, g.indices, P.root)
    mu, var, m4 = _exact_spread(oracle_lib, P, trees, g.two_m)
    assert float(mu) == pytest.approx(E.kemeny_exact(g.offsets, g.indices), rel=1e-12)
    omega = 24000
    f, _ = oracle_lib.estimate_f(P, seed=17, s0=0, count=omega, threads=8)
    K, se, _, _ = oracle_lib.reduce_estimate(f, g.two_m)
    s2 = (se * math.sqrt(omega)) ** 2
    tol = 4.5 * math.sqrt(float(m4 - var * var) / omega)
    assert abs(s2 - float(var)) < tol, (s2, float(var), tol)
    # and the mean within 4.5 exact standard errors
    assert abs(K - float(mu)) < 4.5 * math.sqrt(float(var) / omega)


def test_interval_coverage_on_grid(gen, oracle_lib):
    """The interval K-hat +- 1.96 se (reading A10: a normal approximation in
    place of the Hoeffding bound of Theorem 3.6) covers the exact kappa of the
    3x3 grid (9.5) in about 95% of 800 independent estimates of 200 trees
    each; the tolerance is 4.5 binomial standard deviations.  An se off by a
    factor of two would cover about 67% or 99.99% of the time."""
    g = gen.grid(3, 3)
    P = oracle_lib.prepare_graph(g)
    reps, omega = 800, 200
    f, _ = oracle_lib.estimate_f(P, seed=29, s0=0, count=reps * omega, threads=8)
    cover = 0
    for r in range(reps):
        K, se, _, _ = oracle_lib.reduce_estimate(f[r * omega:(r + 1) * omega], g.two_m)
        cover += abs(K - 9.5) <= 1.959963984540054 * se
    p = cover / reps
    assert abs(p - 0.95) < 4.5 * math.sqrt(0.95 * 0.05 / reps), p


# --------------------------------------------------------- sampler pins

def test_root_and_bfs_rules(gen, oracle_lib):
    g = gen.grid(32, 32)
    P = oracle_lib.prepare_graph(g)
    assert P.root == 33          # first degree-4 vertex
    assert P.depth0 == 60        # eccentricity of (1,1) in the 32x32 grid
    # BFS parent = smallest-index neighbour one level up
    for v in range(g.n):
        if v == P.root:
            assert P.p0[v] == -1
            continue
        nb = g.indices[g.offsets[v]:g.offsets[v + 1]]
        ups = [u for u in nb if P.dist[u] == P.dist[v] - 1]
        assert P.p0[v] == min(ups)
    # preorder intervals nest exactly like subtrees of tau0
    for v in range(g.n):
        if v != P.root:
            u = P.p0[v]
            assert P.in0[u] < P.in0[v] <= P.out0[v] <= P.out0[u]


def test_dfs_tau0_rule(gen, oracle_lib):
    """The depth-first reference tree of section 5 (Exp-II)."""
    # hand-traced: 3x3 grid (id 3i+j) from 0, rows ascending:
    # 0 -> 1 -> 2 -> 5 -> 4 -> 3 -> 6 -> 7 -> 8, a Hamiltonian path
    g = gen.grid(3, 3)
    assert list(oracle_lib.dfs_tree(g.offsets, g.indices, 0)) == [-1, 0, 1, 4, 5, 2, 3, 6, 7]
    # K4 from 0: the chain 0-1-2-3; from 2: 2-0-1-3
    g = gen.complete(4)
    assert list(oracle_lib.dfs_tree(g.offsets, g.indices, 0)) == [-1, 0, 1, 2]
    assert list(oracle_lib.dfs_tree(g.offsets, g.indices, 2)) == [2, 0, -1, 1]
    # star from a leaf: the leaf's only neighbour, the centre, then every other leaf
    g = gen.star(6)
    assert list(oracle_lib.dfs_tree(g.offsets, g.indices, 3)) == [3, 0, 0, -1, 0, 0]
    # the defining property of a depth-first tree of an undirected graph: it
    # spans, and every graph edge joins a vertex to one of its tree ancestors
    for g in (gen.grid(8, 8), gen.largest_component(gen.gnm(60, 150, 3)), gen.barabasi_albert(80, 2, 1),
              gen.road_like(800, seed=2)):
        r = int(np.argmax(np.diff(g.offsets)))
        par = oracle_lib.dfs_tree(g.offsets, g.indices, r)
        depth = np.full(g.n, -1)
        depth[r] = 0
        for v in range(g.n):
            chain = []
            x = v
            while depth[x] < 0:
                chain.append(x)
                x = par[x]
                assert len(chain) <= g.n
            for i, y in enumerate(reversed(chain)):
                depth[y] = depth[x] + 1 + i
        assert par[r] == -1

        def is_anc(a, b):
            while depth[b] > depth[a]:
                b = par[b]
            return a == b
        for v in range(g.n):
            nb = g.indices[g.offsets[v]:g.offsets[v + 1]]
            if v != r:
                assert par[v] in nb
            for u in nb:
                assert is_anc(u, v) or is_anc(v, u)


def test_wilson_order_independent(gen, oracle_lib):
    """Cycle popping: parents and per-vertex draw counts do not depend on the
    order in which walks are started."""
    rng = np.random.default_rng(0)
    for g in (gen.grid(10, 10), gen.barabasi_albert(60, 2, 3), gen.largest_component(gen.gnm(50, 90, 4))):
        P = oracle_lib.prepare_graph(g)
        for s in range(15):
            base = oracle_lib.wilson(P, 99, s)
            for _ in range(3):
                order = rng.permutation(g.n).astype(np.int32)
                other = oracle_lib.wilson(P, 99, s, order)
                assert np.array_equal(base[0], other[0])
                assert np.array_equal(base[1], other[1])
                assert base[2] == other[2]


@pytest.mark.parametrize("name,count", [("K4", 8000), ("grid3", 19200), ("petersen", 60000)])
def test_tree_uniformity_chi2(gen, oracle_lib, name, count):
    from oracle import exact as E
    g = {"K4": lambda: gen.complete(4), "grid3": lambda: gen.grid(3, 3), "petersen": gen.petersen}[name]()
    P = oracle_lib.prepare_graph(g)
    trees = E.spanning_trees(g.offsets, g.indices, P.root)
    index = {t.tobytes(): i for i, t in enumerate(trees)}
    parents, _, _ = oracle_lib.sample(P, seed=2024, s0=0, count=count, threads=4)
    hits = np.zeros(len(trees), np.int64)
    for t in parents:
        hits[index[t.tobytes()]] += 1
    assert hits.sum() == count
    assert stats.chisquare(hits).pvalue > 1e-4


def test_mean_draws_equal_phi(gen, oracle_lib):
    """Expected Wilson work is Tr((I - P_r)^-1) (section 2.2, Theorem 3.5)."""
    from oracle import exact as E
    g = gen.grid(32, 32)
    P = oracle_lib.prepare_graph(g)
    phi = E.phi_exact(g.offsets, g.indices, P.root)
    _, steps = oracle_lib.estimate_f(P, seed=0, s0=0, count=2000, threads=8)
    se = steps.std(ddof=1) / np.sqrt(len(steps))
    assert abs(steps.mean() - phi) < 4.5 * se, (steps.mean(), phi, se)


def test_estimator_close_to_exact_kemeny(gen, oracle_lib):
    """Unbiasedness at scale: K-hat within 4.5 standard errors of exact K."""
    from oracle import exact as E
    for g, count in ((gen.grid(32, 32), 4000), (gen.torus(20, 20), 1000), (gen.hypercube(8), 400)):
        P = oracle_lib.prepare_graph(g)
        f, _ = oracle_lib.estimate_f(P, seed=5, s0=0, count=count, threads=8)
        K, se, _, _ = oracle_lib.reduce_estimate(f, g.two_m)
        Kx = E.kemeny_exact(g.offsets, g.indices)
        assert abs(K - Kx) < 4.5 * se, (g.name, K, Kx, se)


def test_estimator_close_to_exact_kemeny_on_workload_shapes(gen, oracle_lib):
    """Unbiasedness on the irregular shapes the measured workloads have, at
    the largest sizes a dense eigensolve finishes in seconds: a road-like
    graph (mean degree below 3, tau0 depth in the hundreds) and a power-law
    Chung-Lu graph (degrees up to hundreds), each about 7,500 vertices.
    K-hat from 2,000 trees lies within 4.5 standard errors of exact K."""
    from oracle import exact as E
    for g in (gen.road_like(10000, seed=2), gen.chung_lu(8000, 2.2, 10.0, 800.0, seed=3)):
        assert 7000 < g.n < 8000
        P = oracle_lib.prepare_graph(g)
        f, _ = oracle_lib.estimate_f(P, seed=7, s0=0, count=2000, threads=8)
        K, se, _, _ = oracle_lib.reduce_estimate(f, g.two_m)
        Kx = E.kemeny_exact(g.offsets, g.indices)
        assert abs(K - Kx) < 4.5 * se, (g.name, K, Kx, se)


def test_reduce_estimate_exact_sums(oracle_lib):
    f = np.array([2 ** 62, 2 ** 62, 2 ** 62, 5], np.int64)
    K, se, s1, s2 = oracle_lib.reduce_estimate(f, 10)
    assert s1 == 3 * 2 ** 62 + 5
    assert s2 == 3 * 2 ** 124 + 25
    assert K == float(3 * 2 ** 62 + 5) / 40.0


# ---------------------------------------------------------------- section 4

def _k4_tree_id(row):
    return tuple(int(x) for x in row)


def test_bsm_deletion_keeps_the_set_uniform(gen, oracle_lib):
    """Theorem 4.2 (deletion): after replacing the trees that contain the
    deleted edge, the set is uniform over the spanning trees of G' = K4 - e
    (8 trees), the replaced fraction is P(e in a UST of K4) = R_eff(e) = 1/2,
    untouched trees keep their sample index, and the estimate is unbiased on G'."""
    from oracle import exact as E
    g = gen.complete(4)
    S = oracle_lib.samples_init(g.offsets, g.indices, seed=5, count=4000)
    assert S.root == 0
    e = (1, 2)
    g2 = gen.remove_edges(g, [e])
    S2, replaced = oracle_lib.bsm_delete(S, g2.offsets, g2.indices, [e])
    # replaced fraction ~ 1/2 (4.5 sigma)
    assert abs(replaced / 4000 - 0.5) < 4.5 * math.sqrt(0.25 / 4000)
    kept = S2.ids < 4000
    assert np.array_equal(S2.parents[kept], S.parents[kept])
    assert sorted(S2.ids[~kept].tolist()) == list(range(4000, 4000 + replaced))
    # no tree uses the deleted edge; uniform over the 8 trees of K4 - e
    for row in S2.parents:
        assert row[1] != 2 and row[2] != 1
    trees = E.spanning_trees(g2.offsets, g2.indices, 0)
    assert len(trees) == 8
    counts = {}
    for row in S2.parents:
        counts[_k4_tree_id(row)] = counts.get(_k4_tree_id(row), 0) + 1
    assert len(counts) == 8
    expect = 4000 / 8
    chi2 = sum((c - expect) ** 2 / expect for c in counts.values())
    assert chi2 < 24.32  # 7 degrees of freedom, p = 0.001
    K, se, _, _ = oracle_lib.reduce_estimate(S2.f, g2.two_m)
    assert abs(K - E.kemeny_exact(g2.offsets, g2.indices)) < 4.5 * se


def test_bsm_deletion_estimate_unbiased_on_grid(gen, oracle_lib):
    """Three deletion batches on a 6x6 grid; after each the estimate over the
    maintained set matches the exact Kemeny constant of the current graph."""
    from oracle import exact as E
    g = gen.grid(6, 6)
    S = oracle_lib.samples_init(g.offsets, g.indices, seed=9, count=3000)
    batches = [[(7, 8)], [(14, 20), (21, 22)], [(1, 7), (28, 29)]]
    for batch in batches:
        g = gen.remove_edges(g, batch)
        assert gen.is_connected(g)
        S, replaced = oracle_lib.bsm_delete(S, g.offsets, g.indices, batch)
        assert replaced > 0
        K, se, _, _ = oracle_lib.reduce_estimate(S.f, g.two_m)
        assert abs(K - E.kemeny_exact(g.offsets, g.indices)) < 4.5 * se


def _resistance(offsets, indices, u, v):
    n = len(offsets) - 1
    L = np.zeros((n, n))
    for x in range(n):
        for y in indices[offsets[x]:offsets[x + 1]]:
            L[x, y] -= 1.0
            L[x, x] += 1.0
    Lp = np.linalg.pinv(L)
    return Lp[u, u] + Lp[v, v] - 2 * Lp[u, v]


@pytest.mark.parametrize("name,pairs", [("K4", [(1, 2), (0, 3)]), ("grid3", [(0, 8), (1, 4), (2, 6)]),
                                        ("petersen", [(0, 5), (2, 8)]), ("C6", [(0, 3), (1, 2)])])
def test_path_current_mean_is_effective_resistance(gen, oracle_lib, name, pairs):
    """Over all spanning trees, the signed path count has mean R(u, v) exactly
    (Kirchhoff's current flow), for adjacent and non-adjacent pairs."""
    g = {"K4": gen.complete(4), "grid3": gen.grid(3, 3), "petersen": gen.petersen(), "C6": gen.cycle(6)}[name]
    from oracle import exact as E
    P = oracle_lib.prepare_graph(g)
    trees = E.spanning_trees(g.offsets, g.indices, P.root)
    for u, v in pairs:
        path = oracle_lib.reference_path(g.offsets, g.indices, u, v)
        assert path[0] == u and path[-1] == v
        mean = sum(oracle_lib.path_current(t, path) for t in trees) / len(trees)
        assert abs(mean - _resistance(g.offsets, g.indices, u, v)) < 1e-12


def test_bsm_insertion_keeps_the_set_uniform(gen, oracle_lib):
    """Theorem 4.1 (insertion): from a uniform set on K4 - e, inserting e
    replaces a binomial share R_G'(e) = 1/2 of the trees by uniform trees through
    e; the set is then uniform over the 16 spanning trees of K4, untouched trees
    keep their index, and the estimate is unbiased on K4."""
    from oracle import exact as E
    g0 = gen.remove_edges(gen.complete(4), [(1, 2)])
    S = oracle_lib.samples_init(g0.offsets, g0.indices, seed=21, count=4000, root=0)
    g1 = gen.add_edges(g0, [(1, 2)])
    S2, replaced, rhat = oracle_lib.bsm_insert(S, g1.offsets, g1.indices, 1, 2, serial=0)
    assert abs(rhat - _resistance(g0.offsets, g0.indices, 1, 2)) < 0.05
    assert abs(replaced / 4000 - 0.5) < 4.5 * math.sqrt(0.25 / 4000) + 0.02
    kept = S2.ids < 4000
    assert np.array_equal(S2.parents[kept], S.parents[kept])
    for t in S2.parents[~kept]:
        assert t[1] == 2 or t[2] == 1  # replacements go through the new edge
        assert t[0] == -1
    counts = {}
    for row in S2.parents:
        counts[tuple(int(x) for x in row)] = counts.get(tuple(int(x) for x in row), 0) + 1
    assert len(counts) == 16
    expect = 4000 / 16
    chi2 = sum((c - expect) ** 2 / expect for c in counts.values())
    assert chi2 < 37.70  # 15 degrees of freedom, p = 0.001
    K, se, _, _ = oracle_lib.reduce_estimate(S2.f, g1.two_m)
    assert abs(K - E.kemeny_exact(g1.offsets, g1.indices)) < 4.5 * se


def test_bsm_mixed_updates_unbiased_on_grid(gen, oracle_lib):
    """Insertions and deletions on a 6x6 grid; the maintained estimate stays
    within the CLT interval of the exact Kemeny constant of the current graph."""
    from oracle import exact as E
    g = gen.grid(6, 6)
    S = oracle_lib.samples_init(g.offsets, g.indices, seed=13, count=3000)
    serial = 0
    for kind, e in [("add", (0, 35)), ("del", (7, 8)), ("add", (3, 20)), ("add", (10, 25)), ("del", (14, 20))]:
        if kind == "add":
            g = gen.add_edges(g, [e])
            S, _, _ = oracle_lib.bsm_insert(S, g.offsets, g.indices, e[0], e[1], serial)
            serial += 1
        else:
            g = gen.remove_edges(g, [e])
            S, _ = oracle_lib.bsm_delete(S, g.offsets, g.indices, [e])
        K, se, _, _ = oracle_lib.reduce_estimate(S.f, g.two_m)
        assert abs(K - E.kemeny_exact(g.offsets, g.indices)) < 4.5 * se


# ------------------------------------- improved sample maintenance (Algorithm 3)

def _ism_cases(gen):
    # (graph, non-edge to insert), (graph, non-bridge edge to delete)
    return [(gen.grid(3, 3), (0, 8)), (gen.cycle(6), (0, 3)), (gen.petersen(), (0, 2)),
            (gen.gnm(7, 11, 1), None), (gen.complete(4), None)]


def _non_edge(g):
    for x in range(g.n):
        row = set(int(y) for y in g.indices[g.offsets[x]:g.offsets[x + 1]])
        for y in range(x + 1, g.n):
            if y not in row:
                return (x, y)
    return None


def test_link_cut_bipartite_theorem_4_4(gen, oracle_lib):
    """Theorem 4.4 exactly, by enumeration.  Over all trees tau of G and all
    d(tau) link-cut choices, every spanning tree of G' = G + e through e is
    reached exactly d(tau_e) times (the number of edges of G joining the two
    parts of tau_e - e); hence the weighted mean of f' with weights
    d(tau)/d(tau_e) is the mean of f' over the trees of G' through e, and the
    weights themselves average R/(1-R) with R the share of G''s trees through e.
    Some new trees are reached more often than others, yet each carries the
    same total weight (the point Example 4.3 makes on a schematic case)."""
    from oracle import exact as E
    uneven = False
    for g, e in _ism_cases(gen):
        if e is None:
            e = _non_edge(g)
        if e is None:
            continue
        u, v = e
        root = oracle_lib.prepare_graph(g).root
        g2 = gen.add_edges(g, [e])
        P2 = oracle_lib.prepare(g2.offsets, g2.indices, root)
        old = E.spanning_trees(g.offsets, g.indices, root)
        new = E.spanning_trees(g2.offsets, g2.indices, root)
        through = {tuple(int(x) for x in t): t for t in new if t[u] == v or t[v] == u}
        reached = {k: 0 for k in through}
        weight_of = {k: Fraction(0) for k in through}
        wf = Fraction(0)
        wsum = Fraction(0)
        for t in old:
            up, dn = oracle_lib.tree_path(t, u, v)
            d = len(up) + len(dn)
            for j in range(d):
                te, d_old = oracle_lib.link_cut(t, u, v, j)
                assert d_old == d
                key = tuple(int(x) for x in te)
                assert key in through, (g.name, "link-cut left the trees of G' through e")
                reached[key] += 1
                d_new = len(oracle_lib.crossing_edges(g2.offsets, g2.indices, te, u, v)[0]) - 1
                w = Fraction(d, d_new) / d          # choice probability 1/d(tau), weight d(tau)/d(tau_e)
                wf += w * oracle_lib.f_of_tree(P2, te)
                wsum += w
                weight_of[key] += w
        for key, t in through.items():
            assert reached[key] == len(oracle_lib.crossing_edges(g2.offsets, g2.indices, t, u, v)[0]) - 1
        # reached unevenly, yet every new tree carries the same total weight (Example 4.3's point)
        uneven |= len(set(reached.values())) > 1
        assert set(weight_of.values()) == {Fraction(1)}
        mean_through = Fraction(sum(oracle_lib.f_of_tree(P2, t) for t in through.values()), len(through))
        assert wf / wsum == mean_through
        assert wsum / len(old) == Fraction(len(through), len(old))   # = R / (1 - R)
    assert uneven


def test_cut_link_bipartite_theorem_4_5(gen, oracle_lib):
    """Theorem 4.5 exactly, by enumeration: over all trees of G through e and all
    cut-link choices, every spanning tree of G' = G - e is reached exactly
    d(tau') times (the length of its tree path between the endpoints of e), so
    weights d(tau)/d(tau') (old over new, as in the theorem) give the mean of f'
    over all trees of G'.  The weight printed in Algorithm 3's deletion branch,
    d(tau')/d(tau), gives a different mean on some of these graphs."""
    from oracle import exact as E
    printed_differs = False
    for g, _ in _ism_cases(gen):
        src = np.repeat(np.arange(g.n), np.diff(g.offsets))
        cand = [(int(a), int(b)) for a, b in zip(src, g.indices) if a < b]
        root = oracle_lib.prepare_graph(g).root
        for a, b in cand[:: max(1, len(cand) // 3)]:
            g2 = gen.remove_edges(g, [(a, b)])
            if not gen.is_connected(g2):
                continue
            P2 = oracle_lib.prepare(g2.offsets, g2.indices, root)
            old = [t for t in E.spanning_trees(g.offsets, g.indices, root) if t[a] == b or t[b] == a]
            new = {tuple(int(x) for x in t): t for t in E.spanning_trees(g2.offsets, g2.indices, root)}
            reached = {k: 0 for k in new}
            wf = wsum = pf = psum = Fraction(0)
            for t in old:
                d = len(oracle_lib.crossing_edges(g2.offsets, g2.indices, t, a, b)[0])
                for j in range(d):
                    tn, d_old = oracle_lib.cut_link(t, g2.offsets, g2.indices, a, b, j)
                    assert d_old == d
                    key = tuple(int(x) for x in tn)
                    assert key in new
                    reached[key] += 1
                    up, dn = oracle_lib.tree_path(tn, a, b)
                    d_new = len(up) + len(dn)
                    f = oracle_lib.f_of_tree(P2, tn)
                    wf += Fraction(d, d_new) / d * f
                    wsum += Fraction(d, d_new) / d
                    pf += Fraction(d_new, d) / d * f
                    psum += Fraction(d_new, d) / d
            for key, t in new.items():
                up, dn = oracle_lib.tree_path(t, a, b)
                assert reached[key] == len(up) + len(dn)
            mean_new = Fraction(sum(oracle_lib.f_of_tree(P2, t) for t in new.values()), len(new))
            assert wf / wsum == mean_new
            printed_differs |= pf / psum != mean_new
    assert printed_differs


def test_ism_estimate_tracks_exact_kemeny(gen, oracle_lib):
    """Algorithm 3 end to end on a 4x4 grid: an insertion, then a deletion of
    an edge, each over 120 independent sets of 24 trees.  The mean
    weighted estimate is within 4 standard errors of the exact kappa of the
    new graph, and the weights always sum to one."""
    from oracle import exact as E
    g0 = gen.grid(4, 4)
    g1 = gen.add_edges(g0, [(0, 15)])
    g2 = gen.remove_edges(g1, [(5, 6)])
    k1 = E.kemeny_exact(g1.offsets, g1.indices)
    k2 = E.kemeny_exact(g2.offsets, g2.indices)
    e1, e2, b1, b2 = [], [], [], []
    for seed in range(120):
        W = oracle_lib.ism_init(g0.offsets, g0.indices, seed=seed, count=24, threads=1)
        W, _ = oracle_lib.ism_insert(W, g1.offsets, g1.indices, 0, 15)
        assert abs(sum(W.w) - 1.0) < 1e-12
        k_, b_ = oracle_lib.weighted_estimate(W)
        e1.append(k_)
        b1.append(b_)
        W, _ = oracle_lib.ism_delete(W, g2.offsets, g2.indices, 5, 6)
        assert abs(sum(W.w) - 1.0) < 1e-12
        k_, b_ = oracle_lib.weighted_estimate(W)
        e2.append(k_)
        b2.append(b_)
    for est, bars, k in ((e1, b1, k1), (e2, b2, k2)):
        est = np.array(est)
        se = est.std(ddof=1) / math.sqrt(len(est))
        assert abs(est.mean() - k) < 4 * se + 1e-3 * k, (est.mean(), k, se)
        # the error bar of each weighted estimate (reading A30) against the
        # spread of the 120 independent estimates: the mean squared bar and the
        # empirical variance agree within 4.5 standard deviations of a sample
        # variance of 120 values (relative sd sqrt(2/119) for a normal spread)
        ratio = float(np.mean(np.square(bars))) / float(est.var(ddof=1))
        assert abs(ratio - 1.0) < 4.5 * math.sqrt(2.0 / 119.0), ratio
