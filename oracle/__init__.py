"""CPU oracle for the 2-forest-sampling Kemeny-constant estimator.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no
code with the GPU library (``paper_2511_16356_amd``) and never imports it.

``kc_oracle.c`` (plain C, gcc) holds the sampler and the four forms of
f(tau); ``exact.py`` (numpy/scipy, FP64) holds the exact Kemeny constant, the
expected Wilson work, closed forms and spanning-tree enumeration used to pin
the oracle to the mathematics.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import math
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kc_oracle.c")
_LIB = os.path.join(_HERE, "libkc_oracle.so")
_lib = None

F_NAIVE, F_PEREDGE, F_WALK = 1, 3, 4
# f(tau) in three independent forms: the definition of Theorem 3.3 (naive), the
# per-edge sums of Theorem 3.4 (peredge, the default) and the tau0-ancestor walk
# of the complexity remark after Theorem 3.5 (walk)
FORMS = {"naive": F_NAIVE, "peredge": F_PEREDGE, "walk": F_WALK}

ERRORS = {1: "invalid graph", 2: "graph is disconnected", 3: "out of memory", 6: "step limit"}


def build(force: bool = False) -> str:
    """Compile kc_oracle.c into libkc_oracle.so (gcc -O2 -pthread)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-pthread", "-shared", "-fPIC",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        p, i64, i32, u64, u32 = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                 ctypes.c_uint64, ctypes.c_uint32)
        lib.orc_philox.restype = None
        lib.orc_philox.argtypes = [p, p, p]
        lib.orc_arrow.restype = u32
        lib.orc_arrow.argtypes = [u64, u64, u32, u32, u32]
        lib.orc_prepare.restype = ctypes.c_int
        lib.orc_prepare.argtypes = [i64, p, p, i32, p, p, p, p, p, p]
        lib.orc_wilson_two_roots.restype = ctypes.c_int
        lib.orc_wilson_two_roots.argtypes = [i64, p, p, i32, i32, u64, u64, p, p, p]
        lib.orc_wilson_order.restype = ctypes.c_int
        lib.orc_wilson_order.argtypes = [i64, p, p, i32, u64, u64, p, p, p, p]
        lib.orc_f.restype = ctypes.c_int
        lib.orc_f.argtypes = [i64, p, i32, p, p, p, p, ctypes.c_int, p]
        lib.orc_sample.restype = ctypes.c_int
        lib.orc_sample.argtypes = [i64, p, p, i32, u64, i64, i64, ctypes.c_int, i64, p, p, p]
        lib.orc_estimate.restype = ctypes.c_int
        lib.orc_estimate.argtypes = [i64, p, p, i32, p, p, p, u64, i64, i64, ctypes.c_int,
                                     ctypes.c_int, i64, p, p]
        lib.orc_estimate_ids.restype = ctypes.c_int
        lib.orc_estimate_ids.argtypes = [i64, p, p, i32, p, p, p, u64, p, i64, ctypes.c_int,
                                         ctypes.c_int, i64, p, p]
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _check(st: int):
    if st != 0:
        raise RuntimeError("oracle: " + ERRORS.get(st, "error %d" % st))


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    _load().orc_philox(_ptr(c), _ptr(k), _ptr(out))
    return out


def arrow(seed: int, s: int, v: int, k: int, deg: int) -> int:
    return int(_load().orc_arrow(seed, s, v, k, deg))


@dataclass
class Prepared:
    """Graph with root, BFS tree tau0 and tau0 numbering (oracle side)."""

    n: int
    offsets: np.ndarray
    indices: np.ndarray
    root: int
    p0: np.ndarray
    dist: np.ndarray
    in0: np.ndarray
    out0: np.ndarray
    depth0: int

    @property
    def two_m(self) -> int:
        return int(self.offsets[-1])

    @property
    def degrees(self) -> np.ndarray:
        return np.diff(self.offsets)


def prepare(offsets, indices, root: int = -1) -> Prepared:
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    adj = np.ascontiguousarray(indices, dtype=np.int32)
    n = off.shape[0] - 1
    p0 = np.zeros(n, np.int32); dist = np.zeros(n, np.int32)
    in0 = np.zeros(n, np.int32); out0 = np.zeros(n, np.int32)
    r = ctypes.c_int32(); dep = ctypes.c_int32()
    _check(_load().orc_prepare(n, _ptr(off), _ptr(adj), root, ctypes.byref(r), _ptr(p0),
                               _ptr(dist), _ptr(in0), _ptr(out0), ctypes.byref(dep)))
    return Prepared(n, off, adj, int(r.value), p0, dist, in0, out0, int(dep.value))


def prepare_graph(g, root: int = -1) -> Prepared:
    return prepare(g.offsets, g.indices, root)


def with_tau0(P: Prepared, p0) -> Prepared:
    """Same graph and root, but an arbitrary fixed spanning tree tau0 given by
    its parent array (root -> -1); recomputes its preorder numbering."""
    p0 = np.ascontiguousarray(p0, dtype=np.int32)
    n = P.n
    children = [[] for _ in range(n)]
    for v in range(n):
        if v != P.root:
            children[int(p0[v])].append(v)
    in0 = np.zeros(n, np.int32); out0 = np.zeros(n, np.int32)
    t = 0
    stack = [(P.root, 0)]
    in0[P.root] = t; t += 1
    while stack:
        x, i = stack.pop()
        if i < len(children[x]):
            stack.append((x, i + 1))
            c = children[x][i]
            in0[c] = t; t += 1
            stack.append((c, 0))
        else:
            out0[x] = t - 1
    return Prepared(n, P.offsets, P.indices, P.root, p0, P.dist, in0, out0, P.depth0)


def dfs_tree(offsets, indices, root: int) -> np.ndarray:
    """Depth-first spanning tree from `root` (one of the reference-tree choices
    compared in section 5, Exp-II): the search scans each row in ascending
    order and a vertex's parent is the vertex it was first reached from.
    Returns the parent array (root -> -1)."""
    off = np.asarray(offsets, dtype=np.int64)
    adj = np.asarray(indices, dtype=np.int32)
    n = len(off) - 1
    parent = np.full(n, -1, np.int32)
    seen = np.zeros(n, bool)
    seen[root] = True
    stack = [(root, int(off[root]))]   # (vertex, next row position to scan)
    while stack:
        x, e = stack[-1]
        if e == off[x + 1]:
            stack.pop()
            continue
        stack[-1] = (x, e + 1)
        y = int(adj[e])
        if not seen[y]:
            seen[y] = True
            parent[y] = x
            stack.append((y, int(off[y])))
    return parent


def wilson(P: Prepared, seed: int, s: int, order=None):
    """One Wilson tree: (parent [n] int32 with root -1, draws [n] uint32, total draws)."""
    n = P.n
    parent = np.zeros(n, np.int32); cnt = np.zeros(n, np.uint32)
    steps = ctypes.c_int64()
    o = None if order is None else np.ascontiguousarray(order, dtype=np.int32)
    _check(_load().orc_wilson_order(n, _ptr(P.offsets), _ptr(P.indices), P.root, seed, s,
                                    _ptr(o), _ptr(parent), _ptr(cnt), ctypes.byref(steps)))
    return parent, cnt, int(steps.value)


def f_of_tree(P: Prepared, parent, form: str = "peredge") -> int:
    par = np.ascontiguousarray(parent, dtype=np.int32)
    f = ctypes.c_int64()
    _check(_load().orc_f(P.n, _ptr(P.offsets), P.root, _ptr(P.p0), _ptr(P.in0), _ptr(P.out0),
                         _ptr(par), FORMS[form], ctypes.byref(f)))
    return int(f.value)


def sample(P: Prepared, seed: int, s0: int, count: int, threads: int = 1, max_steps: int = 0):
    """Trees for samples s0..s0+count-1: parents [count, n], draws [count, n], totals [count]."""
    n = P.n
    parents = np.zeros((count, n), np.int32)
    cnts = np.zeros((count, n), np.uint32)
    steps = np.zeros(count, np.int64)
    _check(_load().orc_sample(n, _ptr(P.offsets), _ptr(P.indices), P.root, seed, s0, count,
                              threads, max_steps, _ptr(parents), _ptr(cnts), _ptr(steps)))
    return parents, cnts, steps


def estimate_f(P: Prepared, seed: int, s0: int, count: int, threads: int = 1,
               form: str = "peredge", max_steps: int = 0):
    """Per-sample f (int64) and total draws for samples s0..s0+count-1."""
    f = np.zeros(count, np.int64)
    steps = np.zeros(count, np.int64)
    _check(_load().orc_estimate(P.n, _ptr(P.offsets), _ptr(P.indices), P.root, _ptr(P.p0),
                                _ptr(P.in0), _ptr(P.out0), seed, s0, count, threads,
                                FORMS[form], max_steps, _ptr(f), _ptr(steps)))
    return f, steps


def estimate_ids(P: Prepared, seed: int, ids, threads: int = 1, form: str = "peredge",
                 max_steps: int = 0):
    """Per-sample f (int64) and total draws for the listed sample ids."""
    ids = np.ascontiguousarray(ids, dtype=np.int64)
    count = int(ids.shape[0])
    f = np.zeros(count, np.int64)
    steps = np.zeros(count, np.int64)
    _check(_load().orc_estimate_ids(P.n, _ptr(P.offsets), _ptr(P.indices), P.root, _ptr(P.p0),
                                    _ptr(P.in0), _ptr(P.out0), seed, _ptr(ids), count, threads,
                                    FORMS[form], max_steps, _ptr(f), _ptr(steps)))
    return f, steps


def reduce_estimate(f, two_m: int):
    """Theorem 3.3's estimator from exact per-sample values.

    Returns (K, stderr, sum_f, sum_f2): sum_f and sum_f2 are exact Python
    integers; K = float(sum_f) / (2m * count) (one correctly-rounded integer to
    double conversion, one double division); stderr is the sample standard
    deviation of f/2m over sqrt(count), from the exact sums."""
    vals = [int(x) for x in np.asarray(f, dtype=np.int64)]
    w = len(vals)
    s1 = sum(vals)
    s2 = sum(x * x for x in vals)
    K = float(s1) / float(two_m * w)
    if w > 1:
        mean = float(s1) / w
        var = (float(s2) - w * mean * mean) / (w - 1)
        se = math.sqrt(max(var, 0.0) / w) / two_m
    else:
        se = float("nan")
    return K, se, s1, s2


# ------------------------------------------------------ basic sample maintenance

@dataclass
class SampleSet:
    """The sample set S of section 4: trees kept between updates, with the
    sample index each was drawn with and its f on the current graph."""
    offsets: np.ndarray
    indices: np.ndarray
    root: int
    seed: int
    parents: np.ndarray  # [count, n] int32
    ids: np.ndarray      # [count] int64
    next_id: int
    f: np.ndarray        # [count] int64

    @property
    def two_m(self) -> int:
        return int(self.offsets[-1])


def samples_init(offsets, indices, seed: int, count: int, root: int = -1, threads: int = 8) -> SampleSet:
    """Samples 0..count-1 of the graph, kept as a set."""
    P = prepare(offsets, indices, root)
    parents, _, _ = sample(P, seed, 0, count, threads=threads)
    f = np.array([f_of_tree(P, t) for t in parents], np.int64)
    return SampleSet(P.offsets, P.indices, P.root, seed, parents, np.arange(count, dtype=np.int64), count, f)


def bsm_delete(S: SampleSet, offsets_new, indices_new, edges, threads: int = 8):
    """Algorithm 2 (basic sample maintenance), deletion case, for a batch of
    edges removed at once: the trees that contain a deleted edge are replaced
    by fresh uniform spanning trees of G' (the set's seed, the next unused
    sample indices in slot order); the others are uniform spanning trees of
    G' already (Theorem 4.2).  f is evaluated on G' for every tree, since the
    degrees, 2m and tau0 (rebuilt on G' from the same root) change.
    Returns (new set, number of replaced trees)."""
    P = prepare(offsets_new, indices_new, S.root)
    par = S.parents.copy()
    ids = S.ids.copy()
    redo = []
    for t in range(par.shape[0]):
        row = par[t]
        for a, b in edges:
            if row[a] == b or row[b] == a:
                redo.append(t)
                break
    if redo:
        fresh, _, _ = sample(P, S.seed, S.next_id, len(redo), threads=threads)
        for k, t in enumerate(redo):
            par[t] = fresh[k]
            ids[t] = S.next_id + k
    f = np.array([f_of_tree(P, t) for t in par], np.int64)
    return SampleSet(P.offsets, P.indices, P.root, S.seed, par, ids, S.next_id + len(redo), f), len(redo)


# ------------------------------------------- basic sample maintenance: inserts

def update_uniform(seed: int, slot: int, serial: int) -> float:
    """The replacement draw of resident tree `slot` at insertion number
    `serial`: Philox4x32-10 with key (seed_lo, seed_hi) and counter
    (slot, serial, 2^32-1, 2^32-1) (a counter no tree sample uses), x = o0 |
    o1 << 32, uniform = (x >> 11) * 2^-53 in [0, 1)."""
    o = philox4x32_10([slot, serial, 0xFFFFFFFF, 0xFFFFFFFF], [seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF])
    x = int(o[0]) | (int(o[1]) << 32)
    return (x >> 11) * 2.0 ** -53


def reference_path(offsets, indices, u: int, v: int) -> list:
    """A fixed u -> v path: breadth-first search from u (rows ascending), each
    vertex reached from the first vertex that reaches it."""
    n = len(offsets) - 1
    pred = np.full(n, -1, np.int64)
    pred[u] = u
    q = [u]
    h = 0
    while h < len(q) and pred[v] < 0:
        x = q[h]
        h += 1
        for y in indices[offsets[x]:offsets[x + 1]]:
            if pred[y] < 0:
                pred[y] = x
                q.append(int(y))
    path = [v]
    while path[-1] != u:
        path.append(int(pred[path[-1]]))
    return path[::-1]


def path_current(parent, path) -> int:
    """Signed number of edges of `path` that the tree's own u -> v path uses,
    +1 in the path's direction and -1 against it.  Its mean over uniform
    spanning trees is the effective resistance R(u, v): the tree path's
    direction on an edge has mean equal to the unit u -> v current there
    (Kirchhoff), and the currents summed along any u -> v path give the
    potential difference."""
    u, v = path[0], path[-1]

    def ancestors(x):
        out = set()
        while x != -1:
            out.add(int(x))
            x = int(parent[x])
        return out

    au, av = ancestors(u), ancestors(v)
    up, dn = au - av, av - au  # tree path: up from u to the meeting point, then down to v
    c = 0
    for a, b in zip(path[:-1], path[1:]):
        if (a in up and parent[a] == b) or (b in dn and parent[b] == a):
            c += 1
        elif (b in up and parent[b] == a) or (a in dn and parent[a] == b):
            c -= 1
    return c


def wilson_two_roots(P: Prepared, u: int, v: int, seed: int, s: int):
    n = P.n
    parent = np.zeros(n, np.int32); cnt = np.zeros(n, np.uint32)
    steps = ctypes.c_int64()
    _check(_load().orc_wilson_two_roots(n, _ptr(P.offsets), _ptr(P.indices), u, v, seed, s,
                                        _ptr(parent), _ptr(cnt), ctypes.byref(steps)))
    return parent


def bsm_insert(S: SampleSet, offsets_new, indices_new, u: int, v: int, serial: int):
    """Algorithm 2 (basic sample maintenance), insertion of edge (u, v):
    R(u, v) on the old graph is estimated from the set's own trees
    (path_current), each tree is replaced independently with probability
    R_G'(e) = R / (1 + R) (Theorem 4.1; a binomial number of replacements,
    each tree drawn by update_uniform), and every replacement is a uniform
    spanning tree of G' through e: Wilson's algorithm with u and v both in the
    tree, then the edge (v -> u) and the path from r re-oriented toward r.
    f is evaluated on G' for every tree.  Returns (new set, replaced, R-hat)."""
    path = reference_path(S.offsets, S.indices, u, v)
    csum = sum(path_current(t, path) for t in S.parents)
    count = S.parents.shape[0]
    rhat = csum / count
    p = rhat / (1.0 + rhat) if rhat > 0.0 else 0.0  # a share of trees: an estimate R <= 0 replaces none
    redo = [t for t in range(count) if update_uniform(S.seed, t, serial) < p]
    P = prepare(offsets_new, indices_new, S.root)
    par = S.parents.copy()
    ids = S.ids.copy()
    for k, t in enumerate(redo):
        tree = wilson_two_roots(P, u, v, S.seed, S.next_id + k)
        tree[v] = u
        prev, x = -1, P.root
        while x != -1:
            nx = int(tree[x])
            tree[x] = prev
            prev, x = x, nx
        par[t] = tree
        ids[t] = S.next_id + k
    f = np.array([f_of_tree(P, t) for t in par], np.int64)
    return (SampleSet(P.offsets, P.indices, P.root, S.seed, par, ids, S.next_id + len(redo), f),
            len(redo), rhat)


# ---------------------------------------- improved sample maintenance (ISM)

def ism_draw(seed: int, slot: int, serial: int, count: int) -> int:
    """The link-cut or cut-link choice for resident tree `slot` at update
    number `serial`: Philox4x32-10, key (seed_lo, seed_hi), counter
    (slot, serial, 2^32-2, 2^32-1) (a counter no tree sample uses), x = o0 |
    o1 << 32, choice floor(x * count / 2^64) in [0, count)."""
    o = philox4x32_10([slot, serial, 0xFFFFFFFE, 0xFFFFFFFF], [seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF])
    x = int(o[0]) | (int(o[1]) << 32)
    return (x * count) >> 64


def tree_path(parent, u: int, v: int):
    """The tree path between u and v: (vertices from u up to, not including,
    the lowest common ancestor; the same from v)."""
    av = set()
    y = v
    while y != -1:
        av.add(int(y))
        y = int(parent[y])
    up = []
    x = u
    while x not in av:
        up.append(int(x))
        x = int(parent[x])
    dn = []
    y = v
    while y != x:
        dn.append(int(y))
        y = int(parent[y])
    return up, dn


def link_cut(parent, u: int, v: int, j: int):
    """link-cut(tau, e) of section 4.2: add e = {u, v} to the tree, which closes
    a cycle with the tree path between u and v, and remove the j-th edge of that
    path (edges {x, p(x)} for x on u's side from u upward, then on v's side from
    v upward).  The cut-off part is re-hung through e, so the result is rooted
    at r again.  Returns (new parent array, d(tau) = length of the path)."""
    up, dn = tree_path(parent, u, v)
    d = len(up) + len(dn)
    new = np.array(parent, dtype=np.int32, copy=True)
    side, other = (up[: j + 1], v) if j < len(up) else (dn[: j - len(up) + 1], u)
    prev = other
    for x in side:
        new[x] = prev
        prev = x
    return new, d


def in_subtree(parent, c: int) -> np.ndarray:
    """inside[x] = c is x or one of x's tree ancestors."""
    n = len(parent)
    inside = np.zeros(n, bool)
    known = np.zeros(n, bool)
    inside[c] = True
    known[c] = True
    for x in range(n):
        chain = []
        y = x
        while y != -1 and not known[y]:
            chain.append(y)
            y = int(parent[y])
        val = bool(inside[y]) if y != -1 else False
        for z in chain:
            inside[z] = val
            known[z] = True
    return inside


def crossing_edges(offsets, indices, parent, a: int, b: int):
    """The graph edges {x, y} (x < y, rows in ascending order) that join the
    two trees left when the tree edge {a, b} is removed.  Returns (edges, c,
    inside) with c the endpoint on the side away from the root."""
    c = a if parent[a] == b else b
    assert parent[c] == (b if c == a else a), "{a, b} is not a tree edge"
    inside = in_subtree(parent, c)
    n = len(offsets) - 1
    out = []
    for x in range(n):
        for y in indices[offsets[x]:offsets[x + 1]]:
            y = int(y)
            if x < y and inside[x] != inside[y]:
                out.append((x, y))
    return out, c, inside


def cut_link(parent, offsets, indices, a: int, b: int, j: int):
    """cut-link(tau, e) of section 4.2: remove the tree edge e = {a, b} and
    join the two parts by the j-th of the crossing edges of the graph (in the
    order of crossing_edges); the detached part is re-hung through it, so the
    result is rooted at r again.  Returns (new parent array, d(tau) = number
    of crossing edges)."""
    cross, c, inside = crossing_edges(offsets, indices, parent, a, b)
    x, y = cross[j]
    xi, yo = (x, y) if inside[x] else (y, x)
    new = np.array(parent, dtype=np.int32, copy=True)
    prev, z = yo, xi
    while True:
        nz = int(parent[z])
        new[z] = prev
        if z == c:
            break
        prev, z = z, nz
    return new, len(cross)


@dataclass
class WeightedSet:
    """The sample set of Algorithm 3: trees with weights that sum to one."""
    S: SampleSet
    w: np.ndarray   # [count] float64
    serial: int     # single-edge updates applied so far (counter of their draws)


def ism_init(offsets, indices, seed: int, count: int, root: int = -1, threads: int = 8) -> WeightedSet:
    S = samples_init(offsets, indices, seed, count, root, threads)
    return WeightedSet(S, np.full(count, 1.0 / count), 0)


def weighted_estimate(W: WeightedSet):
    """kappa-hat = sum_t w_t f_t / 2m over the set (weights sum to one), summed
    in slot order; its standard error sqrt(sum_t w_t^2 (f_t/2m - kappa-hat)^2)."""
    two_m = float(W.S.two_m)
    k = 0.0
    for t in range(len(W.w)):
        k += W.w[t] * float(W.S.f[t])
    k /= two_m
    v = 0.0
    for t in range(len(W.w)):
        dlt = float(W.S.f[t]) / two_m - k
        v += W.w[t] * W.w[t] * dlt * dlt
    return k, math.sqrt(v)


def _normalise(w, group, target):
    s = 0.0
    for t in group:
        s += w[t]
    for t in group:
        w[t] *= target / s


def ism_insert(W: WeightedSet, offsets_new, indices_new, u: int, v: int):
    """Algorithm 3, insertion of e = {u, v}.  R(u, v) on the old graph is
    estimated from the set's own trees, weighted (the path-current count of
    bsm_insert); R' = R / (1 + R) is the share of spanning trees of G' that
    contain e (Theorem 4.1).  ceil(R' |S|) trees are chosen uniformly at
    random (the slots with the smallest update_uniform(seed, slot, serial)),
    each is taken through link-cut with the choice ism_draw(seed, slot, serial,
    d(tau)) and its weight multiplied by d(tau) / d(tau_e), where d(tau_e) is
    the number of edges of the old graph that join the two parts of tau_e - e
    (Theorem 4.4).  The chosen trees' weights are then scaled to sum to R' and
    the others' to 1 - R'; a group that is empty leaves the whole mass to the
    other.  f is evaluated on G' for every tree.  Returns (new set, chosen)."""
    S = W.S
    count = S.parents.shape[0]
    path = reference_path(S.offsets, S.indices, u, v)
    rhat = 0.0
    for t in range(count):
        rhat += W.w[t] * path_current(S.parents[t], path)
    rp = rhat / (1.0 + rhat) if rhat > 0.0 else 0.0
    k = min(count, int(math.ceil(rp * count)))
    order = sorted(range(count), key=lambda t: (update_uniform(S.seed, t, W.serial), t))
    chosen = sorted(order[:k])
    rest = sorted(order[k:])
    par = S.parents.copy()
    w = W.w.copy()
    for t in chosen:
        up, dn = tree_path(par[t], u, v)
        d_old = len(up) + len(dn)
        par[t], _ = link_cut(par[t], u, v, ism_draw(S.seed, t, W.serial, d_old))
        cross, _, _ = crossing_edges(offsets_new, indices_new, par[t], u, v)
        d_new = len(cross) - 1          # e itself crosses in G'
        w[t] *= float(d_old) / float(d_new)
    if chosen and rest:
        _normalise(w, chosen, rp)
        _normalise(w, rest, 1.0 - rp)
    else:
        _normalise(w, chosen or rest, 1.0)
    P = prepare(offsets_new, indices_new, S.root)
    f = np.array([f_of_tree(P, t) for t in par], np.int64)
    S2 = SampleSet(P.offsets, P.indices, P.root, S.seed, par, S.ids.copy(), S.next_id, f)
    return WeightedSet(S2, w, W.serial + 1), len(chosen)


def ism_delete(W: WeightedSet, offsets_new, indices_new, a: int, b: int):
    """Algorithm 3, deletion of e = {a, b}: every tree that contains e is taken
    through cut-link on G' with the choice ism_draw(seed, slot, serial, d(tau)),
    d(tau) being the number of edges of G' that join the two parts of tau - e,
    and its weight multiplied by d(tau) / d(tau'), with d(tau') the length of
    the tree path between a and b in the new tree (Theorem 4.5).  The changed
    trees' weights are then scaled to sum to their total before the update.
    f is evaluated on G' for every tree.  Returns (new set, changed)."""
    S = W.S
    count = S.parents.shape[0]
    par = S.parents.copy()
    w = W.w.copy()
    hit = [t for t in range(count) if par[t][a] == b or par[t][b] == a]
    w_org = 0.0
    for t in hit:
        w_org += w[t]
    for t in hit:
        cross, _, _ = crossing_edges(offsets_new, indices_new, par[t], a, b)
        d_old = len(cross)
        par[t], _ = cut_link(par[t], offsets_new, indices_new, a, b, ism_draw(S.seed, t, W.serial, d_old))
        up, dn = tree_path(par[t], a, b)
        w[t] *= float(d_old) / float(len(up) + len(dn))
    if hit:
        _normalise(w, hit, w_org)
    P = prepare(offsets_new, indices_new, S.root)
    f = np.array([f_of_tree(P, t) for t in par], np.int64)
    S2 = SampleSet(P.offsets, P.indices, P.root, S.seed, par, S.ids.copy(), S.next_id, f)
    return WeightedSet(S2, w, W.serial + 1), len(hit)
