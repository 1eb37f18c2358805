"""Seeded synthetic input graphs (input side only; no part of the method).

Every graph is returned as a canonical CSR: int64 ``offsets`` of length n+1,
int32 ``indices`` with ascending rows, no self-loops, no duplicates, and the
graph connected (generators keep the largest connected component and
relabel it preserving vertex order).

Both the CPU oracle and the GPU library consume these arrays; this module
holds no Kemeny-constant arithmetic.  The heavy generators (random geometric
graphs, Chung-Lu) live in ``graphgen.c`` and are loaded through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import math

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB = os.path.join(_HERE, "libgraphgen.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile graphgen.c into libgraphgen.so next to it (gcc -O2)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        i64, p = ctypes.c_int64, ctypes.c_void_p
        lib.gg_build_csr.restype = i64
        lib.gg_build_csr.argtypes = [i64, i64, p, p, p, p]
        lib.gg_rgg_edges.restype = i64
        lib.gg_rgg_edges.argtypes = [i64, ctypes.c_double, ctypes.c_double, ctypes.c_uint64, p, p, i64]
        lib.gg_chung_lu_edges.restype = i64
        lib.gg_chung_lu_edges.argtypes = [i64, p, ctypes.c_uint64, p, p, i64]
        lib.gg_lcc.restype = i64
        lib.gg_lcc.argtypes = [i64, p, p, p, p]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


@dataclass
class Graph:
    """Canonical undirected simple graph in CSR form."""

    name: str
    offsets: np.ndarray  # int64 [n+1]
    indices: np.ndarray  # int32 [2m]
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def two_m(self) -> int:
        return int(self.offsets[-1])

    @property
    def degrees(self) -> np.ndarray:
        return np.diff(self.offsets)

    def dense_adjacency(self) -> np.ndarray:
        n = self.n
        a = np.zeros((n, n), dtype=np.float64)
        rows = np.repeat(np.arange(n), self.degrees)
        a[rows, self.indices] = 1.0
        return a

    def edges(self) -> np.ndarray:
        """Undirected edges (u < v) as an int64 array [m, 2]."""
        rows = np.repeat(np.arange(self.n, dtype=np.int64), self.degrees)
        cols = self.indices.astype(np.int64)
        keep = rows < cols
        return np.stack([rows[keep], cols[keep]], axis=1)


def from_edges(name: str, n: int, eu, ev, meta=None, keep_lcc: bool = True) -> Graph:
    """Canonical CSR from an undirected edge list (duplicates/self-loops dropped)."""
    lib = _load()
    eu = np.ascontiguousarray(eu, dtype=np.int32)
    ev = np.ascontiguousarray(ev, dtype=np.int32)
    m = int(eu.shape[0])
    offsets = np.zeros(n + 1, dtype=np.int64)
    indices = np.zeros(max(2 * m, 1), dtype=np.int32)
    nnz = lib.gg_build_csr(n, m, _ptr(eu), _ptr(ev), _ptr(offsets), _ptr(indices))
    if nnz < 0:
        raise MemoryError("gg_build_csr failed")
    g = Graph(name, offsets, indices[:nnz].copy(), dict(meta or {}))
    return largest_component(g) if keep_lcc else g


def remove_edges(g: Graph, edges) -> Graph:
    """The same vertex set with the given undirected edges removed (an update
    batch's input; no component step, rows stay ascending)."""
    n = g.n
    e = np.asarray(list(edges), dtype=np.int64).reshape(-1, 2)
    drop = np.concatenate([e[:, 0] * n + e[:, 1], e[:, 1] * n + e[:, 0]])
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(g.offsets))
    keep = ~np.isin(src * n + g.indices.astype(np.int64), drop)
    indices = g.indices[keep].astype(np.int32)
    counts = np.bincount(src[keep], minlength=n)
    offsets = np.zeros(n + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(counts)
    return Graph(g.name + "-del%d" % e.shape[0], offsets, indices, dict(g.meta))


def add_edges(g: Graph, edges) -> Graph:
    """The same vertex set with the given undirected edges added (an update
    batch's input; rows stay ascending)."""
    n = g.n
    e = np.asarray(list(edges), dtype=np.int64).reshape(-1, 2)
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(g.offsets))
    src = np.concatenate([src, e[:, 0], e[:, 1]])
    dst = np.concatenate([g.indices.astype(np.int64), e[:, 1], e[:, 0]])
    order = np.lexsort((dst, src))
    src, dst = src[order], dst[order]
    counts = np.bincount(src, minlength=n)
    offsets = np.zeros(n + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(counts)
    return Graph(g.name + "-add%d" % e.shape[0], offsets, dst.astype(np.int32), dict(g.meta))


def is_connected(g: Graph) -> bool:
    """Whether every vertex is reachable from vertex 0."""
    seen = np.zeros(g.n, dtype=bool)
    seen[0] = True
    stack = [0]
    while stack:
        x = stack.pop()
        for y in g.indices[g.offsets[x]:g.offsets[x + 1]]:
            if not seen[y]:
                seen[y] = True
                stack.append(int(y))
    return bool(seen.all())


def largest_component(g: Graph) -> Graph:
    """Keep the largest connected component, relabelled in original order
    (ties between equally large components go to the one holding the smallest
    vertex)."""
    n = g.n
    if n == 0:
        return g
    off = np.ascontiguousarray(g.offsets, dtype=np.int64)
    idx = np.ascontiguousarray(g.indices, dtype=np.int32)
    off2 = np.zeros(n + 1, dtype=np.int64)
    idx2 = np.empty(max(1, idx.shape[0]), dtype=np.int32)
    n2 = int(_load().gg_lcc(n, _ptr(off), _ptr(idx), _ptr(off2), _ptr(idx2)))
    if n2 < 0:
        raise MemoryError("gg_lcc failed")
    meta = dict(g.meta)
    meta["n_before_lcc"] = n
    if n2 == n:
        g.meta.setdefault("n_before_lcc", n)
        return g
    off2 = off2[: n2 + 1].copy()
    return Graph(g.name, off2, idx2[: int(off2[-1])].copy(), meta)


# ----------------------------------------------------------------- small graphs

def complete(n: int) -> Graph:
    u, v = np.triu_indices(n, 1)
    return from_edges("K%d" % n, n, u, v)


def cycle(n: int) -> Graph:
    u = np.arange(n)
    return from_edges("C%d" % n, n, u, (u + 1) % n)


def path(n: int) -> Graph:
    u = np.arange(n - 1)
    return from_edges("P%d" % n, n, u, u + 1)


def star(n: int) -> Graph:
    """Star K_{1,n-1} with centre 0."""
    v = np.arange(1, n)
    return from_edges("S%d" % n, n, np.zeros_like(v), v)


def grid(rows: int, cols: int) -> Graph:
    """4-neighbour grid, vertex id = cols*i + j."""
    eu, ev = [], []
    for i in range(rows):
        for j in range(cols):
            a = i * cols + j
            if j + 1 < cols:
                eu.append(a); ev.append(a + 1)
            if i + 1 < rows:
                eu.append(a); ev.append(a + cols)
    return from_edges("grid%dx%d" % (rows, cols), rows * cols, eu, ev, {"rows": rows, "cols": cols})


def torus(a: int, b: int) -> Graph:
    """a x b discrete torus (4-regular for a, b >= 3)."""
    eu, ev = [], []
    for i in range(a):
        for j in range(b):
            x = i * b + j
            eu.append(x); ev.append(i * b + (j + 1) % b)
            eu.append(x); ev.append(((i + 1) % a) * b + j)
    return from_edges("torus%dx%d" % (a, b), a * b, eu, ev, {"a": a, "b": b})


def hypercube(d: int) -> Graph:
    n = 1 << d
    u = np.repeat(np.arange(n), d)
    bit = np.tile(1 << np.arange(d), n)
    v = u ^ bit
    keep = u < v
    return from_edges("Q%d" % d, n, u[keep], v[keep], {"d": d})


def petersen() -> Graph:
    outer = [(i, (i + 1) % 5) for i in range(5)]
    spokes = [(i, i + 5) for i in range(5)]
    inner = [(5 + i, 5 + (i + 2) % 5) for i in range(5)]
    e = np.array(outer + spokes + inner)
    return from_edges("petersen", 10, e[:, 0], e[:, 1])


def gnm(n: int, m: int, seed: int) -> Graph:
    """Uniform G(n, m) conditioned on being connected (retries seeds)."""
    for attempt in range(1000):
        rng = np.random.default_rng([seed, attempt])
        u, v = np.triu_indices(n, 1)
        pick = rng.choice(u.shape[0], size=m, replace=False)
        g = from_edges("G(%d,%d)" % (n, m), n, u[pick], v[pick], keep_lcc=False)
        if largest_component(g).n == n:
            g.meta["seed"] = seed
            return g
    raise RuntimeError("no connected G(n,m) found")


def barabasi_albert(n: int, k: int, seed: int) -> Graph:
    """Preferential attachment: each new vertex links to k distinct earlier ones."""
    rng = np.random.default_rng(seed)
    eu, ev, targets = [], [], []
    for v in range(k + 1):
        for u in range(v):
            eu.append(u); ev.append(v); targets += [u, v]
    for v in range(k + 1, n):
        chosen = set()
        while len(chosen) < k:
            chosen.add(targets[rng.integers(len(targets))])
        for u in sorted(chosen):
            eu.append(u); ev.append(v); targets += [u, v]
    return from_edges("BA(%d,%d)" % (n, k), n, eu, ev, {"seed": seed})


# ------------------------------------------------------- large synthetic graphs

def road_like(n_points: int = 1_000_000, full_mean_degree: float = 12.0,
              keep_q: float = 0.2055, seed: int = 0) -> Graph:
    """Thinned random geometric graph, largest component (road-like stand-in).

    n_points uniform points in the unit square, radius r with
    n*pi*r^2 = full_mean_degree, each geometric edge kept with probability
    keep_q; the largest component of the result is kept.  With the defaults
    the component has mean degree close to 2.8.
    """
    lib = _load()
    radius = float(np.sqrt(full_mean_degree / (np.pi * n_points)))
    cap = int(n_points * full_mean_degree * max(keep_q, 0.05) * 0.75) + 1024
    while True:
        eu = np.empty(cap, dtype=np.int32)
        ev = np.empty(cap, dtype=np.int32)
        got = lib.gg_rgg_edges(n_points, radius, keep_q, seed, _ptr(eu), _ptr(ev), cap)
        if got >= 0:
            break
        cap = -got + 16
    meta = {"n_points": n_points, "radius": radius, "keep_q": keep_q, "seed": seed}
    return from_edges("road_like(%d)" % n_points, n_points, eu[:got], ev[:got], meta)


def pareto_weights(n: int, exponent: float, mean: float, cap: float, seed: int) -> np.ndarray:
    """n expected degrees from a power law with density ~ w^-exponent on
    [w_min, cap]; w_min is solved so that the truncated law has the given
    mean.  Returned sorted in non-increasing order."""
    a = exponent

    def tmean(wmin: float) -> float:
        if abs(a - 2.0) < 1e-12:
            num = np.log(cap / wmin)
        else:
            num = (cap ** (2 - a) - wmin ** (2 - a)) / (2 - a)
        den = (cap ** (1 - a) - wmin ** (1 - a)) / (1 - a)
        return float(num / den)

    lo, hi = 1e-6, cap
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if tmean(mid) < mean:
            lo = mid
        else:
            hi = mid
    wmin = 0.5 * (lo + hi)
    rng = np.random.default_rng(seed)
    u = rng.random(n)
    # inverse CDF of the truncated power law
    lo_p, hi_p = wmin ** (1 - a), cap ** (1 - a)
    w = (lo_p + u * (hi_p - lo_p)) ** (1.0 / (1 - a))
    return np.sort(w)[::-1].copy(), wmin


def chung_lu(n: int, exponent: float, mean: float, cap: float, seed: int = 0) -> Graph:
    """Chung-Lu graph with power-law expected degrees, largest component."""
    lib = _load()
    w, wmin = pareto_weights(n, exponent, mean, cap, seed)
    w = np.ascontiguousarray(w, dtype=np.float64)
    est = int(w.sum() / 2 * 1.05) + 1024
    cap_e = est
    while True:
        eu = np.empty(cap_e, dtype=np.int32)
        ev = np.empty(cap_e, dtype=np.int32)
        got = lib.gg_chung_lu_edges(n, _ptr(w), seed + 1, _ptr(eu), _ptr(ev), cap_e)
        if got >= 0:
            break
        cap_e = -got + 16
    meta = {"n_vertices": n, "exponent": exponent, "mean": mean, "cap": cap, "w_min": wmin, "seed": seed}
    return from_edges("chung_lu(%d,%.1f,%g)" % (n, exponent, mean), n, eu[:got], ev[:got], meta)


# ------------------------------------------------------------ named workloads

def workload(name: str, scale: float = 1.0) -> Graph:
    """The named synthetic workloads; ``scale`` < 1 shrinks the vertex count
    (same recipe) for quick tests."""
    if name == "grid32":
        return grid(32, 32)
    if name == "road":
        return road_like(max(1000, int(1_000_000 * scale)), seed=0)
    if name == "social":
        return chung_lu(max(1000, int(1_000_000 * scale)), 2.2, 10.0, 5000.0, seed=0)
    if name == "dense":
        return chung_lu(max(1000, int(3_000_000 * scale)), 2.0, 76.0, 30000.0, seed=0)
    raise KeyError(name)


# ---------------------------------------------------------------- serving mix

def serving_graphs(count: int, lo: int, hi: int, seed: int):
    """`count` resident graphs for the serving mix: types cycle grid, road-like,
    Chung-Lu; vertex counts log-uniform in [lo, hi] (seeded)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        size = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        kind = i % 3
        if kind == 0:
            side = max(4, int(round(math.sqrt(size))))
            g = grid(side, side)
        elif kind == 1:
            g = road_like(max(1000, int(size / 0.8)), seed=int(rng.integers(1 << 30)))
        else:
            g = chung_lu(size, 2.2, 10.0, max(50.0, size ** 0.5 * 5), seed=int(rng.integers(1 << 30)))
        out.append(g)
    return out


def deletion_batch(g: Graph, size: int, rng) -> list:
    """Up to `size` distinct edges drawn with probability proportional to
    d(u) d(v) (the power-law update model), whose removal keeps the graph
    connected: a batch that would disconnect it is halved until it does not."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import connected_components
    deg = np.diff(g.offsets).astype(np.float64)
    src = np.repeat(np.arange(g.n), np.diff(g.offsets))
    mask = src < g.indices
    eu, ev = src[mask], g.indices[mask]
    w = deg[eu] * deg[ev]
    size = min(size, eu.shape[0] - g.n + 1)
    if size <= 0:
        return []
    pick = rng.choice(eu.shape[0], size=size, replace=False, p=w / w.sum())
    batch = [(int(eu[i]), int(ev[i])) for i in pick]
    while batch:
        g2 = remove_edges(g, batch)
        a = csr_matrix((np.ones(g2.indices.shape[0]), g2.indices, g2.offsets), shape=(g2.n, g2.n))
        if connected_components(a, directed=False)[0] == 1:
            return batch
        batch = batch[: len(batch) // 2]
    return batch


def insertion_batch(g: Graph, size: int, rng) -> list:
    """`size` distinct new edges {u, v} (not in the graph, u != v), endpoints
    drawn with probability proportional to their degrees (the power-law update
    model: an edge's probability is proportional to d(u) d(v))."""
    deg = np.diff(g.offsets).astype(np.float64)
    p = deg / deg.sum()
    out, seen = [], set()
    while len(out) < size:
        a, b = (int(x) for x in rng.choice(g.n, size=2, p=p))
        key = (min(a, b), max(a, b))
        if a == b or key in seen or b in g.indices[g.offsets[a]:g.offsets[a + 1]]:
            continue
        seen.add(key)
        out.append(key)
    return out
