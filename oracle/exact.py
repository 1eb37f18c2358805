"""Exact quantities the sampled estimator is pinned against (FP64, numpy).

TEST INFRASTRUCTURE ONLY (see the package docstring).

  kemeny_exact   -- Eq. (1): kappa = Tr(L_norm^+) = sum_{i>=2} 1/sigma_i, from a
                    dense eigensolve of D^-1/2 A D^-1/2 (same spectrum as
                    D^-1 A): kappa = sum over the non-unit eigenvalues of
                    1 / (1 - lambda).
  phi_exact      -- the expected number of Wilson draws, Tr((I - P_r)^-1)
                    (section 2.2 / Theorem 3.5), by a dense solve.
  closed forms   -- Kemeny constants of complete graphs, cycles, paths,
                    stars, tori and hypercubes from their known spectra.
  spanning_trees -- every spanning tree of a tiny graph, as parent arrays
                    rooted at r (brute force over (n-1)-edge subsets).
  tree_count     -- matrix-tree theorem: det of the reduced Laplacian.
"""
from __future__ import annotations

import itertools
from fractions import Fraction
from math import comb

import numpy as np


def _dense(offsets, indices):
    n = len(offsets) - 1
    a = np.zeros((n, n))
    deg = np.diff(offsets)
    rows = np.repeat(np.arange(n), deg)
    a[rows, indices] = 1.0
    return a, deg.astype(np.float64)


def kemeny_exact(offsets, indices) -> float:
    a, d = _dense(offsets, indices)
    s = 1.0 / np.sqrt(d)
    sym = a * s[:, None] * s[None, :]
    lam = np.linalg.eigvalsh(sym)
    # drop the single eigenvalue 1 (connected graph): it is the largest
    lam = np.sort(lam)[:-1]
    return float(np.sum(1.0 / (1.0 - lam)))


def phi_exact(offsets, indices, root: int) -> float:
    """Tr((I - P_r)^-1) with P = D^-1 A and row/column r removed."""
    a, d = _dense(offsets, indices)
    p = a / d[:, None]
    keep = np.array([i for i in range(len(d)) if i != root])
    m = np.eye(len(keep)) - p[np.ix_(keep, keep)]
    return float(np.trace(np.linalg.inv(m)))


def tree_count(offsets, indices) -> int:
    a, d = _dense(offsets, indices)
    lap = np.diag(d) - a
    val = np.linalg.det(lap[1:, 1:])
    return int(round(val))


# ------------------------------------------------------------- closed forms

def kemeny_complete(n: int) -> Fraction:
    return Fraction((n - 1) ** 2, n)


def kemeny_cycle(n: int) -> Fraction:
    return Fraction(n * n - 1, 6)


def kemeny_path(n: int) -> Fraction:
    return Fraction((n - 1) ** 2, 3) + Fraction(1, 6)


def kemeny_star(n: int) -> Fraction:
    """Star K_{1,n-1}: spectrum of P is {1, -1, 0 (n-2 times)}."""
    return Fraction(n) - Fraction(3, 2)


def kemeny_torus(a: int, b: int) -> float:
    """a x b torus: P has eigenvalues (cos 2pi j/a + cos 2pi k/b)/2."""
    total = 0.0
    for j in range(a):
        for k in range(b):
            if j == 0 and k == 0:
                continue
            lam = (np.cos(2 * np.pi * j / a) + np.cos(2 * np.pi * k / b)) / 2.0
            total += 1.0 / (1.0 - lam)
    return total


def kemeny_hypercube(d: int) -> Fraction:
    """Q_d: eigenvalues 1 - 2k/d with multiplicity C(d, k)."""
    return sum((Fraction(comb(d, k) * d, 2 * k) for k in range(1, d + 1)), Fraction(0))


# ------------------------------------------------------ tree enumeration

def spanning_trees(offsets, indices, root: int):
    """All spanning trees as parent arrays rooted at `root` (brute force)."""
    n = len(offsets) - 1
    edges = []
    for u in range(n):
        for e in range(offsets[u], offsets[u + 1]):
            v = int(indices[e])
            if u < v:
                edges.append((u, v))
    out = []
    for sub in itertools.combinations(edges, n - 1):
        adj = [[] for _ in range(n)]
        for u, v in sub:
            adj[u].append(v)
            adj[v].append(u)
        parent = [-2] * n
        parent[root] = -1
        stack = [root]
        seen = 1
        while stack:
            x = stack.pop()
            for y in adj[x]:
                if parent[y] == -2:
                    parent[y] = x
                    seen += 1
                    stack.append(y)
        if seen == n:
            out.append(np.array(parent, dtype=np.int32))
    return out
