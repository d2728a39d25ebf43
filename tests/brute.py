"""Brute-force references for tiny graphs (test-only): spanning-tree enumeration,
matrix-tree counts and dense pseudoinverses.  Independent of both the oracle and the GPU
library: plain numpy on explicit edge lists."""
from __future__ import annotations

import itertools

import numpy as np


def edges_of(g):
    """Undirected edge list (a < b) from a CSR graph."""
    rp, col = g.row_ptr, g.col
    out = []
    for v in range(len(rp) - 1):
        for e in range(rp[v], rp[v + 1]):
            w = int(col[e])
            if v < w:
                out.append((v, w))
    return out


def laplacian(g) -> np.ndarray:
    n = g.n
    L = np.zeros((n, n))
    for a, b in edges_of(g):
        L[a, b] -= 1
        L[b, a] -= 1
        L[a, a] += 1
        L[b, b] += 1
    return L


def pinv(g) -> np.ndarray:
    return np.linalg.pinv(laplacian(g))


def matrix_tree_count(g) -> int:
    """Number of spanning trees = any cofactor of L (matrix-tree theorem)."""
    L = laplacian(g)
    return int(round(np.linalg.det(L[1:, 1:])))


def _connected_subset(n, sub):
    parent = list(range(n))

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    for a, b in sub:
        ra, rb = find(a), find(b)
        if ra == rb:
            return False
        parent[ra] = rb
    return True


def rooted_parents(n, tree_edges, root) -> np.ndarray:
    adj = [[] for _ in range(n)]
    for a, b in tree_edges:
        adj[a].append(b)
        adj[b].append(a)
    par = np.full(n, -2, dtype=np.int32)
    par[root] = -1
    stack = [root]
    while stack:
        x = stack.pop()
        for y in adj[x]:
            if par[y] == -2:
                par[y] = x
                stack.append(y)
    assert (par != -2).all()
    return par


def spanning_trees(g, root):
    """All spanning trees as parent arrays rooted at `root` (n <= ~10)."""
    n = g.n
    E = edges_of(g)
    out = []
    for sub in itertools.combinations(E, n - 1):
        if _connected_subset(n, sub):
            out.append(rooted_parents(n, sub, root))
    return out


def tree_key(par) -> tuple:
    return tuple(int(x) for x in par)


def effective_resistance_from(g, u) -> np.ndarray:
    P = pinv(g)
    d = np.diag(P)
    return d[u] - 2 * P[u, :] + d


def check_tree(g, par, root):
    """Spanning-tree invariants: parent[root] = -1, n-1 edges all in E, every vertex
    reaches root without repeating a vertex (acyclic, spanning)."""
    n = g.n
    assert par[root] == -1
    E = set(edges_of(g))
    for v in range(n):
        if v == root:
            continue
        p = int(par[v])
        assert 0 <= p < n, (v, p)
        assert (min(v, p), max(v, p)) in E, (v, p)
    for v in range(n):
        seen = 0
        x = v
        while x != root:
            x = int(par[x])
            seen += 1
            assert seen <= n, "cycle"


# ---------------------------------------------------------------------------------------
# weighted graphs: conductance per undirected edge, from the CSR weight array
# ---------------------------------------------------------------------------------------
def weight_map(g, w) -> dict:
    rp, col = g.row_ptr, g.col
    out = {}
    for v in range(len(rp) - 1):
        for e in range(rp[v], rp[v + 1]):
            b = int(col[e])
            if v < b:
                out[(v, b)] = float(w[e])
    return out


def laplacian_weighted(g, w) -> np.ndarray:
    n = g.n
    L = np.zeros((n, n))
    for (a, b), c in weight_map(g, w).items():
        L[a, b] -= c
        L[b, a] -= c
        L[a, a] += c
        L[b, b] += c
    return L


def pinv_weighted(g, w) -> np.ndarray:
    return np.linalg.pinv(laplacian_weighted(g, w))


def tree_weight(par, wmap) -> float:
    """Product of the conductances of a parent array's edges."""
    out = 1.0
    for v, p in enumerate(par):
        if p >= 0:
            out *= wmap[(min(v, int(p)), max(v, int(p)))]
    return out
