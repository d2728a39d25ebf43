"""Pins of the weighted-graph oracle (Section "Generalizations", extension to weighted
graphs) against mathematics that does not come from the oracle itself: the weighted
matrix-tree theorem, the weight-proportional spanning-tree distribution, the weighted
Kirchhoff theorem with Ohm's law (mean fixed-point tree flow = effective resistance of the
weighted Laplacian), tree graphs, the unit-weight reduction, and dense pseudoinverses."""
import math

import numpy as np
import pytest
from scipy import stats

import oracle
from paper_2006_13679_amd import graphgen as gg
from tests import brute

TINY = {
    "K4": (lambda: gg.complete(4), 0),
    "C5": (lambda: gg.cycle(5), 0),
    "grid3": (lambda: gg.grid2d(3), 4),
    "K23": (lambda: gg.complete_bipartite(2, 3), 0),
    "pendant_cycle": (lambda: gg.from_edges(6, [(0, 1), (1, 2), (2, 3), (3, 0), (3, 4), (4, 5), (1, 3)]), 1),
}


def _wtiny(name, kind="uniform", seed=3):
    make, u = TINY[name]
    g = make()
    return g, u, gg.edge_weights(g, seed, kind, 0.5, 4.0)


def test_weight_generator_symmetric_and_validation():
    g = gg.rmat(8, 8, 2)
    for kind in ("uniform", "lognormal", "pow2", "ones"):
        w = gg.edge_weights(g, 1, kind, 0.5, 4.0)
        assert (w > 0).all()
        assert oracle.validate_weights(g.row_ptr, g.col, w) == oracle.OK
        L = brute.laplacian_weighted(g, w)
        np.testing.assert_allclose(L, L.T)
        np.testing.assert_allclose(L.sum(axis=1), 0.0, atol=1e-12)
    w = gg.edge_weights(g, 1)
    bad = w.copy()
    bad[3] *= 1.5  # one direction only
    assert oracle.validate_weights(g.row_ptr, g.col, bad) == oracle.EGRAPH
    for val in (0.0, -1.0, np.nan, np.inf):
        bad = w.copy()
        e = 5
        bad[e] = val
        assert oracle.validate_weights(g.row_ptr, g.col, bad) == oracle.EGRAPH


def test_weighted_matrix_tree_theorem():
    """Sum over spanning trees of the product of conductances = any cofactor of L_w."""
    for name in TINY:
        g, u, w = _wtiny(name)
        wm = brute.weight_map(g, w)
        total = sum(brute.tree_weight(p, wm) for p in brute.spanning_trees(g, u))
        L = brute.laplacian_weighted(g, w)
        assert total == pytest.approx(np.linalg.det(L[1:, 1:]), rel=1e-10)


def test_unit_weights_reduce_to_unweighted():
    """All conductances 1: the same trees and steps as the unweighted walk, rho(v) = dist(u, v),
    rho_max = ecc(u), the same tau, and fixed-point sums = 2^k x the integer counts."""
    g = gg.random_connected(60, 0.08, 4)
    u = gg.max_degree_pivot(g)
    w = gg.edge_weights(g, 0, "ones")
    dist, parB, ecc = oracle.bfs(g.row_ptr, g.col, u)
    wB, rho, rmax = oracle.bpath_resistance(g.row_ptr, g.col, w, u)
    assert rmax == ecc and (rho == dist).all()
    assert oracle.tau_weighted(g.n, g.m, rmax, 0.3) == oracle.tau(g.n, g.m, ecc, 0.3)
    k = oracle.fixed_shift(40, rmax)
    P1, S1, C1 = oracle.trees(g.row_ptr, g.col, u, 9, 3, 40)
    P2, S2, A2 = oracle.trees_weighted(g.row_ptr, g.col, w, u, 9, 3, 40, k)
    assert (P1 == P2).all() and (S1 == S2).all()
    assert (A2 == C1 * (1 << k)).all()


@pytest.mark.parametrize("name", ["K4", "grid3", "K23"])
def test_weighted_wilson_distribution_chisquare(name):
    """Wilson's walk with conductance-proportional steps draws each spanning tree with
    probability w(T) / sum of w over all trees."""
    g, u, w = _wtiny(name, "uniform", 5)
    wm = brute.weight_map(g, w)
    trees = brute.spanning_trees(g, u)
    index = {brute.tree_key(p): i for i, p in enumerate(trees)}
    prob = np.array([brute.tree_weight(p, wm) for p in trees])
    prob /= prob.sum()
    samples = max(60 * len(trees), 6000)
    parents, _, _ = oracle.trees_weighted(g.row_ptr, g.col, w, u, 21, 0, samples, 30, want_acc=False)
    counts = np.zeros(len(trees))
    for p in parents:
        counts[index[brute.tree_key(p)]] += 1
    _, pval = stats.chisquare(counts, prob * samples)
    assert pval > 1e-4, (name, pval)


def test_weighted_edge_marginals():
    """P(e in T) = w(e) r_w(e) for trees drawn with probability proportional to their weight
    (the weighted form of the spanning-edge identity)."""
    g = gg.from_edges(8, [(0, 1), (1, 2), (2, 3), (3, 0), (0, 4), (4, 5), (5, 6), (6, 7), (7, 4), (2, 6), (1, 5)])
    w = gg.edge_weights(g, 4, "uniform", 0.5, 4.0)
    wm = brute.weight_map(g, w)
    T = 6000
    parents, _, _ = oracle.trees_weighted(g.row_ptr, g.col, w, 0, 3, 0, T, 30, want_acc=False)
    P = brute.pinv_weighted(g, w)
    dP = np.diag(P)
    for (a, b), c in wm.items():
        pe = c * (dP[a] + dP[b] - 2 * P[a, b])
        freq = np.mean((parents[:, a] == b) | (parents[:, b] == a))
        assert abs(freq - pe) < 5 * math.sqrt(pe * (1 - pe) / T) + 1e-9, (a, b, freq, pe)


@pytest.mark.parametrize("name", list(TINY))
def test_weighted_tree_flow_enumeration_equals_resistance(name):
    """Weighted Kirchhoff theorem + Ohm's law: the weight-averaged fixed-point tree flow,
    divided by 2^k, is the effective resistance of the weighted Laplacian, for every pivot."""
    g, u0, w = _wtiny(name)
    wm = brute.weight_map(g, w)
    P = brute.pinv_weighted(g, w)
    d = np.diag(P)
    k = 40
    for u in range(g.n):
        _, parB, _ = oracle.bfs(g.row_ptr, g.col, u)
        wB, rho, _ = oracle.bpath_resistance(g.row_ptr, g.col, w, u)
        F = oracle.fixed_weights(u, wB, k)
        num = np.zeros(g.n)
        den = 0.0
        for par in brute.spanning_trees(g, u):
            wt = brute.tree_weight(par, wm)
            num += wt * oracle.tree_flow_weighted(u, parB, par, F).astype(np.float64)
            den += wt
        r = d[u] - 2 * P[u, :] + d
        np.testing.assert_allclose(num / den / 2.0 ** k, r, atol=1e-9)


def test_weighted_tree_graph_flow_is_path_resistance():
    """On a tree graph every spanning tree is the graph, so c_T(v) / 2^k = rho(v) = r(u, v)."""
    for seed in range(3):
        g = gg.random_tree(25, seed)
        w = gg.edge_weights(g, seed, "lognormal")
        u = seed
        _, parB, _ = oracle.bfs(g.row_ptr, g.col, u)
        wB, rho, rmax = oracle.bpath_resistance(g.row_ptr, g.col, w, u)
        k = oracle.fixed_shift(1, rmax)
        F = oracle.fixed_weights(u, wB, k)
        par, _ = oracle.wilson_weighted(g.row_ptr, g.col, w, u, 4, 0)
        c = oracle.tree_flow_weighted(u, parB, par, F)
        np.testing.assert_allclose(c / 2.0 ** k, rho, rtol=1e-12)
        P = brute.pinv_weighted(g, w)
        d = np.diag(P)
        np.testing.assert_allclose(rho, d[u] - 2 * P[u, :] + d, atol=1e-9)


def test_bpath_resistance_and_fixed_point_range():
    """rho(v) = sum of 1/w along the BFS parents; the shift keeps tau * 2^k * rho_max <= 2^62,
    so sums of tau trees fit int64."""
    g = gg.rmat(9, 8, 3)
    u = gg.max_degree_pivot(g)
    w = gg.edge_weights(g, 7, "lognormal")
    dist, parB, _ = oracle.bfs(g.row_ptr, g.col, u)
    wB, rho, rmax = oracle.bpath_resistance(g.row_ptr, g.col, w, u)
    wm = brute.weight_map(g, w)
    for v in [1, 5, 77, g.n - 1]:
        r, b = 0.0, v
        while b != u:
            r += 1.0 / wm[(min(b, parB[b]), max(b, parB[b]))]
            b = parB[b]
        assert rho[v] == pytest.approx(r, rel=1e-12)
    assert rmax == rho.max()
    for tau_ in (1, 1000, 123457):
        k = oracle.fixed_shift(tau_, rmax)
        assert tau_ * rmax * 2.0 ** k <= 2.0 ** 62 < tau_ * rmax * 2.0 ** (k + 1)
        F = oracle.fixed_weights(u, wB, k)
        worst = max(sum(int(F[b]) for b in _path(parB, v, u)) for v in range(g.n))
        assert tau_ * worst < 2 ** 63


def _path(parB, v, u):
    out = []
    while v != u:
        out.append(v)
        v = parB[v]
    return out


def test_tau_weighted_scales_with_path_resistance():
    n, m = 1000, 5000
    t1 = oracle.tau_weighted(n, m, 4.0, 0.3)
    assert t1 == oracle.tau(n, m, 4, 0.3)
    assert oracle.tau_weighted(n, m, 2.0, 0.3) == t1 // 4
    q = math.ceil(math.log(2 * m * n) / (2 * 0.49 * 0.09))
    assert oracle.tau_weighted(n, m, 2.5, 0.3) == math.ceil(6.25 * q)


@pytest.mark.parametrize("u", [0, 13])
def test_solve_weighted_matches_pinv_column(u):
    g = gg.grid2d(7)
    w = gg.edge_weights(g, 2, "lognormal")
    x, it, rr = oracle.solve_weighted(g.row_ptr, g.col, w, u, tol=1e-13)
    assert it > 0 and rr < 1e-11
    np.testing.assert_allclose(x, brute.pinv_weighted(g, w)[:, u], atol=1e-10)


def test_combine_weighted_identity():
    """Exact resistances in fixed point through Eq. diag-comp give the pseudoinverse diagonal."""
    g, u, w = _wtiny("pendant_cycle")
    P = brute.pinv_weighted(g, w)
    d = np.diag(P)
    r = d[u] - 2 * P[u, :] + d
    tau_, k = 7, 40
    acc = np.round(r * tau_ * 2.0 ** k).astype(np.int64)
    diag = oracle.combine_weighted(u, tau_, k, acc, P[:, u])
    np.testing.assert_allclose(diag, d, atol=1e-11)


@pytest.mark.parametrize("name", ["K4", "grid3", "K23", "pendant_cycle"])
def test_weighted_end_to_end_within_eps(name):
    g, u, w = _wtiny(name, "uniform", 11)
    out = oracle.diag_lpinv_weighted(g.row_ptr, g.col, w, u, 0.3, 5)
    assert out["status"] == oracle.OK
    d = np.diag(brute.pinv_weighted(g, w))
    assert np.max(np.abs(out["diag"] - d)) <= 0.3
    wB, rho, rmax = oracle.bpath_resistance(g.row_ptr, g.col, w, u)
    assert out["rho_max"] == rmax
    assert out["tau"] == oracle.tau_weighted(g.n, g.m, rmax, 0.3)
    assert out["shift"] == oracle.fixed_shift(out["tau"], rmax)
