"""Pins of the CPU oracle against facts fixed by the paper and by mathematics, not by the
oracle itself: published Philox known-answer vectors, an independent numpy Philox,
exhaustive spanning-tree enumeration (Kirchhoff's theorem, matrix-tree counts, uniformity),
dense pseudoinverses, closed forms and worked examples of the sample-size formula."""
import math
import os

import numpy as np
import pytest
from scipy import stats
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import shortest_path

import oracle
from paper_2006_13679_amd import graphgen as gg
from tests import brute

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# -------------------------------------------------------------------------------------
# Philox4x32-10
# -------------------------------------------------------------------------------------
def _kat_rows():
    rows = []
    with open(os.path.join(GOLD, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            w = [int(x, 16) for x in line.split()]
            rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


def np_philox(ctr, key):
    """Independent vectorised Philox4x32-10 in numpy uint64 arithmetic (test reference).
    ctr: uint64 array (4, N); key: (2, N)."""
    M0, M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
    W0, W1 = np.uint64(0x9E3779B9), np.uint64(0xBB67AE85)
    mask = np.uint64(0xFFFFFFFF)
    c = [np.asarray(x, dtype=np.uint64) & mask for x in ctr]
    k0 = np.asarray(key[0], dtype=np.uint64) & mask
    k1 = np.asarray(key[1], dtype=np.uint64) & mask
    for r in range(10):
        if r:
            k0 = (k0 + W0) & mask
            k1 = (k1 + W1) & mask
        p0 = M0 * c[0]
        p1 = M1 * c[2]
        c = [((p1 >> np.uint64(32)) ^ c[1] ^ k0) & mask, p1 & mask,
             ((p0 >> np.uint64(32)) ^ c[3] ^ k1) & mask, p0 & mask]
    return np.stack(c).astype(np.uint32)


def test_philox_known_answers():
    for ctr, key, want in _kat_rows():
        assert list(oracle.philox4x32_10(ctr, key)) == want
        got = np_philox([[x] for x in ctr], [[x] for x in key])[:, 0]
        assert list(got) == want


def test_philox_matches_numpy_on_counter_grid():
    rng = np.random.default_rng(7)
    ctr = rng.integers(0, 2**32, size=(4, 200), dtype=np.uint64)
    key = rng.integers(0, 2**32, size=(2, 200), dtype=np.uint64)
    ref = np_philox(ctr, key)
    for i in range(200):
        got = oracle.philox4x32_10(ctr[:, i], key[:, i])
        assert (got == ref[:, i]).all()


def test_walk_word_keying():
    """word k of the walk from s in tree t = Philox((k/4, s, t lo, t hi); (seed lo, seed hi))[k%4]."""
    seed = 0x123456789ABCDEF0
    for t in (0, 5, 2**33 + 7):
        for s in (0, 17, 2**31 - 1):
            for k in (0, 1, 2, 3, 4, 9, 2**20 + 3):
                ctr = [[k // 4], [s], [t & 0xFFFFFFFF], [t >> 32]]
                key = [[seed & 0xFFFFFFFF], [seed >> 32]]
                want = int(np_philox(ctr, key)[k % 4, 0])
                assert oracle.walk_word(seed, t, s, k) == want


def test_philox_words_uniform():
    words = np.array([oracle.walk_word(1, t, 3, k) for t in range(40) for k in range(256)], dtype=np.uint64)
    counts = np.bincount((words >> np.uint64(28)).astype(np.int64), minlength=16)
    _, p = stats.chisquare(counts)
    assert p > 1e-4
    bits = np.array([(words >> np.uint64(b)) & np.uint64(1) for b in range(32)]).mean(axis=1)
    assert np.all(np.abs(bits - 0.5) < 0.05)


# -------------------------------------------------------------------------------------
# graph validation and BFS
# -------------------------------------------------------------------------------------
def test_validate_accepts_and_rejects():
    g = gg.grid2d(4)
    assert oracle.validate(g.row_ptr, g.col) == oracle.OK
    rp, col = g.row_ptr.copy(), g.col.copy()
    # self-loop: replace the first neighbour of vertex 0 by 0
    c2 = col.copy(); c2[0] = 0
    assert oracle.validate(rp, c2) == oracle.EGRAPH
    # unsorted row
    c3 = col.copy(); c3[rp[5]], c3[rp[5] + 1] = c3[rp[5] + 1], c3[rp[5]]
    assert oracle.validate(rp, c3) == oracle.EGRAPH
    # asymmetric: drop one direction of an edge by redirecting it
    c4 = col.copy(); c4[rp[0] + 1] = 15
    assert oracle.validate(rp, c4) == oracle.EGRAPH
    # disconnected: two triangles
    d = gg.from_edges(6, [(0, 1), (1, 2), (0, 2), (3, 4), (4, 5), (3, 5)])
    # canonical_csr keeps the largest component only; build raw CSR by hand instead
    rp6 = np.array([0, 2, 4, 6, 8, 10, 12], dtype=np.int64)
    col6 = np.array([1, 2, 0, 2, 0, 1, 4, 5, 3, 5, 3, 4], dtype=np.int32)
    assert d.n == 3
    assert oracle.validate(rp6, col6) == oracle.EGRAPH


def test_bfs_min_id_parent_hand_built():
    # u=0; vertices 3 and 4 are both at distance 2 with two predecessors each
    #   0-1, 0-2, 1-3, 2-3, 1-4, 2-4, 3-5, 4-5
    g = gg.from_edges(6, [(0, 1), (0, 2), (1, 3), (2, 3), (1, 4), (2, 4), (3, 5), (4, 5)])
    dist, parB, ecc = oracle.bfs(g.row_ptr, g.col, 0)
    assert list(dist) == [0, 1, 1, 2, 2, 3]
    assert list(parB) == [-1, 0, 0, 1, 1, 3]
    assert ecc == 3
    dist, parB, ecc = oracle.bfs(g.row_ptr, g.col, 5)
    assert list(dist) == [3, 2, 2, 1, 1, 0]
    assert list(parB) == [1, 3, 3, 5, 5, -1]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_bfs_against_scipy(seed):
    g = gg.random_connected(60, 0.08, seed)
    u = gg.max_degree_pivot(g)
    dist, parB, ecc = oracle.bfs(g.row_ptr, g.col, u)
    A = csr_matrix((np.ones(len(g.col)), g.col, g.row_ptr), shape=(g.n, g.n))
    ref = shortest_path(A, unweighted=True, indices=u).astype(np.int64)
    assert (dist == ref).all() and ecc == ref.max()
    for v in range(g.n):
        if v == u:
            continue
        nb = g.col[g.row_ptr[v]:g.row_ptr[v + 1]]
        cand = [int(w) for w in nb if ref[w] == ref[v] - 1]
        assert parB[v] == min(cand)


# -------------------------------------------------------------------------------------
# tau / eta
# -------------------------------------------------------------------------------------
def test_max_degree_pivot_rule():
    """pivot = -1: the vertex of largest degree, the smallest ID among equal degrees."""
    assert oracle.max_degree_pivot(gg.star(9).row_ptr) == 0
    assert oracle.max_degree_pivot(gg.path(5).row_ptr) == 1          # 1, 2, 3 all have degree 2
    assert oracle.max_degree_pivot(gg.complete(6).row_ptr) == 0
    assert oracle.max_degree_pivot(gg.grid2d(4).row_ptr) == 5        # interior vertices 5, 6, 9, 10
    assert oracle.max_degree_pivot(gg.complete_bipartite(2, 3).row_ptr) == 0  # the side of 2 has degree 3
    # a hand-built graph whose largest degree first appears at the last vertex
    g = gg.from_edges(6, [(0, 1), (1, 2), (2, 3), (3, 4), (5, 0), (5, 1), (5, 2), (5, 3)])
    assert oracle.max_degree_pivot(g.row_ptr) == 5


def test_tau_worked_examples():
    with open(os.path.join(GOLD, "tau_worked_examples.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            n, m, ecc, eps, want = line.split()
            assert oracle.tau(int(n), int(m), int(ecc), float(eps)) == int(want)


def test_eta_worked_examples():
    """eta against hand-worked values (tests/golden/eta_worked_examples.txt): a base-2 log, a
    missing factor 3 or a diameter bound of ecc instead of 2 ecc each move every row."""
    rows = 0
    with open(os.path.join(GOLD, "eta_worked_examples.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            n, m, ecc, eps, kappa, want = line.split()
            got = oracle.eta(int(n), int(m), int(ecc), float(eps), float(kappa))
            assert got == pytest.approx(float(want), rel=1e-14), (n, m, ecc)
            rows += 1
    assert rows == 6
    # kappa <= 0 selects 0.3
    assert oracle.eta(1024, 1984, 32, 0.3, 0.0) == oracle.eta(1024, 1984, 32, 0.3, 0.3)


@pytest.mark.parametrize("name", ["K4", "C5", "grid3", "K23", "pendant_cycle"])
def test_eta_bounds_the_solve_error(name):
    """What eta is for (Appendix proof of the running-time theorem): a solution with relative
    L-norm error eta errs by at most kappa eps / 3 in every entry.  The largest |e_i| over
    e perpendicular to 1 with ||e||_L = c is c sqrt(L+_ii), so the worst case over all such
    errors is eta ||x||_L sqrt(max_i L+_ii), checked for every pivot."""
    g = TINY[name]()
    P = brute.pinv(g)
    for u in range(g.n):
        _, _, ecc = oracle.bfs(g.row_ptr, g.col, u)
        for eps, kappa in ((0.3, 0.3), (0.9, 0.5), (0.05, 0.1)):
            eta = oracle.eta(g.n, g.m, ecc, eps, kappa)
            x = P[:, u]
            xl = math.sqrt(x @ brute.laplacian(g) @ x)
            worst = eta * xl * math.sqrt(np.diag(P).max())
            assert worst <= kappa * eps / 3


# -------------------------------------------------------------------------------------
# Wilson sampler: uniformity, invariants, expected steps, edge marginals
# -------------------------------------------------------------------------------------
TINY = {
    "K4": lambda: gg.complete(4),
    "C5": lambda: gg.cycle(5),
    "grid3": lambda: gg.grid2d(3),
    "K23": lambda: gg.complete_bipartite(2, 3),
    "pendant_cycle": lambda: gg.from_edges(6, [(0, 1), (1, 2), (2, 3), (3, 0), (3, 4), (4, 5), (1, 3)]),
}


def test_matrix_tree_counts():
    assert len(brute.spanning_trees(gg.complete(5), 0)) == 5 ** 3 == brute.matrix_tree_count(gg.complete(5))
    assert len(brute.spanning_trees(gg.grid2d(3), 4)) == 192 == brute.matrix_tree_count(gg.grid2d(3))
    assert len(brute.spanning_trees(gg.cycle(7), 0)) == 7
    assert len(brute.spanning_trees(gg.complete_bipartite(2, 3), 0)) == 2 ** 2 * 3 ** 1


@pytest.mark.parametrize("name", ["K4", "C5", "grid3", "K23"])
def test_wilson_uniform_chisquare(name):
    g = TINY[name]()
    u = 0 if name != "grid3" else 4
    all_trees = brute.spanning_trees(g, u)
    N = len(all_trees)
    assert N == brute.matrix_tree_count(g)
    index = {brute.tree_key(p): i for i, p in enumerate(all_trees)}
    samples = max(100 * N, 4000)
    parents, steps, _ = oracle.trees(g.row_ptr, g.col, u, 11, 0, samples, want_counts=False)
    counts = np.zeros(N, dtype=np.int64)
    for p in parents:
        counts[index[brute.tree_key(p)]] += 1
    assert counts.sum() == samples
    _, pval = stats.chisquare(counts)
    assert pval > 1e-4, (name, pval)


@pytest.mark.parametrize("seed", [0, 1])
def test_wilson_tree_invariants(seed):
    g = gg.random_connected(80, 0.06, seed)
    u = gg.max_degree_pivot(g)
    parents, steps, _ = oracle.trees(g.row_ptr, g.col, u, seed, 0, 20, want_counts=False)
    for p in parents:
        brute.check_tree(g, p, u)
    assert (steps >= g.n - 1).all()


def test_wilson_edge_marginals_and_expected_steps():
    """P(e in UST) = r(e) for every edge (Section "Problem Description and Notation"), and
    the expected number of walk steps is sum_{v != u} deg(v) r(u, v) (Appendix lemma on
    Wilson's running time)."""
    g = gg.from_edges(8, [(0, 1), (1, 2), (2, 3), (3, 0), (0, 4), (4, 5), (5, 6), (6, 7), (7, 4), (2, 6), (1, 5)])
    u = 0
    T = 6000
    parents, steps, _ = oracle.trees(g.row_ptr, g.col, u, 3, 0, T, want_counts=False)
    P = brute.pinv(g)
    dP = np.diag(P)
    for a, b in brute.edges_of(g):
        r = dP[a] + dP[b] - 2 * P[a, b]
        freq = np.mean((parents[:, a] == b) | (parents[:, b] == a))
        sd = math.sqrt(r * (1 - r) / T)
        assert abs(freq - r) < 5 * sd + 1e-9, (a, b, freq, r)
    ruv = dP[u] - 2 * P[u, :] + dP
    deg = g.degrees
    expect = float(sum(deg[v] * ruv[v] for v in range(g.n) if v != u))
    se = steps.std() / math.sqrt(T)
    assert abs(steps.mean() - expect) < 5 * se, (steps.mean(), expect)


# -------------------------------------------------------------------------------------
# Wilson's algorithm per biconnected component (engineering appendix)
# -------------------------------------------------------------------------------------
CUT = {
    "pendant_cycle": lambda: TINY["pendant_cycle"](),
    "bowtie": lambda: gg.from_edges(5, [(0, 1), (1, 2), (2, 0), (2, 3), (3, 4), (4, 2)]),
    "two_squares_bridge": lambda: gg.from_edges(8, [(0, 1), (1, 2), (2, 3), (3, 0), (3, 4), (4, 5), (5, 6),
                                                    (6, 7), (7, 4)]),
    "K4_tail": lambda: gg.from_edges(7, [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3), (3, 4), (4, 5), (4, 6)]),
}


def _blocks_by_cycles(g):
    """Blocks by their definition: two edges share a block iff a simple cycle contains both
    (enumerated by depth-first search on the tiny graph); an edge on no cycle is alone."""
    edges = [tuple(e) for e in brute.edges_of(g)]
    idx = {e: i for i, e in enumerate(edges)}
    par = list(range(len(edges)))

    def find(x):
        while par[x] != x:
            x = par[x]
        return x

    adj = {v: [int(w) for w in g.col[g.row_ptr[v]:g.row_ptr[v + 1]]] for v in range(g.n)}

    def key(a, b):
        return idx[(min(a, b), max(a, b))]

    def dfs(start, v, path, seen):
        for w in adj[v]:
            if w == start and len(path) >= 3:
                cyc = [key(path[i], path[i + 1]) for i in range(len(path) - 1)] + [key(v, start)]
                for e in cyc[1:]:
                    par[find(e)] = find(cyc[0])
            elif w not in seen and w > start:
                seen.add(w)
                dfs(start, w, path + [w], seen)
                seen.discard(w)

    for s0 in range(g.n):
        dfs(s0, s0, [s0], {s0})
    return [find(i) for i in range(len(edges))], edges


@pytest.mark.parametrize("name", list(CUT) + ["K4", "C5", "grid3", "tree", "gnp"])
def test_blocks_match_cycle_definition(name):
    g = CUT[name]() if name in CUT else (TINY[name]() if name in TINY else
                                         gg.random_tree(9, 4) if name == "tree" else gg.random_connected(9, 0.3, 2))
    eb, nb = oracle.blocks(g.row_ptr, g.col)
    lab, edges = _blocks_by_cycles(g)
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    pos = {(int(a), int(b)): i for i, (a, b) in enumerate(zip(rows, g.col))}
    got = [int(eb[pos[(a, b)]]) for a, b in edges]
    assert all(eb[pos[(a, b)]] == eb[pos[(b, a)]] for a, b in edges)  # both entries of an edge
    # the same partition of the edges
    pairs_got = {(i, j) for i in range(len(edges)) for j in range(len(edges)) if got[i] == got[j]}
    pairs_want = {(i, j) for i in range(len(edges)) for j in range(len(edges)) if lab[i] == lab[j]}
    assert pairs_got == pairs_want
    assert nb == len(set(lab))


@pytest.mark.parametrize("name", list(CUT) + ["K4", "grid3"])
def test_wilson_blocks_uniform_chisquare(name):
    """Per-block trees joined at the cut vertices are uniform over the spanning trees of G."""
    g = CUT[name]() if name in CUT else TINY[name]()
    for u in (0, g.n - 1):
        all_trees = brute.spanning_trees(g, u)
        N = len(all_trees)
        assert N == brute.matrix_tree_count(g)
        index = {brute.tree_key(p): i for i, p in enumerate(all_trees)}
        samples = max(100 * N, 3000)
        parents, steps, _ = oracle.trees_blocks(g.row_ptr, g.col, u, 13, 0, samples, want_counts=False)
        counts = np.zeros(N, dtype=np.int64)
        for p in parents:
            counts[index[brute.tree_key(p)]] += 1
        _, pval = stats.chisquare(counts)
        assert pval > 1e-4, (name, u, pval)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_wilson_blocks_tree_invariants_and_tree_graphs(seed):
    """Spanning trees rooted at u on sparse random graphs; on a tree graph every block is a bridge,
    so each walk is one step (n - 1 in all) and the tree is the graph itself."""
    g = gg.random_connected(60, 0.04, seed)
    u = oracle.max_degree_pivot(g.row_ptr)
    parents, steps, _ = oracle.trees_blocks(g.row_ptr, g.col, u, seed, 0, 20, want_counts=False)
    for p in parents:
        brute.check_tree(g, p, u)
    t = gg.random_tree(40, seed)
    parents, steps, _ = oracle.trees_blocks(t.row_ptr, t.col, 5, seed, 0, 5, want_counts=False)
    assert (steps == t.n - 1).all()
    want = brute.rooted_parents(t.n, brute.edges_of(t), 5)
    assert (parents == want).all()


def test_wilson_blocks_expected_steps():
    """Walks stay inside their block: the expected steps are sum over the blocks B of
    sum_{v in B} deg_B(v) r(r_B, v), r_B the vertex of largest degree inside B (smallest ID on
    ties), r the effective resistance of G (equal to that of B between two of its vertices)."""
    g = CUT["K4_tail"]()
    g2 = gg.from_edges(9, [(0, 1), (1, 2), (2, 0), (2, 3), (3, 4), (4, 5), (5, 3), (5, 6), (6, 7), (7, 8), (8, 6),
                           (1, 7)])
    for gr, u in ((g, 6), (g2, 4)):
        T = 8000
        _, steps, _ = oracle.trees_blocks(gr.row_ptr, gr.col, u, 21, 0, T, want_parents=False, want_counts=False)
        eb, nb = oracle.blocks(gr.row_ptr, gr.col)
        P = brute.pinv(gr)
        rows = np.repeat(np.arange(gr.n), np.diff(gr.row_ptr))
        expect = 0.0
        for b in range(nb):
            sel = eb == b
            verts = sorted(set(rows[sel].tolist()))
            degb = {v: int(np.sum(rows[sel] == v)) for v in verts}
            root = min(verts, key=lambda v: (-degb[v], v))
            expect += sum(degb[v] * (P[root, root] + P[v, v] - 2 * P[root, v]) for v in verts)
        se = steps.std() / math.sqrt(T)
        assert abs(steps.mean() - expect) < 5 * se, (steps.mean(), expect)


# -------------------------------------------------------------------------------------
# Aggregation (Algorithm 2): exact expectation by enumeration, closed cases
# -------------------------------------------------------------------------------------
@pytest.mark.parametrize("name", list(TINY))
def test_tree_flow_enumeration_equals_effective_resistance(name):
    """Kirchhoff's theorem: averaged over all spanning trees, the signed count of P(v)'s
    edges on the tree path u->v equals r(u, v)."""
    g = TINY[name]()
    for u in range(g.n):
        _, parB, _ = oracle.bfs(g.row_ptr, g.col, u)
        trees = brute.spanning_trees(g, u)
        total = np.zeros(g.n, dtype=np.int64)
        for par in trees:
            total += oracle.tree_flow(u, parB, par)
        r = brute.effective_resistance_from(g, u)
        np.testing.assert_allclose(total / len(trees), r, atol=1e-12)


def test_tree_flow_tree_graph_is_distance():
    for seed in range(3):
        g = gg.random_tree(30, seed)
        u = seed
        dist, parB, _ = oracle.bfs(g.row_ptr, g.col, u)
        par, _ = oracle.wilson(g.row_ptr, g.col, u, 5, 0)
        c = oracle.tree_flow(u, parB, par)
        assert (c == dist).all()


def test_tree_flow_neighbours_and_bound():
    g = gg.random_connected(50, 0.1, 4)
    u = gg.max_degree_pivot(g)
    dist, parB, _ = oracle.bfs(g.row_ptr, g.col, u)
    for t in range(10):
        par, _ = oracle.wilson(g.row_ptr, g.col, u, 9, t)
        c = oracle.tree_flow(u, parB, par)
        assert (np.abs(c) <= dist).all()
        nb = g.col[g.row_ptr[u]:g.row_ptr[u + 1]]
        assert (c[nb] == (par[nb] == u)).all()
        assert c[u] == 0


def test_trees_threads_equal_one_sequential_call():
    """The parallel-over-trees timing leg: trees split over host threads give the steps and
    counts of one sequential call (also with more threads than trees)."""
    g = gg.rmat(10, 8, 2)
    u = oracle.max_degree_pivot(g.row_ptr)
    _, st, want = oracle.trees(g.row_ptr, g.col, u, 9, 3, 37, want_parents=False)
    for th in (1, 4, 64):
        st2, got = oracle.trees_threads(g.row_ptr, g.col, u, 9, 3, 37, th)
        assert (st2 == st).all() and (got == want).all()


def test_trees_counts_additive():
    g = gg.grid2d(6)
    u = gg.grid_center_pivot(6)
    _, _, c_all = oracle.trees(g.row_ptr, g.col, u, 2, 0, 30, want_parents=False)
    _, _, c_a = oracle.trees(g.row_ptr, g.col, u, 2, 0, 13, want_parents=False)
    _, _, c_b = oracle.trees(g.row_ptr, g.col, u, 2, 13, 17, want_parents=False)
    assert (c_all == c_a + c_b).all()


# -------------------------------------------------------------------------------------
# Solve and combine
# -------------------------------------------------------------------------------------
@pytest.mark.parametrize("maker,u", [(lambda: gg.grid2d(8), 27), (lambda: gg.random_connected(120, 0.05, 1), 3),
                                     (lambda: gg.rmat(9, 8, 2), 0)])
def test_solve_matches_pinv_column(maker, u):
    g = maker()
    x, it, relres = oracle.solve(g.row_ptr, g.col, u, tol=1e-13)
    assert it > 0 and relres < 1e-11
    P = brute.pinv(g)
    np.testing.assert_allclose(x, P[:, u], atol=1e-9 * np.abs(P[:, u]).max())
    assert abs(x.sum()) < 1e-10


def test_combine_identity_with_exact_resistances():
    """Eq. diag-comp: with exact r(u, v) and the exact pivot column, the combination
    reproduces the pseudoinverse diagonal."""
    g = gg.random_connected(40, 0.15, 6)
    P = brute.pinv(g)
    for u in (0, 7):
        r = brute.effective_resistance_from(g, u)
        tau = 1 << 20
        counts = np.round(r * tau).astype(np.int64)
        diag = oracle.combine(u, tau, counts, P[:, u])
        np.testing.assert_allclose(diag, np.diag(P), atol=2.0 / tau)


def test_closed_forms_complete_and_cycle():
    n = 9
    Pk = brute.pinv(gg.complete(n))
    np.testing.assert_allclose(np.diag(Pk), (n - 1) / n ** 2, atol=1e-12)
    Pc = brute.pinv(gg.cycle(n))
    np.testing.assert_allclose(np.diag(Pc), (n * n - 1) / (12 * n), atol=1e-12)
    r = brute.effective_resistance_from(gg.cycle(n), 0)
    d = np.arange(n)
    np.testing.assert_allclose(r, d * (n - d) / n, atol=1e-12)


def test_end_to_end_complete_graph_closed_form():
    n = 7
    g = gg.complete(n)
    res = oracle.diag_lpinv(g.row_ptr, g.col, 0, eps=0.3, seed=4)
    assert res["status"] == oracle.OK and res["ecc"] == 1
    assert res["tau"] == oracle.tau(n, n * (n - 1) // 2, 1, 0.3)
    assert np.max(np.abs(res["diag"] - (n - 1) / n ** 2)) <= 0.3


@pytest.mark.parametrize("name", ["K4", "C5", "grid3", "K23", "pendant_cycle"])
def test_end_to_end_within_eps_at_formula_tau(name):
    g = TINY[name]()
    u = 0
    res = oracle.diag_lpinv(g.row_ptr, g.col, u, eps=0.3, seed=21)
    assert res["status"] == oracle.OK
    assert np.max(np.abs(res["diag"] - np.diag(brute.pinv(g)))) <= 0.3


def test_end_to_end_grid32_statistical():
    """grid 32x32, tau = 1000: every diagonal entry within 5 sample standard errors of the
    dense pseudoinverse (per-vertex spread of c_T(v) from the same trees)."""
    g = gg.grid2d(32)
    u = gg.grid_center_pivot(32)
    assert u == 495
    T = 1000
    res = oracle.diag_lpinv(g.row_ptr, g.col, u, eps=0.3, seed=1, tau_override=T)
    assert res["status"] == oracle.OK and res["tau"] == T and res["ecc"] == 32
    _, parB, _ = oracle.bfs(g.row_ptr, g.col, u)
    parents, _, counts = oracle.trees(g.row_ptr, g.col, u, 1, 0, T)
    assert (counts == res["counts"]).all()
    per = np.stack([oracle.tree_flow(u, parB, p) for p in parents]).astype(np.float64)
    sd = per.std(axis=0, ddof=1)
    exact = np.diag(brute.pinv(g))
    err = np.abs(res["diag"] - exact)
    bound = 5 * sd / math.sqrt(T) + 1e-9
    assert (err <= bound).all(), float(np.max(err - bound))


def test_wilson_worked_example_k4():
    """Hand trace of Wilson's algorithm (ascending starts, successor floor(w deg / 2^32) of
    the ascending adjacency) on K4 rooted at u = 3, seed 0, tree 0.
      walk s=0 uses Philox((0,0,0,0); (0,0)) = the first known-answer vector:
        k=0 at 0 (nbrs 1,2,3): w=0x6627e8d5, floor(w*3/2^32) = 1 -> 2
        k=1 at 2 (nbrs 0,1,3): w=0xe169c58d, floor(w*3/2^32) = 2 -> 3 = u, stop
        retrace: parent[0] = 2, parent[2] = 3
      walk s=1 uses Philox((0,1,0,0); (0,0)) word 0 = 0x6ad0c5ec:
        k=0 at 1 (nbrs 0,2,3): floor(w*3/2^32) = 1 -> 2, in tree: parent[1] = 2
      s=2 is already in the tree.  Total 3 steps."""
    assert int(np_philox([[0], [1], [0], [0]], [[0], [0]])[0, 0]) == 0x6AD0C5EC
    g = gg.complete(4)
    par, steps = oracle.wilson(g.row_ptr, g.col, 3, 0, 0)
    assert list(par) == [2, 2, 3, -1]
    assert steps == 3


# ---------------------------------------------------------------------------------------
# Measures derived from diag(L^+) and spanning-edge counts
# ---------------------------------------------------------------------------------------
def _resistances(P):
    d = np.diag(P)
    return d[:, None] + d[None, :] - 2 * P


@pytest.mark.parametrize("g", [gg.grid2d(4), gg.rmat(7, 6, 2), gg.cycle(9), gg.complete_bipartite(3, 5)])
def test_centralities_match_definitions(g):
    """Farness, closeness and the Kirchhoff index against sums of effective resistances from
    the dense pseudoinverse; NRWB against its original definition with M = L + P."""
    P = brute.pinv(g)
    n = g.n
    R = _resistances(P)
    c = oracle.centralities(np.diag(P))
    np.testing.assert_allclose(c["farness"], R.sum(axis=1), rtol=1e-10)
    np.testing.assert_allclose(c["closeness"], (n - 1) / R.sum(axis=1), rtol=1e-10)
    assert c["kirchhoff"] == pytest.approx(R[np.triu_indices(n, 1)].sum(), rel=1e-10)
    # NRWB: the Lemma's closed form is 1/n + (sum over t != v of the definition's numerators) /
    # ((n-1) * sum of its denominators), with M = L + P inverted densely (the reading taken;
    # the definition as printed sums the per-t ratios instead, which the Lemma's proof does not)
    Minv = np.linalg.inv(brute.laplacian(g) + np.full((n, n), 1.0 / n))
    nrwb = np.empty(n)
    for v in range(n):
        num = den = 0.0
        for t in range(n):
            if t != v:
                num += Minv[t, t] - Minv[t, v]
                den += Minv[t, t] + Minv[v, v] - 2 * Minv[t, v]
        nrwb[v] = 1.0 / n + num / ((n - 1) * den)
    np.testing.assert_allclose(c["nrwb"], nrwb, rtol=1e-10)


def test_centralities_complete_graph_closed_form():
    n = 7
    P = brute.pinv(gg.complete(n))  # r(u,v) = 2/n
    c = oracle.centralities(np.diag(P))
    np.testing.assert_allclose(c["farness"], 2.0 * (n - 1) / n, rtol=1e-12)
    np.testing.assert_allclose(c["closeness"], n / 2.0, rtol=1e-12)
    assert c["kirchhoff"] == pytest.approx(n * (n - 1) / 2 * 2.0 / n, rel=1e-12)


@pytest.mark.parametrize("name,g,u", [("grid3", gg.grid2d(3), 4), ("K4", gg.complete(4), 0),
                                      ("K23", gg.complete_bipartite(2, 3), 1), ("C6", gg.cycle(6), 2)])
def test_edge_counts_over_all_trees_give_resistances(name, g, u):
    """Over every spanning tree once, count(e)/#trees = r(e) (Kirchhoff's theorem); the
    counts sum to (n-1) #trees and sit only at entries (a, b) with a < b."""
    trees = np.stack(brute.spanning_trees(g, u))
    cnt = oracle.edge_counts(g.row_ptr, g.col, trees, u)
    P = brute.pinv(g)
    R = _resistances(P)
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    assert (cnt[rows > g.col] == 0).all()
    assert cnt.sum() == (g.n - 1) * len(trees)
    for e in range(len(g.col)):
        a, b = rows[e], g.col[e]
        if a < b:
            assert cnt[e] / len(trees) == pytest.approx(R[a, b], abs=1e-12)


def test_edge_counts_on_tree_graph_and_sampled_trees():
    g = gg.random_tree(40, 5)
    par, _ = oracle.wilson(g.row_ptr, g.col, 3, 9, 0)
    cnt = oracle.edge_counts(g.row_ptr, g.col, np.stack([par, par]), 3)
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    assert (cnt[rows < g.col] == 2).all()  # a tree graph's only spanning tree holds every edge
    h = gg.grid2d(6)
    parents, _, _ = oracle.trees(h.row_ptr, h.col, 14, 3, 0, 4000, want_counts=False)
    cnt = oracle.edge_counts(h.row_ptr, h.col, parents, 14)
    R = _resistances(brute.pinv(h))
    rows = np.repeat(np.arange(h.n), np.diff(h.row_ptr))
    sel = rows < h.col
    est = cnt[sel] / 4000.0
    # Hoeffding: P(|est - r| > 0.05) <= 2 exp(-2 * 4000 * 0.05^2) ~ 4e-9 per edge
    assert np.abs(est - R[rows[sel], h.col[sel]]).max() <= 0.05


@pytest.mark.parametrize("name", ["K4", "grid3", "pendant_cycle", "K23"])
def test_edge_resistances_and_kirchhoff_denominator(name):
    """Over all spanning trees, count / #trees is every edge's effective resistance (Kirchhoff),
    and with these the denominator 1 - (1 - theta) w(e) r(e) makes the Sherman-Morrison form of
    the Kirchhoff edge centrality, n (1 - theta) w(e) |L+ b_e|^2 / denom, equal n times the change
    of tr(L+) when e is down-weighted to theta w(e) (dense pseudoinverses), unit and random
    weights (exact leverages w(e) r(e) times the tree count standing in for the counts)."""
    g = TINY[name]()
    trees = brute.spanning_trees(g, 0)
    N = len(trees)
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    counts = oracle.edge_counts(g.row_ptr, g.col, np.stack(trees), 0)
    P = brute.pinv(g)
    r_exact = P[rows, rows] + P[g.col, g.col] - 2 * P[rows, g.col]
    r, den = oracle.edge_resistances(g.row_ptr, g.col, counts, N, 0.4)
    np.testing.assert_allclose(r, r_exact, atol=1e-12)
    np.testing.assert_allclose(den, 1 - 0.6 * r_exact, atol=1e-12)
    rng = np.random.default_rng(3)
    for weighted in (False, True):
        w = gg.edge_weights(g, 5, "uniform", 0.5, 3.0) if weighted else np.ones(len(g.col))
        L = brute.laplacian_weighted(g, w) if weighted else brute.laplacian(g)
        Pw = np.linalg.pinv(L)
        lev = w * (Pw[rows, rows] + Pw[g.col, g.col] - 2 * Pw[rows, g.col])
        q = 1000
        for theta in (0.3, 0.8):
            rr, dd = oracle.edge_resistances(g.row_ptr, g.col, lev * q, q, theta, w=w if weighted else None)
            for e in rng.choice(np.flatnonzero(rows < g.col), size=3, replace=False):
                a, b = rows[e], g.col[e]
                be = np.zeros(g.n)
                be[a], be[b] = 1.0, -1.0
                Lt = L - (1 - theta) * w[e] * np.outer(be, be)
                direct = g.n * (np.trace(np.linalg.pinv(Lt)) - np.trace(Pw))
                sm = g.n * (1 - theta) * w[e] * np.sum((Pw @ be) ** 2) / dd[e]
                assert sm == pytest.approx(direct, rel=1e-9), (name, weighted, theta, e)
                assert rr[e] == pytest.approx(lev[e] / w[e], rel=1e-12)


def test_edge_sample_size_worked_example():
    # n = 100, m = 250, eps = 0.5, delta = 1/n: ln(2*250*100) = ln(50000) = 10.8198; 2/0.25 = 8 -> 86.56 -> 87
    assert oracle.edge_sample_size(100, 250, 0.5) == 87
    assert oracle.edge_sample_size(100, 250, 0.5, 0.01) == 87
    assert oracle.edge_sample_size(1000, 250, 0.5, 0.5) == 56  # ln(1000) = 6.9078 * 8 = 55.26


# ---------------------------------------------------------------------------------------
# Pivot by repeated BFS sweeps
# ---------------------------------------------------------------------------------------
def test_sweep_pivot_closed_forms():
    # path P_n: the sweeps alternate between the two ends, bounds are exact, centre floor((n-1)/2)
    for n in (2, 7, 10):
        piv, bound = oracle.sweep_pivot(gg.path(n).row_ptr, gg.path(n).col)
        assert piv == (n - 1) // 2
        assert list(bound) == [max(x, n - 1 - x) for x in range(n)]
    # star: the centre has eccentricity 1
    assert oracle.sweep_pivot(gg.star(9).row_ptr, gg.star(9).col)[0] == 0
    # cycle C_12: sources 0 and 6 alternate; bound max(d(0,x), d(6,x)) is smallest (3) at x = 3
    g = gg.cycle(12)
    piv, bound = oracle.sweep_pivot(g.row_ptr, g.col)
    d0 = np.minimum(np.arange(12), 12 - np.arange(12))
    d6 = np.abs(np.arange(12) - 6)
    assert piv == 3 and list(bound) == list(np.maximum(d0, d6))


def test_sweep_pivot_bounds_are_lower_bounds():
    """Against all-pairs distances: every bound is <= the true eccentricity and equals the
    largest distance from the sources the sweeps visited."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import shortest_path

    for g in (gg.grid2d(9, 5), gg.rmat(9, 8, 3), gg.random_tree(60, 2)):
        A = sp.csr_matrix((np.ones(len(g.col)), g.col, g.row_ptr), shape=(g.n, g.n))
        D = shortest_path(A, unweighted=True).astype(np.int64)
        ecc = D.max(axis=1)
        piv, bound = oracle.sweep_pivot(g.row_ptr, g.col)
        assert (bound <= ecc).all()
        src = int(np.argmax(np.diff(g.row_ptr)))
        want = np.zeros(g.n, dtype=np.int64)
        for _ in range(10):
            want = np.maximum(want, D[src])
            src = int(np.flatnonzero(D[src] == D[src].max())[0])
        assert (bound == want).all() and piv == int(np.argmin(want))


def test_oracle_clean_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    """The oracle's C code, built with gcc's AddressSanitizer and UndefinedBehaviorSanitizer (host
    code only), runs every step once on small graphs with a cut vertex: no invalid access, leak or
    undefined behaviour is reported."""
    import shutil
    import subprocess

    if not shutil.which("gcc"):
        pytest.skip("gcc is not available")
    src = os.path.join(os.path.dirname(oracle.__file__), "ustd_oracle.c")
    drv = os.path.join(os.path.dirname(oracle.__file__), "sanitize_driver.c")
    exe = tmp_path / "orc_san"
    flags = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
    subprocess.check_call(["gcc", "-std=c11", *flags, src, drv, "-o", str(exe), "-lm"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    out = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "ok" in out.stdout and "runtime error" not in out.stderr and "ERROR:" not in out.stderr
