"""The seeded input generators (shared by the oracle side and the HIP side), checked
against plain definitions: R-MAT against a per-edge loop over the same random stream,
random hyperbolic graphs against an all-pairs distance test, CSR invariants."""
import math

import numpy as np

from paper_2006_13679_amd import graphgen as gg


def _csr_ok(g):
    rp, col = g.row_ptr, g.col
    assert rp[0] == 0 and rp[-1] == len(col) and (np.diff(rp) >= 1).all()
    rows = np.repeat(np.arange(g.n), np.diff(rp))
    assert (col != rows).all()
    for v in range(g.n):
        r = col[rp[v]:rp[v + 1]]
        assert (np.diff(r) > 0).all()
    fwd = set(zip(rows.tolist(), col.tolist()))
    assert all((b, a) in fwd for a, b in fwd)
    # connected: BFS from 0 reaches everything
    seen = np.zeros(g.n, bool)
    seen[0] = True
    frontier = [0]
    while frontier:
        nxt = []
        for v in frontier:
            for w in col[rp[v]:rp[v + 1]]:
                if not seen[w]:
                    seen[w] = True
                    nxt.append(int(w))
        frontier = nxt
    assert seen.all()


def test_rmat_edges_match_per_edge_definition():
    scale, ef, seed, chunk = 6, 3, 11, 50
    s, d = gg.rmat_edges(scale, ef, seed, chunk=chunk)
    rng = np.random.default_rng(seed)
    M = ef << scale
    a, ab, abc = 0.57, 0.76, 0.95
    want_s, want_d = np.zeros(M, np.int64), np.zeros(M, np.int64)
    for lo in range(0, M, chunk):
        L = min(M, lo + chunk) - lo
        for level in range(scale):
            r = rng.random(L)
            for i in range(L):
                if r[i] < a:
                    sb, db = 0, 0
                elif r[i] < ab:
                    sb, db = 0, 1
                elif r[i] < abc:
                    sb, db = 1, 0
                else:
                    sb, db = 1, 1
                want_s[lo + i] |= sb << level
                want_d[lo + i] |= db << level
    assert (s == want_s).all() and (d == want_d).all()


def test_rmat_graph_is_canonical():
    g = gg.rmat(9, 8, 2)
    _csr_ok(g)
    assert g.n <= 512 and 2 * g.m == len(g.col)


def test_rhg_edges_match_all_pairs():
    n, seed = 1500, 3
    rng = np.random.default_rng(seed)
    theta = rng.random(n) * 2 * np.pi
    u01 = rng.random(n)
    R = 2 * math.log(n) + 0.5
    r = np.arccosh(1.0 + u01 * (math.cosh(R) - 1.0))
    s, d = gg._rhg_edges(r, theta, R)
    got = set(zip(np.minimum(s, d).tolist(), np.maximum(s, d).tolist()))
    assert len(got) == len(s)  # each pair once
    ch, sh = np.cosh(r), np.sinh(r)
    dth = np.abs(theta[:, None] - theta[None, :])
    dth = np.minimum(dth, 2 * np.pi - dth)
    cd = ch[:, None] * ch[None, :] - sh[:, None] * sh[None, :] * np.cos(dth)
    iu = np.triu_indices(n, 1)
    mask = cd[iu] < math.cosh(R)
    want = set(zip(iu[0][mask].tolist(), iu[1][mask].tolist()))
    assert got == want


def test_rhg_average_degree_and_shape():
    g = gg.hyperbolic(20000, 20.0, 3.0, seed=1)
    assert abs(2 * g.m / g.n - 20.0) <= 0.2 and g.n >= 19000
    deg = np.diff(g.row_ptr)
    assert deg.max() > 50 * np.median(deg)  # heavy tail of a power law with exponent 3
    _csr_ok(gg.hyperbolic(3000, 20.0, 3.0, seed=2))


def test_grid_and_batch_recipe():
    g = gg.grid2d(5, 4)
    _csr_ok(g)
    assert g.n == 20 and g.m == 5 * 3 + 4 * 4
    ms = gg.batch_members(8, 123)
    for i, m in enumerate(ms):
        rng = np.random.default_rng(i)
        if i < 4:
            scale, ef = int(rng.integers(10, 17)), int(rng.integers(8, 17))
            assert m["graph"].name == "rmat-s%d-ef%d-seed%d" % (scale, ef, i)
            assert m["pivot"] == gg.max_degree_pivot(m["graph"])
        else:
            side = int(rng.integers(16, 257))
            assert m["graph"].n == side * side and m["pivot"] == gg.grid_center_pivot(side)
        assert m["seed"] == i and m["tau_cap"] == 123
