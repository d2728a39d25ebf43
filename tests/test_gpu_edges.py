"""GPU edge cases against the oracle: empty tree ranges on every entry point, the exact size
boundaries of the sampler's layouts (16-bit columns and reorder-buffer IDs up to n = 65536,
the LDS tree bitmap up to n = 131072), tree indices and seeds with high bits set, one tree
per batch, and a batch of one member."""
import numpy as np
import pytest
import torch

import oracle
from paper_2006_13679_amd import api
from paper_2006_13679_amd import graphgen as gg

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def gpu():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    api.lib()
    return torch.device("cuda:0")


def test_empty_tree_ranges(gpu):
    g = gg.grid2d(6)
    G = api.Graph.from_host(g.row_ptr, g.col)
    p = api.problem(G, pivot=7, seed=2, tau_override=5)
    say("empty ranges")
    par, steps = api.sample_trees(G, p, 3, 0)
    assert par.shape == (0, g.n) and steps.numel() == 0
    counts = torch.full((g.n,), 7, dtype=torch.int64, device="cuda")
    out, rep = api.flow_counts(G, p, 3, 0, counts=counts)
    assert (out.cpu().numpy() == 7).all() and rep["walk_steps"] == 0
    # no trees: only the fold of the input moves each (a > b) entry onto its (b, a) entry
    ec = torch.full((len(g.col),), 3, dtype=torch.int64, device="cuda")
    out, _ = api.edge_counts(G, p, 0, 0, counts=ec)
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    want = np.where(rows < g.col, 6, 0)
    assert (out.cpu().numpy() == want).all()
    tc = api.tree_counts(G, p, torch.empty((0, g.n), dtype=torch.int32), counts=torch.zeros(g.n, dtype=torch.int64,
                                                                                               device="cuda"))
    assert (tc.cpu().numpy() == 0).all()


@pytest.mark.parametrize("n,pivot", [(65536, 5), (65537, 5), (131072, 70000), (131073, 70000)])
def test_layout_boundaries_stars(gpu, n, pivot):
    """Stars with a leaf pivot: every tree is the star, reached through long walks (centre ->
    random leaves -> centre ...) at the largest vertex IDs of each layout."""
    g = gg.star(n)
    G = api.Graph.from_host(g.row_ptr, g.col)
    p = api.problem(G, pivot=pivot, seed=3, tau_override=4)
    say("star", n, pivot)
    par, steps = api.sample_trees(G, p, 0, 4)
    _, want_steps, want_counts = oracle.trees(g.row_ptr, g.col, pivot, 3, 0, 4, want_parents=False)
    par = par.cpu().numpy()
    assert par[0, pivot] == -1 and par[0, 0] == pivot and (np.delete(par[0], [0, pivot]) == 0).all()
    assert (steps.cpu().numpy() == want_steps).all()
    counts, _ = api.flow_counts(G, p, 0, 4)
    assert (counts.cpu().numpy() == want_counts).all()


def test_high_tree_index_and_seed(gpu):
    g = gg.rmat(9, 8, 4)
    u = gg.max_degree_pivot(g)
    G = api.Graph.from_host(g.row_ptr, g.col)
    seed = 0xFFFFFFFF00000001
    t0 = (1 << 40) + 12345
    p = api.problem(G, pivot=u, seed=seed, tau_override=100)
    say("high tree index")
    par, steps = api.sample_trees(G, p, t0, 9)
    want_par, want_steps, _ = oracle.trees(g.row_ptr, g.col, u, seed, t0, 9, want_counts=False)
    assert (par.cpu().numpy() == want_par).all() and (steps.cpu().numpy() == want_steps).all()


def test_one_tree_per_batch(gpu):
    g = gg.rmat(10, 8, 6)
    u = gg.max_degree_pivot(g)
    G = api.Graph.from_host(g.row_ptr, g.col)
    say("one tree per batch")
    p1 = api.problem(G, pivot=u, seed=5, tau_override=37, trees_per_batch=1)
    pa = api.problem(G, pivot=u, seed=5, tau_override=37)
    d1, c1, r1 = api.diag_lpinv_p(G, p1)
    da, ca, ra = api.diag_lpinv_p(G, pa)
    assert r1["n_batches"] == 37 and r1["trees_per_batch"] == 1
    assert torch.equal(c1, ca) and torch.equal(d1, da)
    _, _, want = oracle.trees(g.row_ptr, g.col, u, 5, 0, 37, want_parents=False)
    assert (c1.cpu().numpy() == want).all()


def test_batch_of_one_member(gpu):
    g = gg.grid2d(12)
    G = api.Graph.from_host(g.row_ptr, g.col)
    say("batch of one")
    p = api.problem(G, pivot=gg.grid_center_pivot(12), seed=4, tau_override=300)
    (db,), (cb,), (rb,) = api.batch_diag_lpinv([G], [p])
    ds, cs, rs = api.diag_lpinv_p(G, p)
    assert torch.equal(cb, cs) and torch.equal(db, ds)
    assert rb["tau"] == rs["tau"] == 300 and rb["walk_steps"] == rs["walk_steps"]


def test_two_tree_pools_match_one(gpu):
    """A graph past the LDS bitmap runs its batches on two pools and two streams; the counts,
    walk totals and diagonal are those of a single-pool run with the same batch split and of
    a run split by tree ranges (integer counts: any order of batches gives the same sums)."""
    g = gg.rmat(18, 8, 2)
    assert g.n > 131072
    u = gg.max_degree_pivot(g)
    G = api.Graph.from_host(g.row_ptr, g.col)
    tau_ = 9000
    say("two pools", g.n, tau_)
    p2 = api.problem(G, pivot=u, seed=6, tau_override=tau_)
    ws = api.Workspace("cuda")
    assert api.workspace_bytes(p2) > 0
    d2, c2, r2 = api.diag_lpinv_p(G, p2, ws=ws)
    assert r2["n_batches"] >= 2
    p1 = api.problem(G, pivot=u, seed=6, tau_override=tau_, trees_per_batch=-(-tau_ // r2["n_batches"]))
    d1, c1, r1 = api.diag_lpinv_p(G, p1, ws=ws)
    assert r1["n_batches"] == r2["n_batches"]
    assert torch.equal(c1, c2) and torch.equal(d1, d2)
    assert r1["walk_steps"] == r2["walk_steps"] and r1["walk_draws"] == r2["walk_draws"]
    part = torch.zeros_like(c2)
    steps = 0
    for b0, c in [(0, 4000), (4000, 5000)]:
        _, rp = api.flow_counts(G, p2, b0, c, counts=part)
        steps += rp["walk_steps"]
    assert torch.equal(part, c2) and steps == r2["walk_steps"]
    _, st, want = oracle.trees(g.row_ptr, g.col, u, 6, 8990, 10, want_parents=False)
    got, rp = api.flow_counts(G, p2, 8990, 10)
    assert (got.cpu().numpy() == want).all() and rp["walk_steps"] == int(st.sum())


@pytest.mark.parametrize("name,make", [("grid50", lambda: gg.grid2d(50)), ("grid51", lambda: gg.grid2d(51)),
                                       ("rmat11", lambda: gg.rmat(11, 4, 1))])
def test_graph_in_lds_boundary(gpu, name, make):
    """Small unweighted graphs whose row pointers, flag words and 16-bit columns fit 40 KB are
    sampled from LDS (grid 50x50: 39,604 B; R-MAT 11 with edge factor 4: 38,164 B), with the
    long re-walks' Philox words computed by the whole wave; grid 51x51 (41,212 B) just misses.
    Parents, steps and counts match the oracle on both sides."""
    g = make()
    u = gg.max_degree_pivot(g) if name.startswith("rmat") else gg.grid_center_pivot(int(name[4:]))
    G = api.Graph.from_host(g.row_ptr, g.col)
    p = api.problem(G, pivot=u, seed=8, tau_override=70)
    say("graph in LDS", name, g.n)
    par, steps = api.sample_trees(G, p, 3, 70)
    want_par, want_steps, _ = oracle.trees(g.row_ptr, g.col, u, 8, 3, 70, want_counts=False)
    assert (par.cpu().numpy() == want_par).all() and (steps.cpu().numpy() == want_steps).all()
    counts, rep = api.flow_counts(G, p, 0, 70)
    _, st, want = oracle.trees(g.row_ptr, g.col, u, 8, 0, 70, want_parents=False)
    assert (counts.cpu().numpy() == want).all() and rep["walk_steps"] == int(st.sum())
