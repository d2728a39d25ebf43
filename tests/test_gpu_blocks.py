"""GPU parity of Wilson's algorithm per biconnected component (wilson_variant = BLOCKS): the
trees, walk steps and flow counts of the library equal the oracle's per-block variant bit for
bit, on graphs with many cut vertices (R-MAT, sparse random graphs, trees, stars), with one
block (grids, complete graphs), and past the 16-bit and LDS-bitmap sizes of the block-split
graph; the diagonal equals the oracle's."""
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


def cases():
    return [
        ("pendant_cycle", gg.from_edges(6, [(0, 1), (1, 2), (2, 3), (3, 0), (3, 4), (4, 5), (1, 3)]), 5),
        ("bowtie", gg.from_edges(5, [(0, 1), (1, 2), (2, 0), (2, 3), (3, 4), (4, 2)]), 0),
        ("K4_tail", gg.from_edges(7, [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3), (3, 4), (4, 5), (4, 6)]), 6),
        ("star", gg.star(12), 4),
        ("tree", gg.random_tree(60, 2), 7),
        ("path", gg.path(30), 13),
        ("K5", gg.complete(5), 2),
        ("grid12", gg.grid2d(12), 66),
        ("gnp", gg.random_connected(300, 0.008, 4), -1),
        ("rmat10", gg.rmat(10, 8, 3), -1),
        ("rmat13", gg.rmat(13, 8, 1), -1),
    ]


@pytest.mark.parametrize("idx", range(len(cases())))
def test_block_trees_and_counts_bit_exact(gpu, idx):
    name, g, piv = cases()[idx]
    u = piv if piv >= 0 else oracle.max_degree_pivot(g.row_ptr)
    G = api.Graph.from_host(g.row_ptr, g.col)
    T = 40 if g.n > 2000 else 90
    say("blocks", name, g.n, T)
    p = api.problem(G, pivot=u, seed=31, trees_per_batch=32, wilson_variant=api.WILSON_BLOCKS)
    parents, steps = api.sample_trees(G, p, 3, min(T, 32))
    want_par, want_steps, _ = oracle.trees_blocks(g.row_ptr, g.col, u, 31, 3, min(T, 32), want_counts=False)
    assert (steps.cpu().numpy() == want_steps).all()
    assert (parents.cpu().numpy() == want_par).all()
    counts, rep = api.flow_counts(G, p, 5, T)
    _, st, want = oracle.trees_blocks(g.row_ptr, g.col, u, 31, 5, T, want_parents=False)
    assert (counts.cpu().numpy() == want).all() and rep["walk_steps"] == int(st.sum())


@pytest.mark.parametrize("scale", [15, 17])
def test_block_split_graph_sizes(gpu, scale):
    """R-MAT 15 (block-split graph past the 16-bit columns) and R-MAT 17 (past the LDS bitmap: tree
    state in the records, edge entries)."""
    g = gg.rmat(scale, 8, 3)
    u = oracle.max_degree_pivot(g.row_ptr)
    G = api.Graph.from_host(g.row_ptr, g.col)
    p = api.problem(G, pivot=u, seed=9, trees_per_batch=16, wilson_variant=api.WILSON_BLOCKS)
    say("blocks large", scale, g.n)
    parents, steps = api.sample_trees(G, p, 1, 6)
    want_par, want_steps, _ = oracle.trees_blocks(g.row_ptr, g.col, u, 9, 1, 6, want_counts=False)
    assert (steps.cpu().numpy() == want_steps).all() and (parents.cpu().numpy() == want_par).all()
    counts, rep = api.flow_counts(G, p, 0, 20)
    _, st, want = oracle.trees_blocks(g.row_ptr, g.col, u, 9, 0, 20, want_parents=False)
    assert (counts.cpu().numpy() == want).all() and rep["walk_steps"] == int(st.sum())


def test_block_variant_diag(gpu):
    """ApproxDiagLpinv with the per-block sampler: counts equal to the oracle's over all tau trees,
    the diagonal within 1e-10 of the oracle's; the plain variant's diagonal is within the error
    bound of both (the two samplers draw the same distribution)."""
    g = gg.rmat(12, 8, 2)
    u = oracle.max_degree_pivot(g.row_ptr)
    G = api.Graph.from_host(g.row_ptr, g.col)
    p = api.problem(G, pivot=u, eps=0.3, seed=4, solve_tol=1e-12, wilson_variant=api.WILSON_BLOCKS)
    diag, counts, rep = api.diag_lpinv_p(G, p)
    _, _, ecc = oracle.bfs(g.row_ptr, g.col, u)
    tau = oracle.tau(g.n, g.m, ecc, 0.3)
    assert rep["tau"] == tau
    _, st, want = oracle.trees_blocks(g.row_ptr, g.col, u, 4, 0, tau, want_parents=False)
    assert (counts.cpu().numpy() == want).all() and rep["walk_steps"] == int(st.sum())
    x, _, _ = oracle.solve(g.row_ptr, g.col, u, tol=1e-12)
    ref = oracle.combine(u, tau, want, x)
    d = diag.cpu().numpy()
    assert np.abs(d - ref).max() <= 1e-10 * np.abs(ref).max()
    plain, _, rp_ = api.diag_lpinv_p(G, api.problem(G, pivot=u, eps=0.3, seed=4, solve_tol=1e-12))
    assert np.abs(plain.cpu().numpy() - d).max() <= 2 * 0.3


def test_block_variant_rejects_weights_and_batches(gpu):
    g = gg.grid2d(5)
    w = gg.edge_weights(g, 1, "uniform", 1.0, 2.0)
    Gw = api.Graph.from_host(g.row_ptr, g.col, weight=w)
    with pytest.raises(api.UstdError) as e:
        api.diag_lpinv_p(Gw, api.problem(Gw, pivot=0, wilson_variant=api.WILSON_BLOCKS))
    assert e.value.status == api.EINVAL
    G = api.Graph.from_host(g.row_ptr, g.col)
    with pytest.raises(api.UstdError) as e:
        api.batch_diag_lpinv([G], [api.problem(G, pivot=0, wilson_variant=api.WILSON_BLOCKS)])
    assert e.value.status == api.EINVAL
