"""Parity at the full workload sizes, with the problem settings the benchmark times
(eps = 0.3, Philox seed 1, max-degree pivot, mixed-precision solve to 1e-12).  The oracle
checks what it can compute at that size: the whole run for R-MAT scale 16; single trees at
chosen indices and flow counts over short tree ranges for the 1M-vertex hyperbolic graph
and R-MAT scale 22; for the batch of 64, whole members and bit-identity with single calls.
Properties that hold at any size (the solve residual, the combination) are checked on the
complete outputs."""
import numpy as np
import pytest
import scipy.sparse as sp
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


def _laplacian(g):
    A = sp.csr_matrix((np.ones(len(g.col)), g.col, g.row_ptr), shape=(g.n, g.n))
    return sp.diags(np.asarray(A.sum(axis=1)).ravel()) - A


def _check_solution(g, u, x, tol):
    """x solves L x = e_u - 1/n to relative residual tol, with zero mean."""
    b = -np.full(g.n, 1.0 / g.n)
    b[u] += 1.0
    r = b - _laplacian(g) @ x
    assert np.linalg.norm(r) <= 2 * tol * np.linalg.norm(b)
    assert abs(x.sum()) <= 1e-9 * np.abs(x).sum()


def _check_combine(diag, counts, x, u, tau):
    want = counts / tau - x[u] + 2.0 * x
    want[u] = x[u]
    np.testing.assert_allclose(diag, want, rtol=1e-14, atol=1e-14)


def _sampled(g, u, seed, tau, trees, count_range):
    G = api.Graph.from_host(g.row_ptr, g.col)
    p = api.problem(G, pivot=u, eps=0.3, seed=seed, solve_mode=api.SOLVE_MIXED, solve_tol=1e-12)
    for t in trees:
        say("tree", g.name, t)
        parents, steps = api.sample_trees(G, p, t, 1)
        want_par, want_steps = oracle.wilson(g.row_ptr, g.col, u, seed, t)
        assert int(steps[0]) == want_steps
        assert (parents[0].cpu().numpy() == want_par).all()
    t0, cnt = count_range
    say("counts", g.name, t0, cnt)
    counts, rep = api.flow_counts(G, p, t0, cnt)
    _, st, want = oracle.trees(g.row_ptr, g.col, u, seed, t0, cnt, want_parents=False)
    assert (counts.cpu().numpy() == want).all() and rep["walk_steps"] == int(st.sum())
    return G, p


def _full_run_properties(g, G, p, u):
    say("full run", g.name)
    diag, counts, rep = api.diag_lpinv_p(G, p)
    x, _ = api.solve_pivot_column(G, p)
    x = x.cpu().numpy()
    _check_solution(g, u, x, 1e-12)
    _check_combine(diag.cpu().numpy(), counts.cpu().numpy(), x, u, rep["tau"])
    return diag, counts, rep


def test_rmat16_whole_run(gpu):
    g = gg.rmat(16, 16, 1)
    u = gg.max_degree_pivot(g)
    G = api.Graph.from_host(g.row_ptr, g.col)
    p = api.problem(G, pivot=u, eps=0.3, seed=1, solve_mode=api.SOLVE_MIXED, solve_tol=1e-12)
    say("rmat16 gpu")
    diag, counts, rep = api.diag_lpinv_p(G, p)
    _, parB, ecc = oracle.bfs(g.row_ptr, g.col, u)
    tau = oracle.tau(g.n, g.m, ecc, 0.3)
    assert rep["tau"] == tau == 4576 and rep["ecc"] == ecc
    say("rmat16 oracle trees")
    _, st, want = oracle.trees(g.row_ptr, g.col, u, 1, 0, tau, want_parents=False)
    assert (counts.cpu().numpy() == want).all() and rep["walk_steps"] == int(st.sum())
    say("rmat16 oracle solve")
    x, _, rr = oracle.solve(g.row_ptr, g.col, u, tol=1e-12)
    ref = oracle.combine(u, tau, want, x)
    d = diag.cpu().numpy()
    assert np.abs(d - ref).max() <= 1e-10 * np.abs(ref).max()
    xg, _ = api.solve_pivot_column(G, p)
    _check_combine(d, counts.cpu().numpy(), xg.cpu().numpy(), u, tau)


def test_rmat16_weighted_sampled(gpu):
    """The weighted benchmark workload (R-MAT 16, conductances uniform in [1, 4), seed 1):
    tau, rho_max and the fixed-point shift exactly; the first and last trees and the
    fixed-point counts of two trees bit for bit; the full run's solve residual (weighted
    Laplacian) and combination."""
    g = gg.rmat(16, 16, 1)
    u = gg.max_degree_pivot(g)
    w = gg.edge_weights(g, 1, "uniform", 1.0, 4.0)
    G = api.Graph.from_host(g.row_ptr, g.col, weight=w)
    p = api.problem(G, pivot=u, eps=0.3, seed=1, solve_tol=1e-12)
    _, _, rmax = oracle.bpath_resistance(g.row_ptr, g.col, w, u)
    tau = oracle.tau_weighted(g.n, g.m, rmax, 0.3)
    k = oracle.fixed_shift(tau, rmax)
    for t in (0, tau - 1):
        say("weighted tree", t)
        parents, steps = api.sample_trees(G, p, t, 1)
        want_par, want_steps = oracle.wilson_weighted(g.row_ptr, g.col, w, u, 1, t)
        assert int(steps[0]) == want_steps
        assert (parents[0].cpu().numpy() == want_par).all()
    say("weighted counts")
    counts, rep = api.flow_counts(G, p, tau // 2, 2)
    assert rep["rho_max"] == rmax and rep["fixed_shift"] == k
    _, st, want = oracle.trees_weighted(g.row_ptr, g.col, w, u, 1, tau // 2, 2, k, want_parents=False)
    assert (counts.cpu().numpy() == want).all() and rep["walk_steps"] == int(st.sum())
    say("weighted full run")
    diag, counts, rep = api.diag_lpinv_p(G, p)
    assert rep["tau"] == tau and rep["fixed_shift"] == k
    x, _ = api.solve_pivot_column(G, p)
    x = x.cpu().numpy()
    A = sp.csr_matrix((w, g.col, g.row_ptr), shape=(g.n, g.n))
    L = sp.diags(np.asarray(A.sum(axis=1)).ravel()) - A
    b = -np.full(g.n, 1.0 / g.n)
    b[u] += 1.0
    assert np.linalg.norm(b - L @ x) <= 2e-12 * np.linalg.norm(b)
    c = counts.cpu().numpy().astype(np.float64)
    want_d = c / np.ldexp(float(tau), k) - x[u] + 2.0 * x
    want_d[u] = x[u]
    np.testing.assert_allclose(diag.cpu().numpy(), want_d, rtol=1e-14, atol=1e-14)


def test_rhg_1m_sampled(gpu):
    g = gg.hyperbolic(1_000_000, 20.0, 3.0, seed=1)
    u = gg.max_degree_pivot(g)
    _, _, ecc = oracle.bfs(g.row_ptr, g.col, u)
    tau = oracle.tau(g.n, g.m, ecc, 0.3)
    G, p = _sampled(g, u, 1, tau, [0, tau - 1], (tau // 2, 2))
    _full_run_properties(g, G, p, u)


@pytest.mark.slow
def test_rmat22_sampled(gpu):
    g = gg.rmat(22, 16, 1)
    u = gg.max_degree_pivot(g)
    _, _, ecc = oracle.bfs(g.row_ptr, g.col, u)
    tau = oracle.tau(g.n, g.m, ecc, 0.3)
    assert g.n > 131072  # global tree bitmap and 32-bit columns
    G, p = _sampled(g, u, 1, tau, [0, tau - 1], (4321, 1))
    _full_run_properties(g, G, p, u)


def test_batch64_members(gpu):
    members = gg.batch_members(64, 4096)
    graphs = [api.Graph.from_host(m["graph"].row_ptr, m["graph"].col) for m in members]
    probs = [api.problem(G, pivot=m["pivot"], eps=0.3, seed=m["seed"], tau_cap=m["tau_cap"],
                         solve_mode=api.SOLVE_MIXED, solve_tol=1e-12) for G, m in zip(graphs, members)]
    say("batch64 gpu")
    diags, counts, reps = api.batch_diag_lpinv(graphs, probs)
    ns = [m["graph"].n for m in members]
    rmat_small = min(range(32), key=lambda i: ns[i])
    grid_small = min(range(32, 64), key=lambda i: ns[i])
    grid_big = max(range(32, 64), key=lambda i: ns[i])
    rmat_big = max(range(32), key=lambda i: ns[i])
    for i in (rmat_small, grid_small):
        g, m = members[i]["graph"], members[i]
        say("batch member vs oracle", i, g.name, reps[i]["tau"])
        _, st, want = oracle.trees(g.row_ptr, g.col, reps[i]["pivot"], m["seed"], 0, reps[i]["tau"],
                                   want_parents=False)
        assert (counts[i].cpu().numpy() == want).all() and reps[i]["walk_steps"] == int(st.sum())
    for i in (grid_big, rmat_big, rmat_small):
        say("batch member vs single call", i, members[i]["graph"].name)
        d1, c1, r1 = api.diag_lpinv_p(graphs[i], api.with_engine(probs[i], api.ENGINE_WORKGROUP),
                                      ws=api.Workspace(graphs[i].row_ptr.device))
        assert torch.equal(c1, counts[i]) and torch.equal(d1, diags[i]) and r1["tau"] == reps[i]["tau"]
    g, m = members[grid_big]["graph"], members[grid_big]
    say("batch big grid tree")
    parents, steps = api.sample_trees(graphs[grid_big], probs[grid_big], 4095, 1)
    want_par, want_steps = oracle.wilson(g.row_ptr, g.col, m["pivot"], m["seed"], 4095)
    assert int(steps[0]) == want_steps and (parents[0].cpu().numpy() == want_par).all()


def test_rmat16_edge_counts_q_trees(gpu):
    """Spanning-edge counts of all q = ceil(2 eps^-2 ln(2m n)) trees at eps = 0.3 (the edges
    workload of the benchmark), bit-exact against the oracle's trees."""
    g = gg.rmat(16, 16, 1)
    u = gg.max_degree_pivot(g)
    q = oracle.edge_sample_size(g.n, g.m, 0.3)
    G = api.Graph.from_host(g.row_ptr, g.col)
    assert api.edge_sample_size(g.n, g.m, 0.3) == q
    say("rmat16 edges gpu", q)
    got, rep = api.edge_counts(G, api.problem(G, pivot=u, eps=0.3, seed=1), 0, q)
    say("rmat16 edges oracle")
    parents, st, _ = oracle.trees(g.row_ptr, g.col, u, 1, 0, q, want_counts=False)
    want = oracle.edge_counts(g.row_ptr, g.col, parents, u)
    assert (got.cpu().numpy() == want).all() and rep["walk_steps"] == int(st.sum())
