"""Parity at the full workload sizes, with the problem settings the benchmark times
(eps = 0.3, Philox seed 1, max-degree pivot, mixed-precision solve to 1e-12).  The oracle
checks what it can compute at that size: the whole run for R-MAT scale 16; single trees at
chosen indices and flow counts over short tree ranges for the 1M-vertex hyperbolic graph
and R-MAT scale 22 (across the full run's batch boundaries and at the end), with the full run's
counts equal to range calls split elsewhere; for the batch of 64, whole members against the
oracle and every member bit-identical to its single call.
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


def _threads():
    import os

    n = len(os.sched_getaffinity(0))
    cap = os.environ.get("OMP_NUM_THREADS")
    return max(1, min(n, int(cap))) if cap and cap.isdigit() and int(cap) > 0 else n


def _oracle_range(g, u, seed, t0, cnt, parB):
    return oracle.trees_threads(g.row_ptr, g.col, u, seed, t0, cnt, _threads(), parB=parB)


def _full_size_checks(g, u, ranges, split):
    """The benchmark's problem (eps 0.3, seed 1, mixed-precision solve to 1e-12) end to end, then:
    the first and last trees bit for bit; flow counts of tree ranges at the full run's batch
    boundaries and of the last 16 trees against the oracle; the full run's counts equal to the
    sum of two range calls split elsewhere (other batch boundaries); the solve residual and the
    combination on the complete outputs; and the GPU's FP64 and mixed-precision pivot columns
    against the oracle's FP64 column, with the diagonal difference they make at identical
    counts (Eq. diag-comp) within 1e-10 of the diagonal's magnitude."""
    _, parB, ecc = oracle.bfs(g.row_ptr, g.col, u)
    tau = oracle.tau(g.n, g.m, ecc, 0.3)
    G = api.Graph.from_host(g.row_ptr, g.col)
    p = api.problem(G, pivot=u, eps=0.3, seed=1, solve_mode=api.SOLVE_MIXED, solve_tol=1e-12)
    say("full run", g.name, "tau", tau)
    diag, counts, rep = api.diag_lpinv_p(G, p)
    assert rep["tau"] == tau and rep["ecc"] == ecc
    per = -(-tau // rep["n_batches"])  # the full run's batch size (equal split)
    say("batches", rep["n_batches"], "of", per)
    for t in (0, tau - 1):
        say("tree", g.name, t)
        parents, steps = api.sample_trees(G, p, t, 1)
        want_par, want_steps = oracle.wilson(g.row_ptr, g.col, u, 1, t)
        assert int(steps[0]) == want_steps and (parents[0].cpu().numpy() == want_par).all()
    for t0, cnt in ranges(tau, per):
        say("counts vs oracle", g.name, t0, cnt)
        got, r = api.flow_counts(G, p, t0, cnt)
        st, want = _oracle_range(g, u, 1, t0, cnt, parB)
        assert (got.cpu().numpy() == want).all() and r["walk_steps"] == int(st.sum())
    say("additivity", g.name, split)
    part, r1 = api.flow_counts(G, p, 0, split)
    part, r2 = api.flow_counts(G, p, split, tau - split, counts=part)
    assert torch.equal(part, counts) and r1["walk_steps"] + r2["walk_steps"] == rep["walk_steps"]
    x64, rf = api.solve_pivot_column(G, _fp64(p))
    xm, rm = api.solve_pivot_column(G, p)
    xm = xm.cpu().numpy()
    _check_solution(g, u, xm, 1e-12)
    c = counts.cpu().numpy()
    d = diag.cpu().numpy()
    _check_combine(d, c, xm, u, tau)
    say("oracle solve", g.name)
    xo, _, _ = oracle.solve(g.row_ptr, g.col, u, tol=1e-12)
    ref = oracle.combine(u, tau, c, xo)
    dmax = np.abs(ref).max()
    for name, x in (("fp64", x64.cpu().numpy()), ("mixed", xm)):
        dd = oracle.combine(u, tau, c, x) - ref
        rel = np.abs(dd).max() / dmax
        say("diag vs oracle at identical counts", name, "%.3e" % rel, "x rel %.3e" % (np.abs(x - xo).max() / np.abs(xo).max()))
        assert rel <= 1e-10, (name, rel)
    assert rf["solve_converged"] == 1 and rm["solve_converged"] == 1


def _fp64(p):
    q = api.Problem.from_buffer_copy(p)
    q.solve_mode = api.SOLVE_FP64
    return q


@pytest.fixture(scope="module")
def rhg1m():
    return gg.hyperbolic(1_000_000, 20.0, 3.0, seed=1)


def test_rhg_1m_full_size(gpu, rhg1m):
    """Hyperbolic graph, 1M vertices: two tree pools, batches of an equal split; ranges across
    each batch boundary and the last 16 trees."""
    g = rhg1m
    u = gg.max_degree_pivot(g)

    def ranges(tau, per):
        out = [(b - 8, 16) for b in range(per, tau, per)]
        return out + [(tau - 16, 16)]

    _full_size_checks(g, u, ranges, 7001)


@pytest.mark.slow
def test_rmat22_full_size(gpu):
    """R-MAT scale 22 (the benchmark's default workload): two batches; ranges across the batch
    boundary and the last 16 trees."""
    g = gg.rmat(22, 16, 1)
    u = gg.max_degree_pivot(g)
    assert g.n > 131072  # tree state in the records, 32-bit columns, edge entries

    def ranges(tau, per):
        return [(per - 8, 16), (tau - 16, 16)]

    _full_size_checks(g, u, ranges, 3001)


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
    ws1 = api.Workspace(graphs[0].row_ptr.device)
    for i in range(len(members)):
        say("batch member vs single call", i, members[i]["graph"].name)
        d1, c1, r1 = api.diag_lpinv_p(graphs[i], api.with_engine(probs[i], api.ENGINE_WORKGROUP), ws=ws1)
        assert torch.equal(c1, counts[i]) and torch.equal(d1, diags[i]), i
        for k in ("tau", "walk_steps", "pivot", "ecc", "solve_iters", "solve_relres"):
            assert r1[k] == reps[i][k], (i, k)
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
