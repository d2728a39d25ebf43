"""The allocation-free entry point (ustd_diag_lpinv_noalloc): the library's static device
scratch in place of a caller workspace.  Its counts, walk steps and diagonal must equal those
of ustd_diag_lpinv (same one-workgroup solve engine) on two calls in a row, the second on a
smaller graph, so the scratch's leftover contents from the first call cannot matter."""
import ctypes

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


def _compare(g, u, seed, **kw):
    G = api.Graph.from_host(g.row_ptr, g.col)
    p = api.problem(G, pivot=u, eps=0.3, seed=seed, solve_tol=1e-12, **kw)
    say("noalloc", g.name, g.n)
    diag = torch.full((g.n,), float("nan"), dtype=torch.float64, device="cuda")
    counts = torch.full((g.n,), -1, dtype=torch.int64, device="cuda")
    rep = api.diag_lpinv_noalloc_p(G, p, diag, counts)
    say("noalloc trees per batch", rep["trees_per_batch"], "batches", rep["n_batches"], "tau", rep["tau"])
    d1, c1, r1 = api.diag_lpinv_p(G, api.with_engine(p, api.ENGINE_WORKGROUP), ws=api.Workspace(G.row_ptr.device))
    assert torch.equal(counts, c1)
    assert torch.equal(diag, d1)
    for k in ("tau", "walk_steps", "pivot", "ecc", "solve_iters", "solve_relres"):
        assert rep[k] == r1[k], k
    assert rep["solve_converged"] == 1
    return rep


def test_noalloc_matches_workspace_entry_point_twice(gpu):
    # first call: several batches of trees through the 64 MiB scratch
    g1 = gg.rmat(14, 16, 1)
    r = _compare(g1, -1, 3)
    assert r["n_batches"] >= 2
    _, st, want = oracle.trees(g1.row_ptr, g1.col, r["pivot"], 3, 0, r["tau"], want_parents=False)
    assert r["walk_steps"] == int(st.sum())
    # second call, smaller graph: the first call's contents of the scratch must not matter
    g2 = gg.grid2d(24)
    r2 = _compare(g2, gg.grid_center_pivot(24), 5, tau_override=300)
    assert r2["tau"] == 300


def test_noalloc_rejects_problems_beyond_the_scratch(gpu):
    """A problem whose workspace does not fit the static scratch even at one tree per batch is
    refused with USTD_ENOMEM before any device work (fake device pointers are never read)."""
    p = api.Problem(n=1 << 21, nnz=1 << 25, d_row_ptr=0x1000, d_col=0x2000, pivot=0, eps=0.3, seed=1)
    diag = torch.empty(8, dtype=torch.float64, device="cuda")
    rc = api.lib().ustd_diag_lpinv_noalloc(ctypes.byref(p), api._ptr(diag), None, None, None)
    assert rc == api.ENOMEM
    assert b"static scratch" in api.lib().ustd_last_error()
    # an explicit trees_per_batch that does not fit is refused too
    g = gg.rmat(12, 8, 2)
    G = api.Graph.from_host(g.row_ptr, g.col)
    q = api.problem(G, pivot=-1, trees_per_batch=8192)
    d = torch.empty(g.n, dtype=torch.float64, device="cuda")
    assert api.lib().ustd_diag_lpinv_noalloc(ctypes.byref(q), api._ptr(d), None, None, None) == api.ENOMEM
