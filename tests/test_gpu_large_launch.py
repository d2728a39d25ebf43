"""Launches with one work-item per (vertex, tree) past 2^31 work-items: a dispatch counts its
work-items in 32 bits, so the library splits such launches into tree chunks.  Parent arrays of
a sample past that size equal the oracle's on both sides of the chunk boundary; the per-block
sampler's join over more trees than one chunk gives the same counts and steps as two calls
that each fit in one chunk."""
import pytest
import torch

import oracle
from paper_2006_13679_amd import api
from paper_2006_13679_amd import graphgen as gg

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def big():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    api.lib()
    g = gg.rmat(19, 8, 7)
    u = oracle.max_degree_pivot(g.row_ptr)
    return g, u, api.Graph.from_host(g.row_ptr, g.col), (1 << 31) // g.n


def test_parents_of_a_sample_past_one_launch(big):
    g, u, G, chunk = big
    count = chunk + 61
    assert count <= 8192 and count * g.n > (1 << 31)
    p = api.problem(G, pivot=u, seed=13, trees_per_batch=8192)
    say("parents of", count, "trees, n =", g.n, "chunk", chunk)
    parents, steps = api.sample_trees(G, p, 0, count)
    for t in (0, chunk - 1, chunk, count - 1):
        say("tree", t)
        want_par, want_steps = oracle.wilson(g.row_ptr, g.col, u, 13, t)
        assert int(steps[t]) == want_steps, t
        assert (parents[t].cpu().numpy() == want_par).all(), t
    del parents


def test_block_join_past_one_launch(big):
    g, u, G, chunk = big
    count = 8192
    assert count > chunk
    p = api.problem(G, pivot=u, seed=17, trees_per_batch=count, wilson_variant=api.WILSON_BLOCKS)
    say("per-block counts of", count, "trees in one batch")
    whole, rw = api.flow_counts(G, p, 0, count)
    assert rw["n_batches"] == 1
    say("the same trees in two calls of at most one chunk")
    part, r1 = api.flow_counts(G, p, 0, chunk)
    part, r2 = api.flow_counts(G, p, chunk, count - chunk, counts=part)
    assert torch.equal(whole, part)
    assert rw["walk_steps"] == r1["walk_steps"] + r2["walk_steps"]
    say("last trees against the oracle")
    tail, rt = api.flow_counts(G, p, count - 4, 4)
    _, st, want = oracle.trees_blocks(g.row_ptr, g.col, u, 17, count - 4, 4, want_parents=False)
    assert (tail.cpu().numpy() == want).all() and rt["walk_steps"] == int(st.sum())
