"""Planned batches (ustd_batch_plan_*): executions, HIP-graph replays and every schedule the
autotuner tries give results bit-identical to the one-shot batch call and to single calls; the
counts of some members are checked against the oracle; the tuner's cache round-trips."""
import json

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


def _members():
    """Mixed sizes and depths: R-MAT, grids (one past 16384 vertices: the level-by-level BFS
    replay), a path, a weighted R-MAT member and a mixed-precision solve."""
    out = []
    for g, piv, seed, kw in [
        (gg.rmat(10, 8, 1), -1, 3, dict(tau_cap=90)),
        (gg.grid2d(12), 78, 4, dict(tau_override=70)),
        (gg.rmat(11, 12, 2), -1, 5, dict(tau_cap=80, trees_per_batch=30)),
        (gg.path(30), 0, 6, dict(tau_cap=40)),
        (gg.grid2d(130), 8450, 7, dict(tau_cap=6)),
        (gg.grid2d(16), 0, 8, dict(tau_cap=30, solve_mode=api.SOLVE_MIXED)),
    ]:
        G = api.Graph.from_host(g.row_ptr, g.col)
        out.append((g, None, G, api.problem(G, pivot=piv, seed=seed, solve_tol=1e-12, **kw)))
    g = gg.rmat(9, 8, 4)
    w = gg.edge_weights(g, 5, "uniform", 0.5, 4.0)
    Gw = api.Graph.from_host(g.row_ptr, g.col, weight=w)
    out.append((g, w, Gw, api.problem(Gw, pivot=gg.max_degree_pivot(g), seed=9, tau_override=50)))
    return out


@pytest.fixture(scope="module")
def batch(gpu):
    mem = _members()
    graphs, probs = [m[2] for m in mem], [m[3] for m in mem]
    say("one-shot batch", [m[0].n for m in mem])
    diags, counts, reps = api.batch_diag_lpinv(graphs, probs)
    return mem, graphs, probs, diags, counts, reps


def _same(plan, diags, counts, reps, r2, tag, same_sampler=True):
    """Counts, diagonals and the committed walk steps are the same for every schedule; the
    speculative draws are a property of the sampler variant (the layout)."""
    for i in range(len(diags)):
        assert torch.equal(plan.counts[i], counts[i]), (tag, i)
        assert torch.equal(plan.diags[i], diags[i]), (tag, i)
        for k in ("tau", "pivot", "ecc", "walk_steps", "solve_iters", "solve_relres", "fixed_shift"):
            assert r2[i][k] == reps[i][k], (tag, i, k)
        assert r2[i]["walk_draws"] >= r2[i]["walk_steps"], (tag, i)
        if same_sampler:
            assert r2[i]["walk_draws"] == reps[i]["walk_draws"], (tag, i)


def test_one_shot_matches_single_calls_and_oracle(batch):
    mem, graphs, probs, diags, counts, reps = batch
    for i, (g, w, G, p) in enumerate(mem):
        say("single", i, g.n)
        d1, c1, r1 = api.diag_lpinv_p(G, api.with_engine(p, api.ENGINE_WORKGROUP), ws=api.Workspace(G.row_ptr.device))
        assert torch.equal(counts[i], c1) and torch.equal(diags[i], d1), i
        assert reps[i]["walk_steps"] == r1["walk_steps"] and reps[i]["solve_iters"] == r1["solve_iters"], i
    for i in (0, 3, 4):
        g, _, _, p = mem[i]
        _, st, want = oracle.trees(g.row_ptr, g.col, reps[i]["pivot"], p.seed, 0, reps[i]["tau"], want_parents=False)
        assert (counts[i].cpu().numpy() == want).all() and reps[i]["walk_steps"] == int(st.sum()), i


SCHEDULES = [
    dict(),
    dict(group_fills=1),
    dict(group_fills=4),
    dict(group_fills=-1),
    dict(agg_chunk=4),
    dict(agg_chunk=8),
    dict(layout=api.LAYOUT_RECORDS),
    dict(fill_trees=37),  # many pool fills, a member split across fills
    dict(group_fills=1, agg_chunk=4, layout=api.LAYOUT_RECORDS, fill_trees=101),
    dict(branches=2),
    dict(branches=3, fill_trees=53),
    dict(branches=4, agg_chunk=4),
]


@pytest.mark.parametrize("sched", SCHEDULES, ids=[json.dumps(s) for s in SCHEDULES])
def test_plan_schedules_bit_identical(batch, sched):
    """Every schedule, executed twice on one plan, gives the one-shot call's results."""
    mem, graphs, probs, diags, counts, reps = batch
    say("plan", sched)
    plan = api.BatchPlan(graphs, probs, ws=api.Workspace(graphs[0].row_ptr.device), schedule=api.Schedule(**sched))
    try:
        got = plan.schedule()
        for k, v in sched.items():
            assert got[k] == v, k
        for rep in range(2):
            for d in plan.diags:
                d.fill_(float("nan"))
            plan.execute()
            r2 = plan.reports()
            _same(plan, diags, counts, reps, r2, (sched, rep), same_sampler=sched.get("layout", 0) == 0)
        if sched.get("fill_trees") == 37:
            assert r2[0]["n_batches"] >= 8
    finally:
        plan.close()


def test_graph_replays_match_eager(batch):
    """One captured execution replayed three times, with eager library work, torch work and
    host synchronisations between the replays; every replay rewrites outputs that were
    overwritten before it and equals the eager results."""
    mem, graphs, probs, diags, counts, reps = batch
    dev = graphs[0].row_ptr.device
    plan = api.BatchPlan(graphs, probs, ws=api.Workspace(dev))
    try:
        say("capture")
        plan.capture()
        other = gg.rmat(9, 8, 11)
        Go = api.Graph.from_host(other.row_ptr, other.col)
        po = api.problem(Go, pivot=-1, seed=12, tau_cap=40)
        want_o, _, _ = api.diag_lpinv_p(Go, po, ws=api.Workspace(dev))
        for k in range(3):
            for d, c in zip(plan.diags, plan.counts):
                d.fill_(-1.0)
                c.fill_(-7)
            torch.cuda.synchronize()
            say("replay", k)
            plan.replay()
            r2 = plan.reports()
            _same(plan, diags, counts, reps, r2, ("replay", k))
            assert all(r["ms_sample"] == 0.0 for r in r2)  # no timers inside a graph
            d_o, _, _ = api.diag_lpinv_p(Go, po, ws=api.Workspace(dev))  # eager work between replays
            assert torch.equal(d_o, want_o)
            x = torch.randn(4096, device=dev).sum()
            torch.cuda.synchronize()
            assert torch.isfinite(x)
        plan.execute()  # eager execution after the replays
        _same(plan, diags, counts, reps, plan.reports(), "eager after replays")
    finally:
        plan.close()


def test_plan_outlives_its_graphs(batch):
    """A plan is not destroyed while a graph captured from it is alive (the graph uses its memory)."""
    mem, graphs, probs, diags, counts, reps = batch
    plan = api.BatchPlan(graphs[:3], probs[:3], ws=api.Workspace(graphs[0].row_ptr.device))
    plan.capture()
    rc = api.lib().ustd_batch_plan_destroy(plan._h)
    assert rc == api.EINVAL
    plan.replay()  # still valid
    r2 = plan.reports()
    for i in range(3):
        assert torch.equal(plan.counts[i], counts[i]), i
    plan.close()  # the graph first, then the plan


def test_graph_refuses_host_driven_solve(batch):
    mem, graphs, probs, diags, counts, reps = batch
    probs2 = list(probs)
    probs2[1] = api.with_engine(probs[1], api.ENGINE_MULTI)
    plan = api.BatchPlan(graphs, probs2, ws=api.Workspace(graphs[0].row_ptr.device))
    try:
        with pytest.raises(api.UstdError) as e:
            plan.capture()
        assert e.value.status == api.EINVAL and "problem 1" in str(e.value)
        plan.execute()  # eager execution drives that solve from the host
        r2 = plan.reports()
        for i in range(len(diags)):
            assert torch.equal(plan.counts[i], counts[i]), i
            assert r2[i]["walk_steps"] == reps[i]["walk_steps"], i
            assert r2[i]["solve_relres"] <= 1e-12, i
    finally:
        plan.close()


def test_autotune_cache_round_trip(batch, tmp_path):
    mem, graphs, probs, diags, counts, reps = batch
    small_g, small_p = graphs[:4], probs[:4]
    path = str(tmp_path / "tune.json")
    ws = api.Workspace(graphs[0].row_ptr.device)
    say("autotune")
    s1, ms1, hit1 = api.batch_autotune(small_g, small_p, ws=ws, cache_path=path)
    assert not hit1 and ms1 > 0
    entries = json.load(open(path))
    assert len(entries) == 1
    (key, val), = entries.items()
    assert key.endswith("-graph")
    assert val["group_fills"] == s1.group_fills and val["fill_trees"] == s1.fill_trees
    assert val["branches"] == s1.branches
    s2, ms2, hit2 = api.batch_autotune(small_g, small_p, ws=ws, cache_path=path)
    assert hit2 and s2.as_dict() == s1.as_dict() and abs(ms2 - ms1) < 1e-3 + 1e-6 * ms1
    s3, _, hit3 = api.batch_autotune(small_g, small_p, ws=ws, cache_path=path, graph=False)  # its own entry
    assert not hit3 and len(json.load(open(path))) == 2
    plan = api.BatchPlan(small_g, small_p, ws=ws, schedule=s1)
    try:
        plan.execute()
        r2 = plan.reports()
        for i in range(4):
            assert torch.equal(plan.counts[i], counts[i]) and torch.equal(plan.diags[i], diags[i]), i
            assert r2[i]["walk_steps"] == reps[i]["walk_steps"], i
    finally:
        plan.close()
