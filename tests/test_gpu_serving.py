"""The continuous-batching server: each query's result is the same alone
(bc_compute on its own) and in a concurrent mix, within relative 1e-9;
admission by HBM footprint queues or rejects; errors stay per query."""
import sys
import threading

import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def bcm():
    import paper_1602_00963_amd as m
    m.lib()
    return m


@pytest.fixture(scope="module")
def ctx(bcm):
    c = bcm.Context(0)
    yield c
    c.close()


def alone(bcm, G, S):
    G.reset()
    G.compute(S, mode="batched", batch=256)
    return G.scores()


def test_mix_equals_alone(bcm, ctx):
    graphs = [gg.rmat(10, 8, 101), gg.rmat(11, 16, 102), gg.road_grid(40, 30, 0.05, 0.01, 3)]
    Gs = [bcm.Graph(ctx, g) for g in graphs]
    rng = np.random.default_rng(5)
    queries = []
    for i in range(14):
        gi = i % len(graphs)
        cand = graphs[gi].non_isolated()
        k = int(rng.integers(20, min(700, len(cand))))
        queries.append((gi, gg.sample(cand, k, 1000 + i)))
    say("case serving mix: submit", len(queries))
    srv = bcm.Server(ctx, max_inflight=3, batch=256)
    tickets = [srv.submit(Gs[gi], S) for gi, S in queries]
    stats = [srv.wait(t) for t in tickets]
    srv.close()
    for (gi, S), t, st in zip(queries, tickets, stats):
        ref = alone(bcm, Gs[gi], S)
        ok = oracle.close(t.out, ref, 1e-9)
        assert ok.all(), (gi, len(S), np.nonzero(~ok)[0][:5])
        assert st["latency_ms"] >= 0 and st["sources"] == len(S)
    # two queries against the oracle directly
    for (gi, S), t in list(zip(queries, tickets))[:2]:
        ref, _ = oracle.bc(graphs[gi], S)
        assert oracle.close(t.out, ref, 1e-9).all()
    for G in Gs:
        G.close()


def test_serving_long_diameter_graph(bcm, ctx):
    """A road-like strip (hundreds of levels: the server runs it one source
    per workgroup) served beside an R-MAT graph (batched): every query equals
    the oracle, and on an 80 x 80 lattice (most counts wrap 64 bits) the jobs
    after the first exact-count probe go to extended counts directly."""
    graphs = [gg.road_grid(300, 4, 0.05, 0.01, 3), gg.rmat(10, 8, 101), gg.full_grid(80, 80)]
    Gs = [bcm.Graph(ctx, g) for g in graphs]
    assert Gs[0].stats()["bfs_depth"] > 64 and Gs[2].stats()["bfs_depth"] > 64 and Gs[1].stats()["bfs_depth"] <= 64
    rng = np.random.default_rng(9)
    queries = []
    for i in range(12):
        gi = i % len(graphs)
        cand = graphs[gi].non_isolated()
        k = int(rng.integers(30, min(400, len(cand))))
        queries.append((gi, gg.sample(cand, k, 3000 + i)))
    say("case serving long diameter: submit", len(queries))
    srv = bcm.Server(ctx, max_inflight=3, batch=256)
    tickets = [srv.submit(Gs[gi], S) for gi, S in queries]
    for t in tickets:
        srv.wait(t)
    srv.close()
    for (gi, S), t in zip(queries, tickets):
        ref, _ = oracle.bc(graphs[gi], S, nthreads=4)
        ok = oracle.close(t.out, ref, 1e-9)
        assert ok.all(), (gi, len(S), np.nonzero(~ok)[0][:5])
    for G in Gs:
        G.close()


def test_submit_from_threads(bcm, ctx):
    g = gg.rmat(10, 16, 7)
    G = bcm.Graph(ctx, g)
    srv = bcm.Server(ctx, max_inflight=4, batch=128)
    cand = g.non_isolated()
    subsets = [gg.sample(cand, 64 + 37 * i, 200 + i) for i in range(8)]
    results = [None] * len(subsets)

    def run(i):
        t = srv.submit(G, subsets[i])
        srv.wait(t)
        results[i] = t.out

    th = [threading.Thread(target=run, args=(i,)) for i in range(len(subsets))]
    for t in th:
        t.start()
    for t in th:
        t.join()
    srv.close()
    for S, r in zip(subsets, results):
        ref, _ = oracle.bc(g, S)
        assert oracle.close(r, ref, 1e-9).all()
    G.close()


def test_admission_budget_and_rejection(bcm, ctx):
    g_small = gg.rmat(9, 8, 3)
    g_big = gg.rmat(13, 16, 4)
    Gs, Gb = bcm.Graph(ctx, g_small), bcm.Graph(ctx, g_big)
    ws_small = Gs.workspace_size(mode="batched", batch=64)
    ws_big = Gb.workspace_size(mode="batched", batch=64)
    assert ws_big > 2 * ws_small
    # budget fits the small graph's worst-case workspace (the server sizes its
    # level lists for n * batch entries, at most twice the default) plus a
    # few result arrays, not the 16x larger graph's
    budget = 3 * ws_small + 64 * g_small.n * 8
    assert ws_big > budget
    srv = bcm.Server(ctx, hbm_budget_bytes=budget, max_inflight=2, batch=64)
    S = gg.sample(g_small.non_isolated(), 100, 3)
    tk = [srv.submit(Gs, S) for _ in range(6)]
    tb = srv.submit(Gb, gg.sample(g_big.non_isolated(), 10, 4))
    with pytest.raises(bcm.BCError) as e:
        srv.wait(tb)
    assert e.value.status == 8  # BC_E_REJECTED
    ref, _ = oracle.bc(g_small, S)
    for t in tk:
        srv.wait(t)
        assert oracle.close(t.out, ref, 1e-9).all()
    srv.close()
    Gs.close()
    Gb.close()


def test_bad_query_does_not_disturb_others(bcm, ctx):
    g = gg.rmat(9, 8, 11)
    G = bcm.Graph(ctx, g)
    srv = bcm.Server(ctx, max_inflight=2, batch=64)
    with pytest.raises(bcm.BCError):
        srv.submit(G, np.array([0, g.n + 5], dtype=np.int32))
    S = gg.sample(g.non_isolated(), 50, 1)
    t = srv.submit(G, S)
    srv.wait(t)
    ref, _ = oracle.bc(g, S)
    assert oracle.close(t.out, ref, 1e-9).all()
    empty = srv.submit(G, np.array([], dtype=np.int32))
    srv.wait(empty)
    assert not empty.out.any()
    srv.close()
    G.close()


def _server_ws_bytes(bcm, ctx, G, g, batch):
    """Device bytes the server holds for one batch on G: a probe server runs
    one query, then its held bytes are the workspace plus the pooled
    result array."""
    srv = bcm.Server(ctx, max_inflight=1, batch=batch)
    t = srv.submit(G, gg.sample(g.non_isolated(), 8, 1))
    srv.wait(t, timeout_us=120_000_000)
    held = srv.stats()["held_bytes"]
    srv.close()
    return held - 8 * g.n


def test_idle_workspaces_do_not_block_admission(bcm, ctx):
    """Two workers cache workspaces for two small graphs; the budget is just
    big enough for a larger graph's query alone.  Its query must be admitted
    (idle workspaces are given back) and finish: a regression would time out
    instead of hanging the test."""
    ga, gb, gc = gg.rmat(10, 8, 21), gg.rmat(10, 8, 22), gg.rmat(12, 8, 23)
    Ga, Gb, Gc = (bcm.Graph(ctx, g) for g in (ga, gb, gc))
    wa = _server_ws_bytes(bcm, ctx, Ga, ga, 64)
    wb = _server_ws_bytes(bcm, ctx, Gb, gb, 64)
    wc = _server_ws_bytes(bcm, ctx, Gc, gc, 64)
    assert wc > wa + wb
    budget = wc + 8 * gc.n + 8 * (ga.n + gb.n)  # fits c alone, not next to a's and b's workspaces
    assert budget < wa + wb + wc
    say("case idle workspaces: budget", budget, "ws", wa, wb, wc)
    srv = bcm.Server(ctx, hbm_budget_bytes=budget, max_inflight=2, batch=64)
    Sa, Sb = gg.sample(ga.non_isolated(), 300, 1), gg.sample(gb.non_isolated(), 300, 2)
    ta, tb = srv.submit(Ga, Sa), srv.submit(Gb, Sb)
    srv.wait(ta, timeout_us=120_000_000)
    srv.wait(tb, timeout_us=120_000_000)
    Sc = gg.sample(gc.non_isolated(), 200, 3)
    tc = srv.submit(Gc, Sc)
    srv.wait(tc, timeout_us=120_000_000)
    st = srv.stats()
    srv.close()
    assert st["held_bytes"] <= budget
    for g, S, t in ((ga, Sa, ta), (gb, Sb, tb), (gc, Sc, tc)):
        ref, _ = oracle.bc(g, S)
        assert oracle.close(t.out, ref, 1e-9).all()
    for G in (Ga, Gb, Gc):
        G.close()


def test_batches_run_concurrently(bcm, ctx):
    """Queries on four graphs submitted together run as concurrent batches
    (each on one share of the device while others wait); results equal each
    query alone."""
    graphs = [gg.rmat(12, 16, 300 + i) for i in range(4)]
    Gs = [bcm.Graph(ctx, g) for g in graphs]
    qs = [(i, gg.sample(graphs[i].non_isolated(), 768, 40 + i)) for i in range(4)] * 2
    say("case concurrent batches")
    srv = bcm.Server(ctx, max_inflight=4, batch=256)
    tickets = [srv.submit(Gs[i], S) for i, S in qs]
    for t in tickets:
        srv.wait(t, timeout_us=300_000_000)
    st = srv.stats()
    srv.close()
    say("server stats", st)
    assert st["workers"] == 4 and st["grid_workgroups"] * 4 <= 256 * 4
    assert st["max_inflight_seen"] >= 2
    assert st["mean_inflight"] > 1.0
    for (i, S), t in zip(qs, tickets):
        ref = alone(bcm, Gs[i], S)
        assert oracle.close(t.out, ref, 1e-9).all()
    for G in Gs:
        G.close()


def test_lone_query_takes_free_shares(bcm, ctx):
    """A query alone on the server runs its batches on every free share of
    the device but one; queries arriving meanwhile start on the share left
    free, and every result equals the query alone."""
    big = gg.rmat(14, 16, 77)
    small = gg.rmat(11, 8, 78)
    Gb, Gs = bcm.Graph(ctx, big), bcm.Graph(ctx, small)
    Sb = gg.sample(big.non_isolated(), 2048, 3)
    srv = bcm.Server(ctx, max_inflight=4, batch=128)
    say("case lone query: alone")
    t = srv.submit(Gb, Sb)
    srv.wait(t, timeout_us=300_000_000)
    st = srv.stats()
    say("server stats", st)
    assert st["wide_batches"] == st["batches"] == 16
    assert st["mean_shares"] == 3.0
    assert oracle.close(t.out, alone(bcm, Gb, Sb), 1e-9).all()
    say("case lone query: with arrivals")
    t1 = srv.submit(Gb, Sb)
    small_q = [(gg.sample(small.non_isolated(), 200, 10 + i)) for i in range(6)]
    ts = [srv.submit(Gs, S) for S in small_q]
    for x in [t1] + ts:
        srv.wait(x, timeout_us=300_000_000)
    st = srv.stats()
    say("server stats", st)
    srv.close()
    assert 1.0 < st["mean_shares"] <= 3.0
    assert oracle.close(t1.out, alone(bcm, Gb, Sb), 1e-9).all()
    for S, x in zip(small_q, ts):
        ref, _ = oracle.bc(small, S)
        assert oracle.close(x.out, ref, 1e-9).all()
    Gb.close()
    Gs.close()


@pytest.mark.parametrize("prune", [True, "trees"], ids=["one-round", "iterated"])
def test_server_deg1_subsets(bcm, ctx, prune):
    """Queries on a pruned graph use the 1-degree reduction (one round, or
    iterated until no tree is left) for their source subsets (pendants, tree
    vertices, hubs, ends of 2-vertex components among them); each result
    equals the unpruned oracle on the same subset, alone and mixed."""
    g = gg.disjoint_union(gg.attach_trees(gg.rmat_with_pendants(11, 8, 3, 0.3, 33), [5, 9, 2, 17], 4),
                          gg.star(9), gg.path(2), gg.path(3))
    G = bcm.Graph(ctx, g, prune=prune)
    assert G.stats()["pendants" if prune is True else "tree_vertices"] > 100
    rng = np.random.default_rng(9)
    every = np.arange(g.n, dtype=np.int32)
    subsets = [gg.sample(every, int(rng.integers(50, 900)), 60 + i) for i in range(6)]
    subsets.append(np.arange(g.n - 15, g.n, dtype=np.int32))  # the star, K2 and the short path
    say("case server deg1")
    srv = bcm.Server(ctx, max_inflight=2, batch=128, deg1=True)
    tickets = [srv.submit(G, S) for S in subsets]
    for t in tickets:
        srv.wait(t, timeout_us=300_000_000)
    srv.close()
    for S, t in zip(subsets, tickets):
        ref, _ = oracle.bc(g, S)
        assert oracle.close(t.out, ref, 1e-9).all(), len(S)
        G.reset()
        G.compute(S, mode="batched", batch=128, deg1=True)
        assert oracle.close(t.out, G.scores(), 1e-9).all()
    G.close()
