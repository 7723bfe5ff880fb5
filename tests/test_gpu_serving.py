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
