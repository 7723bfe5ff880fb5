"""GPU parity: the HIP library against the CPU oracle, through the C ABI.

Bar: distances and uint64 path counts bit-exact; the set of sources whose
uint64 count wraps identical to the oracle's; dependencies and scores within
relative 1e-9 (|a-b| <= 1e-9 max(|a|,|b|), exact where either is 0).
"""
import math
import sys

import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu

REL = 1e-9


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


def assert_close(got, ref, rel=REL, what=""):
    ok = oracle.close(got, ref, rel)
    if not ok.all():
        bad = np.nonzero(~ok)[0][:8]
        raise AssertionError(f"{what}: {int((~ok).sum())} mismatches, e.g. at {bad}: {np.asarray(got)[bad]} vs "
                             f"{np.asarray(ref)[bad]}")


def run_bc(bcm, ctx, g, sources=None, prune=False, **opts):
    G = bcm.Graph(ctx, g, prune=prune)
    st = G.compute(sources, **opts)
    out = G.scores()
    G.close()
    return out, st


MODES = [dict(mode="plain"), dict(mode="batched", batch=64), dict(mode="batched", batch=128),
         dict(mode="batched", batch=256), dict(mode="batched", batch=192), dict(mode="batched", batch=1024)]
MODE_IDS = ["plain", "b64", "b128", "b256", "b192", "b1024"]


@pytest.mark.parametrize("opts", MODES, ids=MODE_IDS)
def test_rmat_scale10_all_sources(bcm, ctx, opts):
    """The small R-MAT workload (scale 10, EF 16): every source."""
    g = gg.workload_rmat10()
    say("case rmat10 all sources", opts)
    ref, _ = oracle.bc(g, nthreads=4)
    got, st = run_bc(bcm, ctx, g, **opts)
    assert_close(got, ref, what=str(opts))
    assert st["sources"] == int((g.degrees() > 0).sum())


@pytest.mark.parametrize("opts", MODES, ids=MODE_IDS)
def test_traces_bit_exact(bcm, ctx, opts):
    """d and sigma bit-exact, delta within tolerance, for sampled sources of a
    graph spanning several work units per vertex (hubs beyond 256 edges)."""
    g = gg.rmat(12, 16, 21)
    assert g.degrees().max() > 3 * 256
    S = gg.sample(g.non_isolated(), 80, 3)
    say("case traces rmat12", opts)
    tr = bcm.Graph(ctx, g).trace(S, **opts)
    for i, s in enumerate(S):
        o = oracle.source(g, s)
        assert not o["overflow"] and not tr["overflow"][i]
        assert np.array_equal(tr["d"][i], o["d"]), f"d differs for source {s}"
        assert np.array_equal(tr["sigma"][i], o["sigma"]), f"sigma differs for source {s}"
        dl = o["delta"].copy()
        dl[s] = 0.0
        assert_close(tr["delta"][i], dl, what=f"delta source {s}")


@pytest.mark.parametrize("opts", MODES, ids=MODE_IDS)
def test_closed_forms(bcm, ctx, opts):
    for g, expect in [
        (gg.star(40), lambda n: np.r_[(n - 1) * (n - 2) / 2, np.zeros(n - 1)]),
        (gg.path(70), lambda n: np.array([i * (n - 1 - i) for i in range(n)], dtype=float)),
        (gg.cycle(65), lambda n: np.full(n, (n - 1) * (n - 3) / 8)),
        (gg.cycle(64), lambda n: np.full(n, (n - 2) ** 2 / 8)),
        (gg.complete(30), lambda n: np.zeros(n)),
        (gg.hypercube(9), lambda n: np.full(n, (9 * 2 ** 8 - 2 ** 9 + 1) / 2)),
    ]:
        say("case closed form", g.name, opts)
        got, _ = run_bc(bcm, ctx, g, **opts)
        assert_close(got / 2, expect(g.n), what=f"{g.name} {opts}")


@pytest.mark.parametrize("opts", MODES[:2], ids=MODE_IDS[:2])
def test_overflow_sources_and_extended_counts(bcm, ctx, opts):
    """A 40 x 40 lattice: sources near a corner wrap uint64 (C(78,39) >
    2^64), central ones do not.  The wrapped set must equal the oracle's,
    d stays exact, extended counts match the long-double oracle, and scores
    (computed with the extended rerun) match."""
    g = gg.full_grid(40, 40)
    S = np.array([0, 39, 1599, 20 * 40 + 20, 5 * 40 + 7, 19 * 40 + 21, 1560], dtype=np.int32)
    say("case overflow lattice", opts)
    tr = bcm.Graph(ctx, g).trace(S, **opts)
    for i, s in enumerate(S):
        o = oracle.source(g, s)
        assert bool(tr["overflow"][i]) == o["overflow"], f"overflow flag differs for {s}"
        assert np.array_equal(tr["d"][i], o["d"])
        if o["overflow"]:
            ext = np.ldexp(tr["sigma_mant"][i], tr["sigma_exp"][i])
            ref = o["sigma_ld"].astype(np.float64)
            assert_close(ext, ref, 1e-12, what=f"extended sigma {s}")
        else:
            assert np.array_equal(tr["sigma"][i], o["sigma"])
        dl = o["delta"].copy()
        dl[s] = 0.0
        assert_close(tr["delta"][i], dl, what=f"delta {s}")
    ref, ovf = oracle.bc(g, S)
    assert ovf.sum() >= 3
    got, st = run_bc(bcm, ctx, g, S, **opts)
    assert st["overflowed"] == int(ovf.sum())
    assert st["rerun_extended"] == int(ovf.sum())
    assert_close(got, ref, what="lattice scores")


def test_layered_chain_overflow_exact_boundary(bcm, ctx):
    """16 complete bipartite layers of width 16 stay exact; 17 wrap."""
    for layers, wraps in [(16, False), (17, True)]:
        g = gg.layered_chain(16, layers)
        say("case chain", layers)
        for opts in MODES[:2]:
            tr = bcm.Graph(ctx, g).trace(np.array([0], np.int32), **opts)
            assert bool(tr["overflow"][0]) == wraps
            if not wraps:
                assert int(tr["sigma"][0][1 + 15 * 16]) == 16 ** 15


@pytest.mark.parametrize("opts", MODES[:2] + [MODES[3]], ids=["plain", "b64", "b256"])
def test_extended_mode_everywhere(bcm, ctx, opts):
    """Forcing the extended form on a graph without wrap: counts below 2^53
    are exact in it, scores match."""
    g = gg.rmat(10, 8, 4)
    say("case extended everywhere", opts)
    ref, _ = oracle.bc(g)
    got, _ = run_bc(bcm, ctx, g, sigma="extended", **opts)
    assert_close(got, ref, what="extended scores")
    S = gg.sample(g.non_isolated(), 20, 9)
    tr = bcm.Graph(ctx, g).trace(S, sigma="extended", **opts)
    for i, s in enumerate(S):
        o = oracle.source(g, s)
        assert np.array_equal(tr["d"][i], o["d"])
        assert np.array_equal(np.ldexp(tr["sigma_mant"][i], tr["sigma_exp"][i]), o["sigma"].astype(np.float64))


@pytest.mark.parametrize("opts", [dict(mode="plain"), dict(mode="batched", batch=64),
                                  dict(mode="batched", batch=256)], ids=["plain", "b64", "b256"])
def test_degree1_pruning_equals_unpruned(bcm, ctx, opts):
    """The 1-degree reduction gives the unpruned scores: all sources and a
    subset containing pendants, hubs, and ends of 2-vertex components."""
    g = gg.disjoint_union(gg.rmat_with_pendants(11, 8, 3, 0.3, 33), gg.star(9), gg.path(2), gg.path(3),
                          gg.cycle(5))
    say("case deg1", opts)
    ref, _ = oracle.bc(g)
    got, st = run_bc(bcm, ctx, g, prune=True, deg1=True, **opts)
    assert_close(got, ref, what="pruned all")
    assert st["traversed"] < st["sources"]
    S = gg.sample(np.arange(g.n, dtype=np.int32), 500, 4)
    ref_s, _ = oracle.bc(g, S)
    got_s, _ = run_bc(bcm, ctx, g, S, prune=True, deg1=True, **opts)
    assert_close(got_s, ref_s, what="pruned subset")


@pytest.mark.parametrize("k", [64, 100], ids=["k64", "k100_ragged"])
def test_plain_hip_graph_replay(bcm, ctx, k):
    """Per-source launches replayed from a HIP graph (each launch takes the
    next source of a device list) give the scores of single launches bit for
    bit, over every source of an R-MAT graph (a ragged remainder with k =
    100), twice in a row on the same graph, and the oracle's scores."""
    g = gg.rmat(11, 8, 12)
    say("case plain graph replay", k)
    ref, _ = oracle.bc(g)
    G = bcm.Graph(ctx, g)
    st1 = G.compute(None, mode="plain")
    direct = G.scores()
    G.reset()
    st2 = G.compute(None, mode="plain", graph_launches=k)
    replayed = G.scores()
    assert np.array_equal(replayed, direct)
    assert st2["launches"] == st1["launches"] == st1["traversed"]
    assert_close(replayed, ref, what="replayed scores")
    # a second call on the same graph with fewer sources, then with fewer
    # sources than one replay holds (single launches)
    S = gg.sample(g.non_isolated(), 3 * k + 7, 5)
    for src in (S, S[:k - 1]):
        G.reset()
        G.compute(src, mode="plain")
        a = G.scores()
        G.reset()
        G.compute(src, mode="plain", graph_launches=k)
        assert np.array_equal(G.scores(), a)
        ref_s, _ = oracle.bc(g, src)
        assert_close(G.scores(), ref_s, what=f"replayed subset of {len(src)}")
    G.close()


def test_plain_hip_graph_pruned_and_wrapping(bcm, ctx):
    """Replayed launches carry the 1-degree reduction's folded sources and
    subtree terms, and the extended rerun of wrapping sources."""
    g = gg.disjoint_union(gg.rmat_with_pendants(10, 8, 3, 0.3, 33), gg.star(9), gg.path(2), gg.path(3))
    say("case plain graph replay pruned")
    ref, _ = oracle.bc(g)
    a, _ = run_bc(bcm, ctx, g, prune=True, deg1=True, mode="plain")
    b, st = run_bc(bcm, ctx, g, prune=True, deg1=True, mode="plain", graph_launches=32)
    assert np.array_equal(a, b)
    assert_close(b, ref, what="replayed pruned")
    assert st["traversed"] < st["sources"]
    # a 40 x 40 lattice: sources near the corners wrap uint64 and rerun
    # extended, more of them than one replay holds
    g = gg.full_grid(40, 40)
    S = np.array([r * 40 + c for r in range(6) for c in range(6)] + [20 * 40 + 20, 19 * 40 + 21], np.int32)
    say("case plain graph replay wrapping")
    ref, ovf = oracle.bc(g, S)
    assert ovf.sum() >= 16
    a, _ = run_bc(bcm, ctx, g, S, mode="plain")
    b, st = run_bc(bcm, ctx, g, S, mode="plain", graph_launches=8)
    assert st["rerun_extended"] == int(ovf.sum())
    assert np.array_equal(a, b)
    assert_close(b, ref, what="replayed wrapping")


def test_plain_hip_graph_option_checks(bcm, ctx):
    g = gg.rmat(8, 8, 2)
    G = bcm.Graph(ctx, g)
    for opts in (dict(mode="plain", graph_launches=-1), dict(mode="batched", batch=64, graph_launches=8)):
        with pytest.raises(bcm.BCError):
            G.compute(None, **opts)
    with pytest.raises(bcm.BCError):
        G.compute_noalloc(None, mode="plain", graph_launches=8)
    G.close()


def tree_heavy_graph():
    return gg.disjoint_union(gg.attach_trees(gg.rmat(10, 4, 21), [1, 1, 2, 3, 5, 8, 13, 30, 60, 4, 4, 1, 1, 2], 7),
                             gg.random_tree(40, 3), gg.path(2), gg.star(6),
                             gg.attach_trees(gg.cycle(9), [10, 3], 2), gg.path(1))


@pytest.mark.parametrize("opts", [dict(mode="plain"), dict(mode="batched", batch=64), dict(mode="batched", batch=256),
                                  dict(mode="batched", batch=128, deg2=True)],
                         ids=["plain", "b64", "b256", "b128-deg2"])
def test_tree_reduction_equals_unpruned(bcm, ctx, opts):
    """The 1-degree reduction iterated until no degree-1 vertex is left (every
    hanging tree folded into its attachment vertex, tree components scored in
    closed form) gives the unpruned scores: all sources, and subsets holding
    tree vertices at every depth, attachment vertices and tree components."""
    g = tree_heavy_graph()
    say("case trees", opts)
    ref, _ = oracle.bc(g)
    G = bcm.Graph(ctx, g, prune="trees")
    assert G.stats()["tree_vertices"] > 150
    st = G.compute(None, deg1=True, **opts)
    assert_close(G.scores(), ref, what="trees all")
    assert st["traversed"] < st["sources"] - 150
    rng = np.random.default_rng(3)
    for t in range(3):
        S = rng.integers(0, g.n, size=int(rng.integers(50, 600))).astype(np.int32)
        G.reset()
        G.compute(S, deg1=True, **opts)
        ref_s, _ = oracle.bc(g, S)
        assert_close(G.scores(), ref_s, what=f"trees subset {t}")
    # sources only inside tree components: no sweep at all
    S = np.arange(g.n - 50, g.n - 10, dtype=np.int32)
    G.reset()
    G.compute(S, deg1=True, **opts)
    ref_s, _ = oracle.bc(g, S)
    assert_close(G.scores(), ref_s, what="tree components")
    G.close()


def test_autotune_shared_by_graph_shape(bcm, ctx):
    """A tuning is kept by graph shape in the context: a graph of the same
    shape loaded afterwards starts from it (batch = 0 uses the tuned batch),
    a graph of another shape does not; scores stay the oracle's."""
    g = gg.rmat(11, 16, 12)
    S = gg.sample(g.non_isolated(), 300, 5)
    A = bcm.Graph(ctx, g)
    tuned = A.autotune(S, budget_ms=20000)
    B = bcm.Graph(ctx, g)  # the same shape, a new graph
    C = bcm.Graph(ctx, gg.road_grid(40, 30, 0.05, 0.01, 3))
    assert A.stats()["tuned_batch"] == tuned["batch"]
    assert B.stats()["tuned_batch"] == tuned["batch"]
    assert C.stats()["tuned_batch"] == 0
    B.compute(S, batch=0)
    ref, _ = oracle.bc(g, S)
    assert_close(B.scores(), ref, what="tuned by shape")
    for G in (A, B, C):
        G.close()


@pytest.mark.parametrize("batch", [64, 256])
def test_degree2_derivation_equals_unpruned(bcm, ctx, batch):
    """2-degree vertices whose neighbours are sources of the same batch get
    their sweep derived (Lemma 1, Eq. (6)); scores unchanged."""
    g = gg.disjoint_union(gg.road_grid(24, 20, 0.2, 0.01, 7), gg.cycle(9), gg.path(7))
    say("case deg2", batch)
    ref, _ = oracle.bc(g)
    got, st = run_bc(bcm, ctx, g, mode="batched", batch=batch, deg2=True)
    assert st["derived"] > 10
    assert_close(got, ref, what="deg2")
    gp = gg.rmat_with_pendants(10, 4, 5, 0.3, 8)
    ref, _ = oracle.bc(gp)
    got, st = run_bc(bcm, ctx, gp, prune=True, mode="batched", batch=batch, deg1=True, deg2=True)
    assert st["derived"] > 0
    assert_close(got, ref, what="deg1+deg2")


@pytest.mark.parametrize("opts", [dict(mode="plain"), dict(mode="batched", batch=64),
                                  dict(mode="batched", batch=256), dict(mode="batched", batch=256, sigma="extended")],
                         ids=["plain", "b64", "b256", "b256-ext"])
def test_bottom_up_levels_forced(bcm, ctx, opts):
    """Direction switching: with a large threshold every level after the
    first few is pulled bottom-up; d and sigma stay bit-exact and scores
    match the oracle on a dense R-MAT graph and on a lattice with pendants
    (pruned)."""
    g = gg.rmat(11, 16, 31)
    S = gg.sample(g.non_isolated(), 300, 32)
    say("case bottom-up", opts)
    ref, _ = oracle.bc(g, S)
    got, st = run_bc(bcm, ctx, g, S, alpha=1000.0, **opts)
    assert st["bottom_up_levels"] > 0
    assert_close(got, ref, what=f"bottom-up {opts}")
    if opts.get("sigma") != "extended":
        tr = bcm.Graph(ctx, g).trace(S[:64], alpha=1000.0, **opts)
        for i, s in enumerate(S[:64]):
            o = oracle.source(g, s)
            assert np.array_equal(tr["d"][i], o["d"]), f"d differs for source {s}"
            assert np.array_equal(tr["sigma"][i], o["sigma"]), f"sigma differs for source {s}"
    gl = gg.disjoint_union(gg.road_grid(28, 24, 0.05, 0.01, 33), gg.star(6))
    ref, _ = oracle.bc(gl)
    got, st = run_bc(bcm, ctx, gl, prune=True, deg1=True, alpha=1000.0, **opts)
    assert st["bottom_up_levels"] > 0
    assert_close(got, ref, what=f"bottom-up lattice {opts}")


@pytest.mark.parametrize("opts", [dict(mode="plain"), dict(mode="batched", batch=128)], ids=["plain", "b128"])
def test_bottom_up_switch_back(bcm, ctx, opts):
    """Direction switching with hysteresis: once bottom-up, a sweep stays
    bottom-up until the frontier holds fewer than n / beta vertices; levels
    and counts stay bit-exact and scores match the oracle whichever
    direction each level takes."""
    g = gg.rmat(11, 16, 41)
    S = gg.sample(g.non_isolated(), 200, 42)
    ref, _ = oracle.bc(g, S)
    say("case switch-back", opts)
    levels = {}
    for beta in (0.0, 2.0, 1000.0):
        got, st = run_bc(bcm, ctx, g, S, alpha=2.0, beta=beta, **opts)
        assert_close(got, ref, what=f"beta {beta} {opts}")
        levels[beta] = st["bottom_up_levels"]
    # beta changes the schedule (longer bottom-up runs, earlier switch back
    # on the small tail frontiers), never the results
    assert len(set(levels.values())) > 1 and min(levels.values()) > 0, levels
    tr = bcm.Graph(ctx, g).trace(S[:64], alpha=2.0, beta=1000.0, **opts)
    for i, s in enumerate(S[:64]):
        o = oracle.source(g, s)
        assert np.array_equal(tr["d"][i], o["d"]) and np.array_equal(tr["sigma"][i], o["sigma"]), s


def test_paper_mapping_mode(bcm, ctx):
    """The paper's active-edge mapping (per level a prefix sum of the
    frontier's degrees, a binary search per edge, the prefix sums reused by
    the backward sweep) gives the oracle's scores: an R-MAT graph, a
    long-diameter road-like strip, a union with isolated vertices and
    repeated sources, and a lattice whose corner counts wrap (those sources
    are rerun by the plain form in extended counts)."""
    cases = [(gg.rmat(11, 16, 5), None),
             (gg.road_grid(300, 4, 0.05, 0.01, 3), None),
             (gg.disjoint_union(gg.rmat(9, 8, 2), gg.star(7), gg.path(1), gg.cycle(6)), np.array([0, 0, 3, 512, 513, 520, 521, 5], np.int32)),
             (gg.full_grid(40, 40), np.array([0, 39, 1560, 1599, 820, 410], np.int32))]
    for g, S in cases:
        say("case plain_scan", g.name)
        ref, ovf = oracle.bc(g, S)
        got, st = run_bc(bcm, ctx, g, S, mode="plain_scan")
        assert_close(got, ref, what=f"plain_scan {g.name}")
        assert st["overflowed"] == int(ovf.sum())


def test_per_workgroup_mode(bcm, ctx):
    """One source per workgroup, hundreds of workgroups at once: the oracle's
    scores on an R-MAT graph (all sources: several sources per workgroup), a
    long-diameter road-like strip, closed forms, a union with isolated
    vertices and repeated sources, and a lattice whose corner counts wrap,
    with every count form (exact: the wrapped set is the oracle's; extended;
    auto: wrapped sources rerun extended)."""
    cases = [(gg.rmat(11, 16, 5), None),
             (gg.road_grid(300, 4, 0.05, 0.01, 3), None),
             (gg.path(70), None), (gg.cycle(65), None), (gg.star(40), None), (gg.hypercube(9), None),
             (gg.disjoint_union(gg.rmat(9, 8, 2), gg.star(7), gg.path(1), gg.cycle(6)),
              np.array([0, 0, 3, 512, 513, 520, 521, 5], np.int32))]
    for g, S in cases:
        say("case per_workgroup", g.name)
        ref, ovf = oracle.bc(g, S, nthreads=4)
        got, st = run_bc(bcm, ctx, g, S, mode="per_workgroup")
        assert_close(got, ref, what=f"per_workgroup {g.name}")
        assert st["overflowed"] == int(ovf.sum()) == 0
    g = gg.full_grid(40, 40)
    S = np.array([0, 39, 1560, 1599, 820, 410, 5 * 40 + 7, 19 * 40 + 21], np.int32)
    ref, ovf = oracle.bc(g, S)
    assert ovf.sum() > 0
    for sm in ["auto", "extended"]:
        say("case per_workgroup lattice", sm)
        got, st = run_bc(bcm, ctx, g, S, mode="per_workgroup", sigma=sm)
        assert_close(got, ref, what=f"per_workgroup lattice {sm}")
    say("case per_workgroup lattice exact")
    G = bcm.Graph(ctx, g)
    st = G.compute(S, mode="per_workgroup", sigma="exact")
    G.close()
    assert st["overflowed"] == int(ovf.sum())


def test_per_workgroup_many_sources_per_workgroup(bcm, ctx):
    """Extended counts with more than 127 sources on one workgroup (one
    workgroup per CU, 33,768 sources): the records' generation tags wrap and
    the workgroup clears its slice; scores against closed forms (a
    15-dimensional hypercube and a path of 1,000 vertices)."""
    d, p = 15, 1000
    g = gg.disjoint_union(gg.hypercube(d), gg.path(p))
    say("case per_workgroup generation wrap", g.n)
    got, st = run_bc(bcm, ctx, g, None, mode="per_workgroup", sigma="extended", grid_per_cu=1)
    assert st["traversed"] == g.n and g.n > 127 * 256
    cube = np.full(2 ** d, (d * 2 ** (d - 1) - 2 ** d + 1) / 2)
    path = np.array([i * (p - 1 - i) for i in range(p)], dtype=float)
    assert_close(got / 2, np.r_[cube, path], what="generation wrap")


def test_auto_mode_choice(bcm, ctx):
    """BC_MODE_AUTO runs a long-diameter graph (a road-like strip, about 300
    levels from its highest-degree vertex) one source per workgroup and a
    small-world graph (R-MAT, a handful of levels) batched, and both give the
    oracle's scores; with 2-degree derivation requested it stays batched."""
    for g, want in [(gg.road_grid(300, 4, 0.05, 0.01, 3), "per_workgroup"), (gg.rmat(11, 16, 5), "batched")]:
        say("case auto mode", g.name)
        S = gg.sample(g.non_isolated(), 400, 13)
        ref, _ = oracle.bc(g, S, nthreads=4)
        G = bcm.Graph(ctx, g)
        depth = G.stats()["bfs_depth"]
        st = G.compute(S, mode="auto")
        assert st["mode"] == want, (g.name, depth, st["mode"])
        assert (depth > 64) == (want == "per_workgroup"), depth
        assert_close(G.scores(), ref, what=f"auto {g.name}")
        G.reset()
        st2 = G.compute(S, mode="auto", deg2=True)
        assert st2["mode"] == "batched"
        assert_close(G.scores(), ref, what=f"auto deg2 {g.name}")
        G.close()


@pytest.mark.parametrize("prune", [True, "trees"], ids=["deg1", "trees"])
def test_per_workgroup_pruned(bcm, ctx, prune):
    """The per-workgroup mode on pruned graphs (one round of 1-degree removal,
    and the iterated tree reduction): every source, and a sampled subset that
    includes removed vertices."""
    g = gg.attach_trees(gg.rmat(11, 8, 7), [1, 1, 2, 3, 5, 9], 4)
    S = gg.sample(np.arange(g.n), 300, 9)
    for src in [None, S]:
        say("case per_workgroup pruned", prune, "all" if src is None else "sample")
        ref, _ = oracle.bc(g, src, nthreads=4)
        got, st = run_bc(bcm, ctx, g, src, prune=prune, deg1=True, mode="per_workgroup")
        assert_close(got, ref, what=f"per_workgroup prune={prune}")


def test_sources_with_repeats_and_isolated(bcm, ctx):
    g = gg.disjoint_union(gg.rmat(9, 8, 2), gg.complete(1))
    nz = g.non_isolated()
    a, b = int(nz[0]), int(nz[1])
    S = np.array([a, a, b, g.n - 1, 7, a], dtype=np.int32)
    ref, _ = oracle.bc(g, S)
    deg = g.degrees()
    for opts in MODES[:2]:
        got, st = run_bc(bcm, ctx, g, S, **opts)
        assert_close(got, ref, what=str(opts))
        assert st["sources"] == int(np.sum(deg[S] > 0))
        assert st["traversed"] == len(set(int(s) for s in S if deg[s] > 0))


@pytest.mark.parametrize("opts", MODES[:3] + [dict(mode="per_workgroup"), dict(mode="auto")],
                         ids=MODE_IDS[:3] + ["wg", "auto"])
def test_degenerate_inputs(bcm, ctx, opts):
    """One vertex, only isolated vertices, an empty source list, a 2-vertex
    component under pruning, and a ragged last batch (130 sources)."""
    say("case degenerate", opts)
    for g in [gg.complete(1), gg.disjoint_union(*[gg.complete(1) for _ in range(5)])]:
        got, st = run_bc(bcm, ctx, g, **opts)
        assert not got.any() and st["sources"] == 0
    g = gg.rmat(9, 8, 41)
    got, st = run_bc(bcm, ctx, g, np.zeros(0, dtype=np.int32), **opts)
    assert not got.any() and st["sources"] == 0 and st["traversed"] == 0
    got, st = run_bc(bcm, ctx, gg.path(2), prune=True, deg1=True, **opts)
    assert not got.any()
    S = gg.sample(g.non_isolated(), 130, 42)
    ref, _ = oracle.bc(g, S)
    got, st = run_bc(bcm, ctx, g, S, **opts)
    assert st["traversed"] == 130
    assert_close(got, ref, what=f"ragged {opts}")


def test_batched_deterministic(bcm, ctx):
    g = gg.rmat(12, 16, 5)
    G = bcm.Graph(ctx, g)
    G.compute(None, mode="batched", batch=256)
    a = G.scores()
    G.reset()
    G.compute(None, mode="batched", batch=256)
    b = G.scores()
    assert np.array_equal(a, b)
    G.close()


def test_run_stats_match_oracle_counts(bcm, ctx):
    """reached vertices, reached CSR entries and DAG edges summed over the
    sources equal the oracle's per-source counts."""
    g = gg.rmat(10, 16, 6)
    S = gg.sample(g.non_isolated(), 300, 2)
    _, _, st = oracle.bc(g, S, want_stats=True)
    for opts in MODES[:2] + [MODES[3]]:
        _, rs = run_bc(bcm, ctx, g, S, **opts)
        assert rs["reached"] == st[:, 0].sum()
        assert rs["reached_nnz"] == st[:, 1].sum()
        assert rs["dag_edges"] == st[:, 2].sum()


@pytest.mark.parametrize("batch", [256, 1024])
def test_rmat_scale16_sampled_sources(bcm, ctx, batch):
    """The scale-16 workload at full size: 1,024 sampled sources through the
    batched launch shapes (1,024 sources per launch is the benchmark's), and
    32 through plain."""
    g = gg.workload_rmat16()
    S = gg.sample(g.non_isolated(), 1024, 11)
    say("case rmat16 sampled", batch)
    ref, _ = oracle.bc(g, S, nthreads=8)
    got, _ = run_bc(bcm, ctx, g, S, mode="batched", batch=batch)
    assert_close(got, ref, what=f"rmat16 batched b{batch}")
    if batch == 256:
        ref2, _ = oracle.bc(g, S[:32], nthreads=8)
        got2, _ = run_bc(bcm, ctx, g, S[:32], mode="plain")
        assert_close(got2, ref2, what="rmat16 plain")


def test_rmat_scale20_pendants_full_size_sampled(bcm, ctx):
    """The scale-20 R-MAT graph with 30% extra pendants at full size, pruned,
    in the benchmark's launch shape (256 sources per launch): 256 sampled
    sources, pendants among them, against the unpruned oracle."""
    g = gg.workload_rmat20_pendants()
    S = gg.sample(np.arange(g.n, dtype=np.int32), 256, 21)
    deg = g.degrees()
    assert np.sum(deg[S] == 1) > 25
    say("case rmat20 pendants sampled", g.n, g.m)
    ref, _ = oracle.bc(g, S, nthreads=8)
    got, st = run_bc(bcm, ctx, g, S, prune=True, deg1=True, mode="batched", batch=256)
    assert st["traversed"] < st["sources"]
    assert_close(got, ref, what="rmat20 pendants pruned")


def test_roadlike_grid_full_size_sampled(bcm, ctx):
    """The 2048 x 2048 road-like lattice at full size: 32 sampled sources in
    automatic count form (nearly all wrap uint64 and are rerun extended);
    scores against the oracle's long-double reruns."""
    g = gg.workload_roadlike_grid()
    S = gg.sample(g.non_isolated(), 32, 23)
    say("case grid2048 sampled", g.n, g.m)
    ref, ovf = oracle.bc(g, S, nthreads=8)
    got, st = run_bc(bcm, ctx, g, S, mode="batched", batch=256)
    assert st["overflowed"] > 0 and ovf.any()
    assert_close(got, ref, what="grid2048")


def test_rmat_pendants_recipe_scale14_all_sources(bcm, ctx):
    """The scale-20 workload's recipe at scale 14 (R-MAT EF 16, seed 3, plus
    30% pendants, seed 33), every source, in the benchmark's launch shape
    (128 sources per launch, top-down only): pruned and unpruned runs both
    equal the oracle over all sources."""
    g = gg.workload_rmat20_pendants(scale=14)
    say("case rmat14 pendants all sources", g.n, g.m)
    ref, _ = oracle.bc(g, nthreads=16)
    got_p, st_p = run_bc(bcm, ctx, g, None, prune=True, deg1=True, mode="batched", batch=128, alpha=-1.0)
    got_u, st_u = run_bc(bcm, ctx, g, None, mode="batched", batch=128, alpha=-1.0)
    assert st_p["traversed"] < st_u["traversed"] and st_p["sources"] == st_u["sources"]
    assert_close(got_p, ref, what="rmat14 pendants pruned")
    assert_close(got_u, ref, what="rmat14 pendants unpruned")


def test_rmat_scale20_pendants_multi_launch(bcm, ctx):
    """The scale-20 graph with pendants, pruned, in the benchmark's tuned
    launch shape (128 sources per launch, top-down only) over several
    launches: 600 sampled sources (pendants among them) against the
    unpruned oracle."""
    g = gg.workload_rmat20_pendants()
    S = gg.sample(np.arange(g.n, dtype=np.int32), 600, 31)
    say("case rmat20 pendants multi-launch", g.n, g.m)
    ref, _ = oracle.bc(g, S, nthreads=16)
    got, st = run_bc(bcm, ctx, g, S, prune=True, deg1=True, mode="batched", batch=128, alpha=-1.0)
    assert st["launches"] >= 4, st["launches"]
    assert_close(got, ref, what="rmat20 pendants multi-launch")


def test_roadlike_grid_multi_launch_extended(bcm, ctx):
    """The 2048 x 2048 lattice in automatic count form over several launches:
    after the one-word probe nearly every source wraps, so the rest run in
    extended form with worst-case lists (four launches of up to 256
    sources); scores against the oracle's long-double reruns."""
    g = gg.workload_roadlike_grid()
    S = gg.sample(g.non_isolated(), 64 + 3 * 256 + 10, 29)
    say("case grid2048 multi-launch", g.n, g.m)
    ref, ovf = oracle.bc(g, S, nthreads=16)
    got, st = run_bc(bcm, ctx, g, S, mode="batched", batch=256)
    assert ovf.mean() > 0.5 and st["launches"] >= 5, (ovf.mean(), st["launches"])
    assert_close(got, ref, what="grid2048 multi-launch")


def test_roadlike_grid_per_workgroup_full_size(bcm, ctx):
    """The 2048 x 2048 lattice at full size in the benchmark's shape for it:
    reverse Cuthill-McKee order, one source per workgroup, automatic counts
    (a one-word probe in exact form that wraps, then extended launches, then
    the probe's sources rerun extended); scores against the oracle's
    long-double reruns."""
    g = gg.workload_roadlike_grid()
    S = gg.sample(g.non_isolated(), 64 + 300, 37)
    say("case grid2048 per_workgroup rcm", g.n, g.m)
    ref, ovf = oracle.bc(g, S, nthreads=16)
    G = bcm.Graph(ctx, g, validate=False, order="rcm")
    st = G.compute(S, mode="per_workgroup")
    got = G.scores()
    G.close()
    assert ovf.mean() > 0.5 and st["launches"] >= 3 and st["overflowed"] >= 32, (ovf.mean(), st)
    assert_close(got, ref, what="grid2048 per_workgroup")


@pytest.mark.parametrize("opts", [dict(mode="plain"), dict(mode="batched", batch=128), dict(mode="per_workgroup")],
                         ids=["plain", "b128", "wg"])
def test_rcm_vertex_order(bcm, ctx, opts):
    """Graphs loaded in reverse Cuthill-McKee order give the oracle's scores
    in caller ids: an R-MAT graph with isolated vertices, a road-like strip,
    a pruned graph with pendants, and a lattice whose corner counts wrap;
    traces of the batched form report d and sigma in caller ids."""
    for g, S, prune in [(gg.disjoint_union(gg.rmat(10, 8, 3), gg.complete(1), gg.path(5)), None, False),
                        (gg.road_grid(300, 5, 0.05, 0.01, 8), None, False),
                        (gg.add_pendants(gg.rmat(10, 8, 4), np.random.default_rng(5).integers(0, 1024, 300)), None, True),
                        (gg.full_grid(40, 40), np.array([0, 39, 1560, 1599, 820, 410], np.int32), False)]:
        say("case rcm", g.name, opts)
        ref, _ = oracle.bc(g, S, nthreads=4)
        G = bcm.Graph(ctx, g, prune=prune, order="rcm")
        G.compute(S, deg1=prune, **opts)
        assert_close(G.scores(), ref, what=f"rcm {g.name} {opts}")
        if opts["mode"] == "batched" and not prune:
            T = (S if S is not None else g.non_isolated())[:5]
            tr = G.trace(T, **opts)
            for i, s in enumerate(T):
                o = oracle.source(g, int(s))
                assert np.array_equal(tr["d"][i], o["d"]), s
                if not o["overflow"]:
                    assert np.array_equal(tr["sigma"][i], o["sigma"]), s
        G.close()


def test_degree2_derivation_extended_counts(bcm, ctx):
    """2-degree derivation on a long-diameter lattice whose counts wrap
    uint64: after the one-word probe the batches run in extended form with
    derived lanes (Eq. (6) on significand/exponent pairs); scores against
    the oracle's long-double reruns."""
    g = gg.road_grid(72, 72, 0.2, 0.0, 5)
    say("case deg2 extended", g.n, g.m)
    G = bcm.Graph(ctx, g)
    st = G.compute(None, mode="batched", batch=256, deg2=True)
    got = G.scores()
    G.close()
    ref, ovf = oracle.bc(g, nthreads=16)
    assert ovf.mean() > 0.5 and st["derived"] > 200, (ovf.mean(), st["derived"])
    assert_close(got, ref, what="deg2 extended")


@pytest.mark.parametrize("batch", [64, 256])
def test_degree2_derived_lanes_traced(bcm, ctx, batch):
    """2-degree vertices derived from their partner lanes (Lemma 1, Eq. (6))
    with the fused backward sweep: their counts and dependencies, as the
    kernel computes them, equal a BFS/Brandes sweep from the vertex itself
    (counts bit-exact, levels from the partners' levels bit-exact,
    dependencies within 1e-9)."""
    g = gg.disjoint_union(gg.road_grid(24, 20, 0.2, 0.01, 7), gg.cycle(9), gg.path(7))
    S = np.arange(g.n, dtype=np.int32)
    say("case deg2 traced", batch)
    G = bcm.Graph(ctx, g)
    st = G.compute(S, mode="batched", batch=batch, deg2=True)
    assert st["derived"] > 20
    tr = G.trace(S, mode="batched", batch=batch, deg2=True)
    G.close()
    for i, s in enumerate(S):
        o = oracle.source(g, int(s))
        assert np.array_equal(tr["d"][i], o["d"]), f"d differs for source {s}"
        if not o["overflow"]:
            assert np.array_equal(tr["sigma"][i], o["sigma"]), f"sigma differs for source {s}"
        dl = o["delta"].copy()
        dl[s] = 0.0
        assert_close(tr["delta"][i], dl, what=f"delta of source {s}")


def test_rmat_scale16_hub_sources_traced(bcm, ctx):
    """Per-source d and sigma bit-exact at full size for sources next to the
    highest-degree vertices: their adjacency lists span many work units, so
    every level combines split entries (partial sums handed between waves)
    in both sweeps; delta within 1e-9."""
    g = gg.workload_rmat16()
    rp = np.asarray(g.row_ptr)
    deg = np.diff(rp)
    hubs = np.argsort(-deg, kind="stable")[:4]
    ci = np.asarray(g.col_idx)
    near = np.unique(np.concatenate([ci[rp[h]:rp[h] + 16] for h in hubs] + [hubs]))
    S = [int(v) for v in near[:64]]
    say("case rmat16 hub trace", len(S), int(deg[hubs[0]]))
    assert deg[hubs[0]] > 4 * 256
    tr = bcm.Graph(ctx, g).trace(S, mode="batched", batch=1024)
    for i, s in enumerate(S):
        o = oracle.source(g, s)
        assert not o["overflow"] and not tr["overflow"][i]
        assert np.array_equal(tr["d"][i], o["d"]), f"d differs for source {s}"
        assert np.array_equal(tr["sigma"][i], o["sigma"]), f"sigma differs for source {s}"
        dl = o["delta"].copy()
        dl[s] = 0.0  # the source's own dependency is not part of any score
        assert_close(tr["delta"][i], dl, what=f"delta of source {s}")


@pytest.mark.parametrize("opts", [dict(mode="batched", batch=128), dict(mode="per_workgroup"),
                                  dict(mode="per_workgroup", sigma="extended")], ids=["b128", "wg", "wg_ext"])
def test_device_score_output_and_workspace(bcm, ctx, opts):
    """A caller-owned workspace of bc_workspace_size bytes (filled with
    garbage first) and a caller stream; scores written to a device tensor."""
    import torch
    g = gg.disjoint_union(gg.rmat(9, 8, 3), gg.road_grid(40, 3, 0.05, 0.01, 2))
    ref, _ = oracle.bc(g)
    G = bcm.Graph(ctx, g)
    nbytes = G.workspace_size(**opts)
    ws = torch.full((nbytes,), 0xA5, dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    G.compute(None, workspace=ws, stream=s, **opts)
    out = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    G.scores("undirected", out=out)
    assert_close(out.cpu().numpy() * 2, ref, what=f"device output {opts}")
    G.close()


def test_autotune_leaves_scores_and_results_unchanged(bcm, ctx):
    g = gg.rmat(11, 16, 12)
    G = bcm.Graph(ctx, g)
    S = gg.sample(g.non_isolated(), 300, 5)
    tuned = G.autotune(S, budget_ms=20000)
    assert tuned["batch"] in (64, 128, 256, 512, 1024) and tuned["gteps"] > 0
    assert not G.scores().any()                 # tuning used scratch scores
    G.compute(S, batch=0)                       # the tuned setting
    ref, _ = oracle.bc(g, S)
    assert_close(G.scores(), ref, what="tuned")
    G.close()


@pytest.mark.parametrize("batch", [64, 256])
def test_long_diameter_lattice_auto_mode(bcm, ctx, batch):
    """A 96 x 96 road-like lattice, every source, automatic count form: about
    90% of sources wrap uint64, so after the probe word the rest run in
    extended form with worst-case level lists; most levels carry about one
    lane per (vertex, word), so the one-lane-per-unit path does most of the
    work; scores match the oracle (long-double reruns)."""
    g = gg.road_grid(96, 96, 0.05, 0.01, 9)
    say("case lattice auto", batch)
    ref, ovf = oracle.bc(g, nthreads=8)
    assert ovf.mean() > 0.5
    got, st = run_bc(bcm, ctx, g, mode="batched", batch=batch)
    assert st["overflowed"] > 0
    assert_close(got, ref, what=f"lattice auto b{batch}")


def test_sparse_sources_on_lattice_exact(bcm, ctx):
    """Few sources far apart on a lattice small enough for exact counts:
    nearly every (vertex, word) has a single lane, so both sweeps run one
    unit per lane; d and sigma bit-exact, delta and scores within 1e-9."""
    g = gg.road_grid(30, 30, 0.05, 0.01, 4)
    S = gg.sample(g.non_isolated(), 48, 12)
    say("case sparse lattice")
    tr = bcm.Graph(ctx, g).trace(S, mode="batched", batch=64)
    for i, s in enumerate(S):
        o = oracle.source(g, s)
        assert not o["overflow"] and not tr["overflow"][i]
        assert np.array_equal(tr["d"][i], o["d"]), f"d differs for source {s}"
        assert np.array_equal(tr["sigma"][i], o["sigma"]), f"sigma differs for source {s}"
    ref, _ = oracle.bc(g, S)
    got, _ = run_bc(bcm, ctx, g, S, mode="batched", batch=64)
    assert_close(got, ref, what="sparse lattice")
