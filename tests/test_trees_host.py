"""The iterated 1-degree reduction on the host (no GPU): every removed vertex
is a cut vertex, so its closed-form score must equal plain Brandes (the
oracle) at that vertex, for all sources and for source multisets; the
folded counts and the residual graph are checked against their
definitions."""
import numpy as np
import pytest

import graphgen as gg
import oracle
import paper_1602_00963_amd as bcm


def tree_graphs():
    core = gg.rmat(8, 4, 12)
    g1 = gg.attach_trees(core, [1, 1, 2, 3, 5, 8, 13, 30, 1, 4], 3)
    g2 = gg.disjoint_union(gg.attach_trees(gg.cycle(7), [6, 1, 9, 2], 5), gg.random_tree(12, 4), gg.path(5),
                           gg.star(4), gg.path(2), gg.path(1))
    g3 = gg.attach_trees(gg.full_grid(5, 6), [20, 15, 1, 1, 1, 7], 8)
    g4 = gg.attach_trees(gg.complete(4), [40], 9)  # one deep tree
    return [g1, g2, g3, g4]


@pytest.mark.parametrize("gi", range(4))
def test_removed_vertex_scores_equal_brandes_all_sources(gi):
    g = tree_graphs()[gi]
    p = bcm.prune_trees_host(g.n, g.row_ptr, g.col_idx)
    ref, _ = oracle.bc(g)
    removed = p["kind"] == 4
    assert removed.sum() > 10
    ok = oracle.close(p["scores"][removed], ref[removed], 1e-12)
    assert ok.all(), np.nonzero(~ok)[0][:5]
    assert not p["scores"][~removed].any()


@pytest.mark.parametrize("gi", range(4))
def test_removed_vertex_scores_equal_brandes_subsets(gi):
    g = tree_graphs()[gi]
    rng = np.random.default_rng(gi)
    removed_ids = None
    for t in range(4):
        k = int(rng.integers(1, g.n))
        S = rng.integers(0, g.n, size=k).astype(np.int32)  # a multiset: repeats count twice
        p = bcm.prune_trees_host(g.n, g.row_ptr, g.col_idx, S)
        removed_ids = np.nonzero(p["kind"] == 4)[0]
        ref, _ = oracle.bc(g, S)
        ok = oracle.close(p["scores"][removed_ids], ref[removed_ids], 1e-12)
        assert ok.all(), (t, removed_ids[~ok][:5])


def test_folding_counts_and_residual_core():
    for g in tree_graphs():
        p = bcm.prune_trees_host(g.n, g.row_ptr, g.col_idx)
        kind, omega = p["kind"], p["omega"]
        kept = kind == 0
        deg = np.diff(g.row_ptr)
        # every vertex is kept, isolated, or folded into exactly one kept vertex
        # (or removed with its whole tree component)
        in_tree_comp = (kind == 4).sum() - omega[kept].sum()
        assert kept.sum() + omega[kept].sum() + in_tree_comp + (kind == 3).sum() == g.n
        assert ((kind == 3) == (deg == 0)).all()
        # the residual graph is the 2-core: every kept vertex keeps >= 2 kept neighbours
        for v in np.nonzero(kept)[0]:
            nb = g.col_idx[g.row_ptr[v]:g.row_ptr[v + 1]]
            assert (kind[nb] == 0).sum() >= 2
        assert p["residual_nnz"] == sum(int((kind[g.col_idx[g.row_ptr[v]:g.row_ptr[v + 1]]] == 0).sum())
                                        for v in np.nonzero(kept)[0])


def test_one_round_is_not_iterated():
    """A 4-vertex tree hanging from a cycle: one round folds only its
    leaves, the iterated reduction folds the whole tree."""
    g = gg.attach_trees(gg.cycle(5), [4], 1)
    one = bcm.prune_deg1_host(g.n, g.row_ptr, g.col_idx)
    it = bcm.prune_trees_host(g.n, g.row_ptr, g.col_idx)
    assert one["omega"].sum() <= it["omega"].sum() and it["omega"].sum() == 4


def test_coverage_counts():
    """Heuristics coverage (host): every non-isolated source is traversed,
    served by the 1-degree reduction or derived by the 2-degree heuristic;
    on a cycle the derived vertices are a maximum independent set (floor(n/2))
    with every derived vertex's neighbours traversed."""
    for n in (9, 10, 11, 64):
        g = gg.cycle(n)
        c = bcm.coverage_host(g.n, g.row_ptr, g.col_idx, deg2=True)
        assert c["two_degree"] == n // 2 and c["traversed"] == n - n // 2
    g = gg.disjoint_union(gg.road_grid(40, 40, 0.1, 0.01, 3), gg.star(5), gg.path(1),
                          gg.attach_trees(gg.cycle(12), [3, 4], 2))
    base = bcm.coverage_host(g.n, g.row_ptr, g.col_idx)
    assert base["traversed"] == base["sources"] == g.n - 1  # one isolated vertex
    for prune in (True, "trees"):
        for deg2 in (False, True):
            c = bcm.coverage_host(g.n, g.row_ptr, g.col_idx, prune=prune, deg1=True, deg2=deg2)
            assert c["sources"] == c["traversed"] + c["one_degree"] + c["two_degree"]
            assert c["one_degree"] > 0 and (c["two_degree"] > 0) == deg2
            assert c["two_degree"] <= c["deg2_candidates"]
    it = bcm.coverage_host(g.n, g.row_ptr, g.col_idx, prune="trees", deg1=True)
    one = bcm.coverage_host(g.n, g.row_ptr, g.col_idx, prune=True, deg1=True)
    assert it["one_degree"] > one["one_degree"]
