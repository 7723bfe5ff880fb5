"""Pins for the CPU oracle: each test checks it against something other than
itself -- exact brute force, an independent O(n^3) method, networkx, closed
forms, path-count identities and invariants of betweenness.

Convention: oracle scores are RAW (ordered pairs, Eq. (3)); closed forms and
networkx use the undirected convention, RAW / 2.
"""
import math
from fractions import Fraction

import networkx as nx
import numpy as np
import pytest

import graphgen as gg
import oracle
from oracle import brute


def undirected(g, sources=None):
    raw, ovf = oracle.bc(g, sources)
    return raw / 2.0, ovf


def nx_graph(g):
    G = nx.Graph()
    G.add_nodes_from(range(g.n))
    u, v = g.edges()
    G.add_edges_from(zip(u.tolist(), v.tolist()))
    return G


def assert_close(a, b, rel=1e-9):
    ok = oracle.close(a, b, rel)
    assert ok.all(), f"mismatch at {np.nonzero(~ok)[0][:10]}: {np.asarray(a)[~ok][:5]} vs {np.asarray(b)[~ok][:5]}"


# ----------------------------------------------------------------- brute force

SMALL = [gg.erdos_renyi(n, p, seed) for seed, (n, p) in enumerate(
    [(6, 0.5), (7, 0.4), (8, 0.35), (8, 0.5), (9, 0.3), (9, 0.25), (7, 0.7), (5, 1.0),
     (9, 0.2), (8, 0.3), (6, 0.3), (9, 0.35)])]
SMALL += [gg.cycle(7), gg.full_grid(3, 3), gg.star(5), gg.path(6),
          gg.disjoint_union(gg.cycle(4), gg.path(3)), gg.complete_bipartite(2, 3)]


@pytest.mark.parametrize("g", SMALL, ids=[g.name for g in SMALL])
def test_brandes_matches_exact_enumeration(g):
    raw_exact, d_exact, sig_exact = brute.bc_exact(g)
    raw, ovf = oracle.bc(g)
    assert not ovf.any()
    for v in range(g.n):
        assert abs(Fraction(raw[v]) - raw_exact[v]) <= Fraction(1, 10 ** 9) * max(1, abs(raw_exact[v]))
        if raw_exact[v] == 0:
            assert raw[v] == 0.0
    for s in range(g.n):
        tr = oracle.source(g, s)
        for t in range(g.n):
            if d_exact[s][t] is None:
                assert tr["d"][t] == -1 and tr["sigma"][t] == 0
            else:
                assert tr["d"][t] == d_exact[s][t]
                assert int(tr["sigma"][t]) == sig_exact[s][t]


def test_bellman_matches_exact_enumeration():
    for g in SMALL[:6]:
        raw_exact, _, _ = brute.bc_exact(g)
        assert_close(oracle.bellman(g), [float(x) for x in raw_exact])


# ------------------------------------------------------- independent methods

def test_r_mat_scale10_three_ways():
    """The small R-MAT workload: Brandes vs the O(n^3) Bellman method vs networkx."""
    g = gg.workload_rmat10()
    raw, ovf = oracle.bc(g)
    assert not ovf.any()
    assert_close(raw, oracle.bellman(g))
    G = nx_graph(g)
    ref = nx.betweenness_centrality(G, normalized=False)
    assert_close(raw / 2, [ref[i] for i in range(g.n)])


@pytest.mark.parametrize("seed", [11, 12, 13])
def test_networkx_random_graphs(seed):
    g = gg.erdos_renyi(120, 0.04, seed)
    G = nx_graph(g)
    ref = nx.betweenness_centrality(G, normalized=False)
    assert_close(undirected(g)[0], [ref[i] for i in range(g.n)])


def test_networkx_subset_sources():
    """Source subsets: networkx's subset routine counts each ordered (s, t)
    pair from s once (and halves for undirected); RAW over a source set S is
    the same sum without the halving."""
    g = gg.rmat(8, 8, 21)
    S = gg.sample(g.non_isolated(), 40, 5)
    raw, _ = oracle.bc(g, S)
    G = nx_graph(g)
    ref = nx.betweenness_centrality_subset(G, sources=S.tolist(), targets=list(range(g.n)),
                                           normalized=False)
    assert_close(raw / 2, [ref[i] for i in range(g.n)])


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("k", [1, 2, 3, 10, 57])
def test_star(k):
    bc, _ = undirected(gg.star(k))
    n = k + 1
    assert bc[0] == (n - 1) * (n - 2) / 2
    assert (bc[1:] == 0).all()


@pytest.mark.parametrize("n", [2, 3, 4, 9, 50])
def test_path(n):
    bc, _ = undirected(gg.path(n))
    assert np.array_equal(bc, [i * (n - 1 - i) for i in range(n)])


@pytest.mark.parametrize("n", [3, 4, 5, 8, 9, 31, 64])
def test_cycle(n):
    bc, _ = undirected(gg.cycle(n))
    expect = (n - 1) * (n - 3) / 8 if n % 2 else (n - 2) ** 2 / 8
    assert_close(bc, np.full(n, expect))


@pytest.mark.parametrize("n", [2, 3, 6, 20])
def test_complete(n):
    bc, _ = undirected(gg.complete(n))
    assert (bc == 0).all()


@pytest.mark.parametrize("p,q", [(1, 5), (2, 3), (3, 7), (6, 6)])
def test_complete_bipartite(p, q):
    bc, _ = undirected(gg.complete_bipartite(p, q))
    assert_close(bc[:p], np.full(p, q * (q - 1) / (2 * p)))
    assert_close(bc[p:], np.full(q, p * (p - 1) / (2 * q)))


@pytest.mark.parametrize("d", [1, 2, 3, 5, 8])
def test_hypercube(d):
    bc, _ = undirected(gg.hypercube(d))
    expect = (d * 2 ** (d - 1) - 2 ** d + 1) / 2
    assert_close(bc, np.full(2 ** d, expect))


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_tree_component_products(seed):
    """In a tree every pair has one path, so BC(v) is the number of unordered
    pairs split by removing v: sum over i<j of |C_i||C_j| (components of T-v),
    computed here by networkx connected components."""
    g = gg.random_tree(60, seed)
    G = nx_graph(g)
    bc, _ = undirected(g)
    for v in range(g.n):
        H = G.copy()
        H.remove_node(v)
        sizes = [len(c) for c in nx.connected_components(H)]
        tot = sum(sizes)
        expect = (tot * tot - sum(s * s for s in sizes)) / 2
        assert bc[v] == expect


# -------------------------------------------------------------- sigma pins

def test_grid_corner_binomials():
    """From a corner of a full k x k lattice, vertex (i, j) has C(i+j, i)
    shortest paths at distance i + j."""
    k = 12
    tr = oracle.source(gg.full_grid(k, k), 0)
    for i in range(k):
        for j in range(k):
            assert tr["d"][i * k + j] == i + j
            assert int(tr["sigma"][i * k + j]) == math.comb(i + j, i)


def test_grid_overflow_boundary():
    """C(66,33) < 2^64 < C(68,34): the 34 x 34 lattice from a corner is exact,
    the 35 x 35 one wraps, and its long-double counts are still right."""
    assert math.comb(66, 33) < 2 ** 64 < math.comb(68, 34)
    t34 = oracle.source(gg.full_grid(34, 34), 0)
    assert not t34["overflow"]
    assert int(t34["sigma"][34 * 34 - 1]) == math.comb(66, 33)
    t35 = oracle.source(gg.full_grid(35, 35), 0)
    assert t35["overflow"]
    far = t35["sigma_ld"][35 * 35 - 1]
    assert abs(float(far) / math.comb(68, 34) - 1) < 1e-15


@pytest.mark.parametrize("d", [4, 10])
def test_hypercube_factorials(d):
    """In Q_d, sigma(s, t) = d(s,t)! (choose the order of the differing bits)."""
    tr = oracle.source(gg.hypercube(d), 0)
    for t in range(2 ** d):
        k = bin(t).count("1")
        assert tr["d"][t] == k and int(tr["sigma"][t]) == math.factorial(k)


@pytest.mark.slow
def test_hypercube_21_wraps_exactly_at_antipode():
    """20! < 2^64 < 21!: in Q_21 only the antipodal target overflows."""
    assert math.factorial(20) < 2 ** 64 < math.factorial(21)
    g = gg.hypercube(21)
    tr = oracle.source(g, 0)
    assert tr["overflow"]
    far = tr["sigma_ld"][2 ** 21 - 1]
    assert abs(float(far) / math.factorial(21) - 1) < 1e-15
    t20 = oracle.source(gg.hypercube(20), 0)
    assert not t20["overflow"] and int(t20["sigma"][2 ** 20 - 1]) == math.factorial(20)


def test_layered_chain_wraps_at_layer_17():
    """Apex plus complete bipartite layers of width 16: a layer-j vertex has
    16^(j-1) paths, so 16 layers stay below 2^64 = 16^16 and 17 wrap."""
    t16 = oracle.source(gg.layered_chain(16, 16), 0)
    assert not t16["overflow"]
    assert int(t16["sigma"][1 + 15 * 16]) == 16 ** 15
    t17 = oracle.source(gg.layered_chain(16, 17), 0)
    assert t17["overflow"]
    assert float(t17["sigma_ld"][1 + 16 * 16]) == float(16 ** 16)


def test_sigma_symmetry():
    g = gg.rmat(9, 8, 4)
    S = gg.sample(g.non_isolated(), 12, 1)
    tr = {int(s): oracle.source(g, s) for s in S}
    for a in S:
        for b in S:
            assert tr[int(a)]["sigma"][b] == tr[int(b)]["sigma"][a]
            assert tr[int(a)]["d"][b] == tr[int(b)]["d"][a]


# ------------------------------------------------------------------ invariants

def pair_distance_sum(g):
    """sum over connected unordered pairs of (d - 1), from networkx BFS."""
    G = nx_graph(g)
    tot = 0
    for s, dist in nx.all_pairs_shortest_path_length(G):
        tot += sum(L - 1 for t, L in dist.items() if t > s)
    return tot


@pytest.mark.parametrize("g", [gg.rmat(9, 8, 7), gg.erdos_renyi(200, 0.02, 3),
                               gg.disjoint_union(gg.cycle(9), gg.rmat(7, 4, 2), gg.path(4))],
                         ids=["rmat9", "er200", "union"])
def test_total_equals_pair_distances(g):
    bc, _ = undirected(g)
    assert abs(bc.sum() - pair_distance_sum(g)) <= 1e-9 * max(1.0, bc.sum())


def test_per_source_delta_sum_including_overflowed():
    """Per source, sum over v != s of delta_s(v) = sum over reachable t of
    (d(s,t) - 1).  It does not depend on sigma's size, so it also checks the
    long-double rerun of an overflowed source."""
    for g, s in [(gg.rmat(9, 8, 3), 5), (gg.full_grid(40, 40), 0), (gg.layered_chain(16, 20), 0)]:
        tr = oracle.source(g, s)
        d = tr["d"]
        reach = d >= 0
        expect = float(np.sum(d[reach] - 1) + 1)   # the t = s term contributes -1
        got = tr["delta"].sum() - tr["delta"][s]
        assert abs(got - expect) <= 1e-9 * expect
    assert oracle.source(gg.full_grid(40, 40), 0)["overflow"]


def test_zero_iff_neighbourhood_is_clique():
    g = gg.erdos_renyi(60, 0.15, 9)
    bc, _ = undirected(g)
    G = nx_graph(g)
    for v in range(g.n):
        nb = list(G.neighbors(v))
        clique = all(G.has_edge(a, b) for i, a in enumerate(nb) for b in nb[i + 1:])
        assert (bc[v] == 0) == clique


def test_relabelling_permutes_scores():
    g = gg.rmat(9, 8, 5)
    perm = gg.permutation(g.n, 77)
    bc, _ = undirected(g)
    bp, _ = undirected(gg.relabel(g, perm))
    assert_close(bp[perm], bc)


def test_disjoint_union_is_union_of_scores():
    a, b = gg.rmat(8, 8, 1), gg.cycle(11)
    u = gg.disjoint_union(a, b)
    bu, _ = undirected(u)
    assert_close(bu[:a.n], undirected(a)[0])
    assert_close(bu[a.n:], undirected(b)[0])


def test_threads_do_not_change_results():
    g = gg.rmat(10, 8, 9)
    r1, _, s1 = oracle.bc(g, nthreads=1, want_stats=True)
    r4, _, s4 = oracle.bc(g, nthreads=4, want_stats=True)
    assert_close(r1, r4, 1e-12)
    assert np.array_equal(s1, s4)


def test_stats_definitions():
    """Per-source stats: reached vertices, directed CSR entries of reached
    vertices, DAG edges (= predecessor relations = edges joining consecutive
    levels).  Checked against a direct count from the distances."""
    g = gg.rmat(8, 8, 6)
    S = gg.sample(g.non_isolated(), 10, 2)
    _, _, st = oracle.bc(g, S, want_stats=True)
    deg = g.degrees()
    for i, s in enumerate(S):
        d = oracle.source(g, s)["d"]
        reach = d >= 0
        u = np.repeat(np.arange(g.n), deg)
        v = g.col_idx
        dag = np.sum((d[u] >= 0) & (d[v] == d[u] + 1))
        assert st[i, 0] == reach.sum() and st[i, 1] == deg[reach].sum() and st[i, 2] == dag
