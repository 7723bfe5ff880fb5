"""The entry point that allocates nothing (bc_compute_noalloc) against
bc_compute in the plain form, through the C ABI: two calls in a row on one
device, the second with a smaller input, each compared with bc_compute's
scores on the same graph and sources (relative 1e-9, exact where either is
0).  Also: a graph whose workspace exceeds the fixed array is refused before
any device work, and the batched mode is refused."""
import sys

import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _pair(bcm, ctx, g, sources, **opts):
    G = bcm.Graph(ctx, g)
    st_ref = G.compute(sources, mode="plain", **opts)
    ref = G.scores()
    G.reset()
    st_na = G.compute_noalloc(sources, **opts)
    got = G.scores()
    G.close()
    return ref, got, st_ref, st_na


def test_noalloc_equals_compute_two_calls():
    import paper_1602_00963_amd as bcm
    ctx = bcm.Context(0)
    # first call: scale-12 R-MAT, 300 sampled sources
    g1 = gg.rmat(12, 8, 31)
    s1 = gg.sample(g1.non_isolated(), 300, 5)
    say("noalloc call 1: rmat(12, 8, 31), 300 sources")
    ref, got, a, b = _pair(bcm, ctx, g1, s1)
    ok = oracle.close(got, ref, 1e-9)
    assert ok.all(), np.nonzero(~ok)[0][:8]
    assert a["launches"] == b["launches"] and a["reached"] == b["reached"] and a["dag_edges"] == b["dag_edges"]
    assert b["kernel_ms"] == 0.0
    # second call, smaller input: a 40 x 40 lattice whose corner counts wrap
    # uint64 (AUTO reruns those sources in extended form inside the call)
    g2 = gg.full_grid(40, 40)
    s2 = np.array([0, 39, 40 * 39, 40 * 40 - 1, 820, 5, 77], dtype=np.int32)
    say("noalloc call 2: 40x40 lattice, 7 sources")
    ref2, got2, a2, b2 = _pair(bcm, ctx, g2, s2)
    ok = oracle.close(got2, ref2, 1e-9)
    assert ok.all(), np.nonzero(~ok)[0][:8]
    assert b2["overflowed"] == a2["overflowed"] > 0
    assert b2["rerun_extended"] == a2["rerun_extended"]
    # and against the oracle on the small case
    want, _ = oracle.bc(g2, s2)
    assert oracle.close(got2, want, 1e-9).all()
    ctx.close()


def test_noalloc_refuses_oversize_and_batched():
    import paper_1602_00963_amd as bcm
    from paper_1602_00963_amd import bc as bcmod
    ctx = bcm.Context(0)
    # a 600,000-vertex path: its plain workspace is larger than the array
    n = 600_000
    g = gg.path(n)
    G = bcm.Graph(ctx, g, validate=False)
    assert G.workspace_size(mode="plain") > 64 << 20
    with pytest.raises(bcm.BCError) as e:
        G.compute_noalloc([0, 1])
    assert e.value.status == bcmod.E_CAPACITY
    G.close()
    g2 = gg.rmat(9, 8, 3)
    G2 = bcm.Graph(ctx, g2)
    with pytest.raises(bcm.BCError) as e:
        G2.compute_noalloc([0, 1], mode="batched")
    assert e.value.status == bcmod.E_INVALID_ARG
    G2.close()
    ctx.close()
