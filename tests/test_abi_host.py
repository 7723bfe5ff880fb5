"""C-ABI checks that need no GPU: the library loads, exports every symbol
the header declares, and its host-side validation and 1-degree reduction
behave as specified."""
import ctypes
import os
import re

import numpy as np
import pytest

import graphgen as gg
import paper_1602_00963_amd as bcm
from paper_1602_00963_amd import bc as bcmod

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "bc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bc_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    L = bcm.lib()
    declared = header_functions()
    assert len(declared) >= 18
    for name in declared:
        assert hasattr(L, name), name
    assert sorted(bcmod.EXPORTED) == declared


def test_status_strings():
    L = bcm.lib()
    for st in range(10):
        assert L.bc_status_string(st)


def test_struct_layouts_match_header(tmp_path):
    """The ctypes mirrors must match the C layout: compile a probe against
    include/bc.h with gcc and compare sizes and field offsets."""
    import subprocess
    structs = {"bc_graph_stats": bcmod.GraphStats, "bc_compute_opts": bcmod.ComputeOpts,
               "bc_run_stats": bcmod.RunStats, "bc_server_config": bcmod.ServerConfig,
               "bc_server_stats": bcmod.ServerStats,
               "bc_query_stats": bcmod.QueryStats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "bc.h"', 'int main(void) {']
    for cname, py in structs.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = dict(line.rsplit(" ", 1) for line in subprocess.check_output([str(exe)], text=True).split("\n") if line)
    for cname, py in structs.items():
        assert int(out[cname]) == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert int(out[f"{cname}.{f}"]) == getattr(py, f).offset, (cname, f)


@pytest.mark.parametrize("g", [gg.star(4), gg.cycle(7), gg.rmat(10, 8, 3), gg.full_grid(5, 6)],
                         ids=["star", "cycle", "rmat", "grid"])
def test_valid_graphs_pass(g):
    bcm.validate_csr(g.n, g.row_ptr, g.col_idx)


def bad_cases():
    ok = gg.cycle(5)
    rp, ci = ok.row_ptr.copy(), ok.col_idx.copy()
    yield "asymmetric", 3, [0, 1, 1, 1], [1]
    yield "self_loop", 2, [0, 2, 3], [0, 1, 0]
    yield "duplicate", 2, [0, 2, 4], [1, 1, 0, 0]
    yield "out_of_range", 2, [0, 1, 2], [5, 0]
    yield "nnz_mismatch", 2, [0, 1, 1], [1, 0]
    bad = ci.copy()
    bad[0], bad[1] = bad[1], bad[0]          # still valid (order is free)
    yield "reordered_ok", 5, rp, bad


@pytest.mark.parametrize("case", list(bad_cases()), ids=lambda c: c[0])
def test_invalid_graphs_rejected(case):
    name, n, rp, ci = case
    if name.endswith("_ok"):
        bcm.validate_csr(n, rp, ci)
        return
    with pytest.raises(bcm.BCError) as e:
        bcm.validate_csr(n, rp, ci)
    assert e.value.status == bcmod.E_INVALID_GRAPH


def test_prune_star_and_k2_and_path():
    # star: 5 pendants on the centre; K2: both ends dropped; P3: both ends
    # are pendants of the middle vertex
    g = gg.disjoint_union(gg.star(5), gg.path(2), gg.path(3))
    p = bcm.prune_deg1_host(g.n, g.row_ptr, g.col_idx)
    assert p["omega"].tolist() == [5, 0, 0, 0, 0, 0, 0, 0, 0, 2, 0]
    assert p["kind"].tolist() == [0, 1, 1, 1, 1, 1, 2, 2, 1, 0, 1]
    assert p["hub"].tolist() == [-1, 0, 0, 0, 0, 0, -1, -1, 9, -1, 9]
    assert len(p["col_idx"]) == 0


def test_prune_residual_is_induced_subgraph():
    g = gg.rmat_with_pendants(11, 8, 5, 0.3, 55)
    p = bcm.prune_deg1_host(g.n, g.row_ptr, g.col_idx)
    deg = g.degrees()
    kept = p["kind"] == 0
    # every removed vertex is degree-1 with a hub of degree >= 2, or a K2 end
    pend = p["kind"] == 1
    assert np.all(deg[pend] == 1)
    hubs = p["hub"][pend]
    assert np.all(deg[hubs] >= 2)
    assert np.array_equal(np.bincount(hubs, minlength=g.n), p["omega"])
    # residual edges are exactly the original edges between kept vertices
    u = np.repeat(np.arange(g.n), deg)
    keep_e = kept[u] & kept[g.col_idx]
    ru = np.repeat(np.arange(g.n), np.diff(p["row_ptr"]))
    assert np.array_equal(np.stack([u[keep_e], g.col_idx[keep_e]]), np.stack([ru, p["col_idx"]]))
    bcm.validate_csr(g.n, p["row_ptr"], p["col_idx"])
