"""The oracle's pins must be able to fail.  Each case plants one plausible
mistake in a copy of the oracle source (on the CPU, in a temp dir), builds it,
and checks that the brute-force / closed-form comparison then fails."""
import ctypes
import os
import subprocess
import tempfile

import numpy as np
import pytest

import graphgen as gg
from oracle import brute

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "brandes.c")

MUTANTS = {
    "drop_one_plus_delta": ("* (1.0 + del[x]);", "* (del[x]);"),
    "swap_sigma_ratio": ("(double)w->sig[v] / (double)w->sig[x]", "(double)w->sig[x] / (double)w->sig[v]"),
    "count_source_itself": ("if (x != s && bc) bc[x] += del[x];", "if (bc) bc[x] += del[x];"),
    "level_off_by_one": ("if (d[x] == d[v] + 1) {\n        uint64_t", "if (d[x] == d[v] + 2) {\n        uint64_t"),
    "sigma_assign_not_add": ("w->sig[x] = before + w->sig[v];", "w->sig[x] = w->sig[v];"),
    "pred_wrong_vertex": ("w->pred[rp[x] + w->npred[x]++] = v;\n      }\n    }\n  }\n  return tail;",
                          "w->pred[rp[x] + w->npred[x]++] = x;\n      }\n    }\n  }\n  return tail;"),
}

GRAPHS = [gg.erdos_renyi(8, 0.35, 3), gg.full_grid(3, 3), gg.cycle(6), gg.erdos_renyi(9, 0.3, 4)]


def build_mutant(tmp, name, old, new):
    text = open(SRC).read()
    assert text.count(old) == 1, name
    path = os.path.join(tmp, name + ".c")
    with open(path, "w") as f:
        f.write(text.replace(old, new))
    so = os.path.join(tmp, name + ".so")
    subprocess.check_call(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-pthread", "-o", so, path])
    lib = ctypes.CDLL(so)
    lib.orc_bc.restype = ctypes.c_int
    lib.orc_bc.argtypes = [ctypes.c_int32] + [ctypes.c_void_p] * 3 + [ctypes.c_int64, ctypes.c_int] + [ctypes.c_void_p] * 3
    return lib


def agrees_with_brute(lib, g):
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(g.col_idx, dtype=np.int32)
    src = np.arange(g.n, dtype=np.int32)
    out = np.zeros(g.n)
    lib.orc_bc(g.n, rp.ctypes.data, ci.ctypes.data, src.ctypes.data, g.n, 1, out.ctypes.data, None, None)
    exact = np.array([float(x) for x in brute.bc_exact(g)[0]])
    return bool(np.allclose(out, exact, rtol=1e-9, atol=1e-12))


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name):
    with tempfile.TemporaryDirectory() as tmp:
        lib = build_mutant(tmp, name, *MUTANTS[name])
        assert not all(agrees_with_brute(lib, g) for g in GRAPHS), f"mutant {name} survived"


def test_unmutated_copy_passes():
    with tempfile.TemporaryDirectory() as tmp:
        lib = build_mutant(tmp, "identity", "#include <math.h>", "#include <math.h>")
        assert all(agrees_with_brute(lib, g) for g in GRAPHS)
