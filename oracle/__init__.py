"""CPU oracle for exact betweenness centrality -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never uses it; the
two share no code.  Scores are RAW (ordered source/target pairs, the paper's
Eq. (3)); halve them for the usual undirected convention.

* :func:`bc`      -- sequential Brandes (Alg. 1) over a source list, with
  checked uint64 path counts and a long-double rerun for sources that wrap.
* :func:`source`  -- the per-source trace (d, sigma, delta, overflow flag).
* :func:`bellman` -- the O(n^3) pair-dependency method (Floyd-Warshall plus
  the Bellman criterion, Lemma 2), independent of Brandes' recursion.
* :mod:`oracle.brute` -- exact rational brute force by path enumeration.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    src = os.path.join(_HERE, "brandes.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread",
                               "-o", tmp, src])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        lib = ctypes.CDLL(_SO)
        vp = ctypes.c_void_p
        lib.orc_source.restype = ctypes.c_int
        lib.orc_source.argtypes = [ctypes.c_int32, vp, vp, ctypes.c_int32, vp, vp, vp, vp, vp]
        lib.orc_bc.restype = ctypes.c_int
        lib.orc_bc.argtypes = [ctypes.c_int32, vp, vp, vp, ctypes.c_int64, ctypes.c_int, vp, vp, vp]
        lib.orc_bellman.restype = ctypes.c_int
        lib.orc_bellman.argtypes = [ctypes.c_int32, vp, vp, vp]
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def _csr(g):
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(g.col_idx, dtype=np.int32)
    return rp, ci


def bc(g, sources=None, nthreads: int = 1, want_stats: bool = False):
    """RAW scores over ``sources`` (default: every vertex).

    Returns ``(raw[n] float64, overflowed[k] bool)`` and, with
    ``want_stats``, also ``stats[k, 3]`` = (vertices reached, directed CSR
    entries of reached vertices, DAG edges) per source.
    """
    rp, ci = _csr(g)
    if sources is None:
        sources = np.arange(g.n, dtype=np.int32)
    src = np.ascontiguousarray(sources, dtype=np.int32)
    out = np.zeros(g.n, dtype=np.float64)
    ovf = np.zeros(len(src), dtype=np.uint8)
    stats = np.zeros((len(src), 3), dtype=np.int64) if want_stats else None
    r = _load().orc_bc(g.n, _ptr(rp), _ptr(ci), _ptr(src), len(src), nthreads,
                       _ptr(out), _ptr(ovf), _ptr(stats))
    if r != 0:
        raise RuntimeError(f"orc_bc failed ({r})")
    if want_stats:
        return out, ovf.astype(bool), stats
    return out, ovf.astype(bool)


def source(g, s: int) -> dict:
    """Per-source trace: d (int32, -1 unreached), sigma (uint64, valid only if
    not overflowed), sigma_ld (long double counts), delta (float64),
    overflow (bool), stats (reached, nnz_r, dag edges)."""
    rp, ci = _csr(g)
    d = np.empty(g.n, dtype=np.int32)
    sig = np.empty(g.n, dtype=np.uint64)
    sld = np.empty(g.n, dtype=np.longdouble)
    dl = np.empty(g.n, dtype=np.float64)
    st = np.zeros(3, dtype=np.int64)
    r = _load().orc_source(g.n, _ptr(rp), _ptr(ci), int(s), _ptr(d), _ptr(sig), _ptr(sld),
                           _ptr(dl), _ptr(st))
    if r < 0:
        raise RuntimeError(f"orc_source failed ({r})")
    return {"d": d, "sigma": sig, "sigma_ld": sld, "delta": dl, "overflow": bool(r), "stats": st}


def bellman(g) -> np.ndarray:
    """RAW scores by the O(n^3) pair-dependency method (all sources)."""
    rp, ci = _csr(g)
    out = np.zeros(g.n, dtype=np.float64)
    if _load().orc_bellman(g.n, _ptr(rp), _ptr(ci), _ptr(out)) != 0:
        raise RuntimeError("orc_bellman failed")
    return out


def close(a, b, rel: float = 1e-9) -> np.ndarray:
    """Elementwise tolerance rule used throughout the tests: |a-b| <=
    rel*max(|a|,|b|), and exact equality where either side is zero."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    zero = (a == 0) | (b == 0)
    ok = np.abs(a - b) <= rel * np.maximum(np.abs(a), np.abs(b))
    return np.where(zero, a == b, ok)
