"""Seeded synthetic graph inputs (their own module: no betweenness arithmetic).

The heavy generators (R-MAT, the road-like lattice, CSR assembly) are plain C
in ``gen.c`` built into ``libgraphgen.so``; the small closed-form families are
numpy.  Every graph is returned as a :class:`Graph` holding a symmetric CSR
(int32 ``row_ptr``/``col_idx``, adjacency sorted, no self-loops or duplicate
pairs), which is the input form both the GPU library and the CPU oracle take.

Workload recipes (the R-MAT parameters follow the paper's experimental
section; the pendant, lattice and serving recipes are synthetic stand-ins):

* ``rmat(scale, ef, seed)``: 2^scale * ef ordered pairs, quadrant
  probabilities (0.57, 0.19, 0.19, 0.05), no noise, seeded relabelling,
  then symmetrised with self-loops and duplicates dropped.
* ``rmat_with_pendants``: the R-MAT graph plus round(frac * 2^scale) new
  degree-1 vertices, each joined to a uniform random original vertex.
* ``road_grid``: R x C lattice minus an exact count of random lattice edges
  plus an exact count of distinct local diagonals.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libgraphgen.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile gen.c into libgraphgen.so (gcc, -O2)."""
    src = os.path.join(_HERE, "gen.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, src])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        lib = ctypes.CDLL(_SO)
        i32p = ctypes.POINTER(ctypes.c_int32)
        i64p = ctypes.POINTER(ctypes.c_int64)
        lib.gg_u64.restype = ctypes.c_uint64
        lib.gg_u64.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        lib.gg_rmat_pairs.restype = None
        lib.gg_rmat_pairs.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_uint64, i32p, i32p]
        lib.gg_permutation.restype = None
        lib.gg_permutation.argtypes = [ctypes.c_int64, ctypes.c_uint64, i32p]
        lib.gg_pendant_pairs.restype = None
        lib.gg_pendant_pairs.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64, i32p, i32p]
        lib.gg_grid_pairs.restype = ctypes.c_int64
        lib.gg_grid_pairs.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                      ctypes.c_uint64, i32p, i32p]
        lib.gg_sample.restype = ctypes.c_int
        lib.gg_sample.argtypes = [i32p, ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64, i32p]
        lib.gg_build_csr.restype = ctypes.c_int64
        lib.gg_build_csr.argtypes = [ctypes.c_int64, ctypes.c_int64, i32p, i32p, i64p, i32p]
        _lib = lib
    return _lib


def _p32(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _p64(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


@dataclass
class Graph:
    """Symmetric simple graph in CSR form (int32 arrays)."""
    n: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def m(self) -> int:
        """Unique undirected edge count."""
        return self.nnz // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr).astype(np.int64)

    def non_isolated(self) -> np.ndarray:
        return np.nonzero(self.degrees() > 0)[0].astype(np.int32)

    def edges(self):
        """Unordered pairs (u < v) as two int arrays."""
        deg = self.degrees()
        u = np.repeat(np.arange(self.n, dtype=np.int64), deg)
        v = self.col_idx.astype(np.int64)
        keep = u < v
        return u[keep], v[keep]


def from_pairs(n: int, src, dst, name: str = "") -> Graph:
    """CSR from unordered pairs; drops self-loops and duplicates."""
    src = np.ascontiguousarray(np.asarray(src, dtype=np.int32))
    dst = np.ascontiguousarray(np.asarray(dst, dtype=np.int32))
    if src.shape != dst.shape:
        raise ValueError("src/dst length mismatch")
    lib = _load()
    rp = np.zeros(n + 1, dtype=np.int64)
    col = np.empty(max(2 * len(src), 1), dtype=np.int32)
    nnz = lib.gg_build_csr(n, len(src), _p32(src), _p32(dst), _p64(rp), _p32(col))
    if nnz < 0:
        raise ValueError("pair list has ids outside [0, n)" if nnz == -2 else "allocation failed")
    if nnz >= 2 ** 31:
        raise ValueError("graph exceeds int32 CSR limits")
    return Graph(n, rp.astype(np.int32), col[:nnz].copy(), name)


def u64(seed: int, ctr: int) -> int:
    """The counter-based splitmix64 draw used throughout this module."""
    return int(_load().gg_u64(seed, ctr))


def rmat_pairs(scale: int, ef: int, seed: int, a=0.57, b=0.19, c=0.19):
    npairs = (1 << scale) * ef
    src = np.empty(npairs, dtype=np.int32)
    dst = np.empty(npairs, dtype=np.int32)
    _load().gg_rmat_pairs(scale, npairs, a, b, c, seed, _p32(src), _p32(dst))
    return src, dst


def rmat(scale: int, ef: int, seed: int, a=0.57, b=0.19, c=0.19) -> Graph:
    src, dst = rmat_pairs(scale, ef, seed, a, b, c)
    return from_pairs(1 << scale, src, dst, name=f"rmat{scale}_ef{ef}_s{seed}")


def rmat_with_pendants(scale: int, ef: int, seed: int, frac: float = 0.3,
                       pend_seed: int | None = None) -> Graph:
    n0 = 1 << scale
    P = int(round(frac * n0))
    src, dst = rmat_pairs(scale, ef, seed)
    ps = np.empty(P, dtype=np.int32)
    pd = np.empty(P, dtype=np.int32)
    _load().gg_pendant_pairs(n0, P, seed * 10 + 3 if pend_seed is None else pend_seed, _p32(ps), _p32(pd))
    return from_pairs(n0 + P, np.concatenate([src, ps]), np.concatenate([dst, pd]),
                      name=f"rmat{scale}_ef{ef}_s{seed}_pend{frac}")


def road_grid(R: int, C: int, drop_frac: float = 0.05, diag_frac: float = 0.01, seed: int = 4) -> Graph:
    nl = R * (C - 1) + (R - 1) * C
    drop = int(round(drop_frac * nl))
    diag = int(round(diag_frac * nl))
    cap = nl + diag
    src = np.empty(max(cap, 1), dtype=np.int32)
    dst = np.empty(max(cap, 1), dtype=np.int32)
    w = _load().gg_grid_pairs(R, C, drop, diag, seed, _p32(src), _p32(dst))
    if w < 0:
        raise ValueError("bad grid arguments")
    return from_pairs(R * C, src[:w], dst[:w], name=f"grid{R}x{C}_s{seed}")


def permutation(n: int, seed: int) -> np.ndarray:
    perm = np.empty(n, dtype=np.int32)
    _load().gg_permutation(n, seed, _p32(perm))
    return perm


def sample(cand, k: int, seed: int) -> np.ndarray:
    """k distinct entries of cand, uniformly (seeded), in draw order."""
    cand = np.ascontiguousarray(np.asarray(cand, dtype=np.int32))
    out = np.empty(max(k, 1), dtype=np.int32)
    if _load().gg_sample(_p32(cand), len(cand), k, seed, _p32(out)) != 0:
        raise ValueError("k exceeds candidate count")
    return out[:k].copy()


# ---------------------------------------------------------------- small families

def star(k: int) -> Graph:
    """Centre 0 with leaves 1..k."""
    return from_pairs(k + 1, np.zeros(k), np.arange(1, k + 1), name=f"star{k}")


def path(n: int) -> Graph:
    return from_pairs(n, np.arange(n - 1), np.arange(1, n), name=f"path{n}")


def cycle(n: int) -> Graph:
    return from_pairs(n, np.arange(n), (np.arange(n) + 1) % n, name=f"cycle{n}")


def complete(n: int) -> Graph:
    u, v = np.triu_indices(n, 1)
    return from_pairs(n, u, v, name=f"K{n}")


def complete_bipartite(p: int, q: int) -> Graph:
    """Side A = 0..p-1, side B = p..p+q-1."""
    u = np.repeat(np.arange(p), q)
    v = p + np.tile(np.arange(q), p)
    return from_pairs(p + q, u, v, name=f"K{p},{q}")


def hypercube(d: int) -> Graph:
    n = 1 << d
    u = np.repeat(np.arange(n, dtype=np.int64), d)
    bit = np.tile(np.arange(d, dtype=np.int64), n)
    v = u ^ (np.int64(1) << bit)
    keep = u < v
    return from_pairs(n, u[keep], v[keep], name=f"Q{d}")


def full_grid(R: int, C: int) -> Graph:
    ids = np.arange(R * C).reshape(R, C)
    u = np.concatenate([ids[:, :-1].ravel(), ids[:-1, :].ravel()])
    v = np.concatenate([ids[:, 1:].ravel(), ids[1:, :].ravel()])
    return from_pairs(R * C, u, v, name=f"grid{R}x{C}")


def random_tree(n: int, seed: int) -> Graph:
    """Uniform random labelled tree: vertex i > 0 joins a random earlier vertex
    after a seeded relabelling (a random recursive tree)."""
    rng = np.random.default_rng(seed)
    parent = np.array([rng.integers(0, i) for i in range(1, n)], dtype=np.int64)
    perm = rng.permutation(n)
    return from_pairs(n, perm[np.arange(1, n)], perm[parent], name=f"tree{n}_s{seed}")


def erdos_renyi(n: int, p: float, seed: int) -> Graph:
    rng = np.random.default_rng(seed)
    u, v = np.triu_indices(n, 1)
    keep = rng.random(len(u)) < p
    return from_pairs(n, u[keep], v[keep], name=f"er{n}_{p}_s{seed}")


def layered_chain(width: int, layers: int) -> Graph:
    """Apex 0, then `layers` layers of `width` vertices; consecutive layers are
    joined completely (apex to all of layer 1).  A vertex of layer j is
    reached from the apex by width**(j-1) shortest paths."""
    n = 1 + width * layers
    us, vs = [np.zeros(width, dtype=np.int64)], [1 + np.arange(width)]
    for j in range(1, layers):
        a = 1 + (j - 1) * width + np.arange(width)
        b = 1 + j * width + np.arange(width)
        us.append(np.repeat(a, width))
        vs.append(np.tile(b, width))
    return from_pairs(n, np.concatenate(us), np.concatenate(vs), name=f"chain{width}x{layers}")


def disjoint_union(*gs: Graph) -> Graph:
    us, vs, off = [], [], 0
    for g in gs:
        u, v = g.edges()
        us.append(u + off)
        vs.append(v + off)
        off += g.n
    return from_pairs(off, np.concatenate(us) if us else [], np.concatenate(vs) if vs else [],
                      name="union")


def relabel(g: Graph, perm: np.ndarray) -> Graph:
    """Vertex i of g becomes perm[i]."""
    u, v = g.edges()
    return from_pairs(g.n, perm[u], perm[v], name=g.name + "_relabel")


def add_pendants(g: Graph, hubs) -> Graph:
    """Attach one new degree-1 vertex to each entry of hubs (repeats allowed)."""
    hubs = np.asarray(hubs, dtype=np.int64)
    u, v = g.edges()
    new = g.n + np.arange(len(hubs))
    return from_pairs(g.n + len(hubs), np.concatenate([u, new]), np.concatenate([v, hubs]),
                      name=g.name + "_pend")


def attach_trees(g: Graph, sizes, seed: int) -> Graph:
    """Hang one seeded random tree of each given size from a uniformly chosen
    vertex of g (an edge from the tree's first vertex to it)."""
    rng = np.random.default_rng(seed)
    u, v = g.edges()
    us, vs = [u], [v]
    n = g.n
    for i, sz in enumerate(sizes):
        t = random_tree(int(sz), seed * 1000 + i) if sz > 1 else None
        if t is not None:
            tu, tv = t.edges()
            us.append(tu + n)
            vs.append(tv + n)
        us.append(np.array([n], dtype=np.int64))
        vs.append(np.array([rng.integers(0, g.n)], dtype=np.int64))
        n += int(sz)
    return from_pairs(n, np.concatenate(us), np.concatenate(vs), name=g.name + "_trees")


# ------------------------------------------------------------- benchmark workloads

def workload_rmat10() -> Graph:
    """R-MAT scale 10, edge factor 16, seed 1."""
    return rmat(10, 16, 1)


def workload_rmat16() -> Graph:
    """R-MAT scale 16, edge factor 16, seed 2."""
    return rmat(16, 16, 2)


def workload_rmat20_pendants(scale: int = 20) -> Graph:
    """R-MAT (scale, EF 16, seed 3) plus 30% extra pendant vertices (seed 33)."""
    return rmat_with_pendants(scale, 16, 3, 0.3, pend_seed=33)


def workload_roadlike_grid(R: int = 2048, C: int = 2048) -> Graph:
    """Road-like lattice: 5% lattice edges removed, 1% local diagonals, seed 4."""
    return road_grid(R, C, 0.05, 0.01, 4)


def serving_graph_specs(count: int = 32, seed: int = 5000, min_scale: int = 12, max_scale: int = 20):
    """(scale, ef, seed) of the serving mix: scale uniform in [min, max], EF in {8,16,32}."""
    specs = []
    for g in range(count):
        s = seed + g
        scale = min_scale + u64(s, 0) % (max_scale - min_scale + 1)
        ef = (8, 16, 32)[u64(s, 1) % 3]
        specs.append((int(scale), int(ef), s))
    return specs
