"""Python binding of libbc (exact betweenness centrality on one MI355X).

Argument marshalling only: every step of the computation runs in the HIP
library.  torch provides device memory (caller workspaces, device score
outputs) and streams.  Importing this module never falls back to anything:
if libbc.so is missing or cannot load, it raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbc.so")

# status codes (include/bc.h)
OK, E_INVALID_ARG, E_INVALID_GRAPH, E_OUT_OF_MEMORY, E_DEVICE, E_BUSY, E_NOT_FOUND, E_TIMEOUT, E_REJECTED, \
    E_CAPACITY = range(10)
LOAD_VALIDATE, LOAD_PRUNE_DEG1, LOAD_DEVICE_PTRS, LOAD_KEEP_ORDER, LOAD_PRUNE_TREES, LOAD_ORDER_RCM = 1, 2, 4, 8, 16, 32
MODE_PLAIN, MODE_BATCHED, MODE_PLAIN_SCAN, MODE_PER_WORKGROUP, MODE_AUTO = 0, 1, 2, 3, 4
MODE_NAMES = {MODE_PLAIN: "plain", MODE_BATCHED: "batched", MODE_PLAIN_SCAN: "plain_scan",
              MODE_PER_WORKGROUP: "per_workgroup", MODE_AUTO: "auto"}
H_DEG1, H_DEG2 = 1, 2
SIGMA_AUTO, SIGMA_EXACT_ONLY, SIGMA_EXTENDED = 0, 1, 2
RAW, UNDIRECTED = 0, 1

EXPORTED = ["bc_context_create", "bc_context_destroy", "bc_graph_load", "bc_graph_stats_get", "bc_graph_free",
            "bc_workspace_size", "bc_compute", "bc_scores", "bc_scores_reset", "bc_trace", "bc_validate_csr",
            "bc_prune_deg1_host", "bc_server_create", "bc_server_destroy", "bc_submit", "bc_wait",
            "bc_status_string", "bc_last_error", "bc_autotune", "bc_compute_noalloc",
            "bc_server_stats_get", "bc_prune_trees_host", "bc_coverage_host", "bc_vertex_order_host"]


class GraphStats(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int64) for f in ("n", "m", "nnz", "isolated", "pendants", "k2_vertices",
                                                 "residual_nnz", "deg2_vertices", "max_degree", "resident_bytes",
                                                 "tree_vertices", "bfs_depth", "tuned_batch")]


class ComputeOpts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("batch", ctypes.c_int32), ("heuristics", ctypes.c_uint32),
                ("sigma_mode", ctypes.c_int32), ("alpha", ctypes.c_double), ("block", ctypes.c_int32),
                ("grid_per_cu", ctypes.c_int32), ("beta", ctypes.c_double), ("graph_launches", ctypes.c_int32)]


class RunStats(ctypes.Structure):
    _fields_ = [("sources", ctypes.c_int64), ("traversed", ctypes.c_int64), ("derived", ctypes.c_int64),
                ("overflowed", ctypes.c_int64), ("rerun_extended", ctypes.c_int64),
                ("first_overflow", ctypes.c_int32 * 8), ("levels", ctypes.c_int64),
                ("bottom_up_levels", ctypes.c_int64), ("reached", ctypes.c_int64), ("reached_nnz", ctypes.c_int64),
                ("dag_edges", ctypes.c_int64), ("launches", ctypes.c_int64), ("te", ctypes.c_double),
                ("raw_te", ctypes.c_double), ("ms", ctypes.c_double), ("kernel_ms", ctypes.c_double),
                ("mode", ctypes.c_int64)]

    def as_dict(self) -> dict:
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["first_overflow"] = [x for x in self.first_overflow if x >= 0]
        d["mode"] = MODE_NAMES.get(self.mode, str(self.mode))
        return d


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_int64), ("max_inflight", ctypes.c_int32),
                ("batch", ctypes.c_int32), ("queue_capacity", ctypes.c_int32), ("heuristics", ctypes.c_uint32)]


class ServerStats(ctypes.Structure):
    _fields_ = [("workers", ctypes.c_int32), ("grid_workgroups", ctypes.c_int32),
                ("max_inflight_seen", ctypes.c_int32), ("batches", ctypes.c_int64), ("mean_inflight", ctypes.c_double),
                ("busy_ms", ctypes.c_double), ("held_bytes", ctypes.c_int64), ("reclaims", ctypes.c_int64),
                ("allocations", ctypes.c_int64), ("wide_batches", ctypes.c_int64), ("mean_shares", ctypes.c_double)]


class QueryStats(ctypes.Structure):
    _fields_ = [("submit_ms", ctypes.c_double), ("start_ms", ctypes.c_double), ("end_ms", ctypes.c_double),
                ("latency_ms", ctypes.c_double), ("sources", ctypes.c_int64), ("te", ctypes.c_double),
                ("status", ctypes.c_int32)]


_lib = None


def lib():
    """Load libbc.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        # One HIP runtime per process: torch bundles its own libamdhip64
        # (same soname as the system one).  Loading torch first makes the
        # dynamic linker bind libbc to that copy, so torch tensors, streams
        # and events and this library share one runtime.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1602_00963_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
        sig = {
            "bc_context_create": [ctypes.c_int, vp],
            "bc_context_destroy": [vp],
            "bc_graph_load": [vp, i32, vp, vp, i64, u32, vp],
            "bc_graph_stats_get": [vp, vp],
            "bc_graph_free": [vp],
            "bc_workspace_size": [vp, vp, vp],
            "bc_compute": [vp, vp, i64, vp, vp, ctypes.c_size_t, vp, vp],
            "bc_scores": [vp, vp, i32, i32],
            "bc_scores_reset": [vp],
            "bc_trace": [vp, vp, i64, vp, vp, vp, vp, vp, vp, vp],
            "bc_validate_csr": [i32, vp, vp, i64],
            "bc_prune_deg1_host": [i32, vp, vp, vp, vp, vp, vp, vp, vp],
            "bc_server_create": [vp, vp, vp],
            "bc_server_destroy": [vp],
            "bc_submit": [vp, vp, vp, i64, vp, vp],
            "bc_wait": [vp, ctypes.c_uint64, i64, vp],
            "bc_autotune": [vp, vp, i64, vp, ctypes.c_double, vp],
            "bc_compute_noalloc": [vp, vp, i64, vp, vp, vp],
            "bc_server_stats_get": [vp, vp],
            "bc_prune_trees_host": [i32, vp, vp, vp, i64, vp, vp, vp, vp],
            "bc_coverage_host": [i32, vp, vp, u32, u32, vp],
            "bc_vertex_order_host": [i32, vp, vp, u32, vp, vp],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.bc_status_string.argtypes = [ctypes.c_int]
        L.bc_status_string.restype = ctypes.c_char_p
        L.bc_last_error.argtypes = []
        L.bc_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


class BCError(RuntimeError):
    def __init__(self, status: int, where: str):
        L = lib()
        msg = L.bc_last_error().decode(errors="replace")
        super().__init__(f"{where}: {L.bc_status_string(status).decode()} ({msg})")
        self.status = status


def _check(st: int, where: str):
    if st != OK:
        raise BCError(st, where)


def _p(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _i32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def validate_csr(n: int, row_ptr, col_idx) -> None:
    rp, ci = _i32(row_ptr), _i32(col_idx)
    _check(lib().bc_validate_csr(n, _p(rp), _p(ci), int(rp[-1]) if len(rp) else 0), "bc_validate_csr")


def prune_deg1_host(n: int, row_ptr, col_idx) -> dict:
    rp, ci = _i32(row_ptr), _i32(col_idx)
    omega, kind, hub = (np.zeros(n, np.int32) for _ in range(3))
    rrp = np.zeros(n + 1, np.int32)
    rci = np.zeros(max(len(ci), 1), np.int32)
    rnnz = ctypes.c_int64(0)
    _check(lib().bc_prune_deg1_host(n, _p(rp), _p(ci), _p(omega), _p(kind), _p(hub), _p(rrp), _p(rci),
                                    ctypes.byref(rnnz)), "bc_prune_deg1_host")
    return {"omega": omega, "kind": kind, "hub": hub, "row_ptr": rrp, "col_idx": rci[:rnnz.value].copy()}


def prune_trees_host(n: int, row_ptr, col_idx, sources=None) -> dict:
    """The iterated 1-degree reduction on the host: omega, kind and the
    closed-form scores of the removed vertices for `sources` (None = all)."""
    rp, ci = _i32(row_ptr), _i32(col_idx)
    src = None if sources is None else _i32(sources)
    omega, kind = np.zeros(n, np.int32), np.zeros(n, np.int32)
    sc = np.zeros(n, np.float64)
    rnnz = ctypes.c_int64(0)
    _check(lib().bc_prune_trees_host(n, _p(rp), _p(ci), _p(src), 0 if src is None else len(src), _p(omega),
                                     _p(kind), _p(sc), ctypes.byref(rnnz)), "bc_prune_trees_host")
    return {"omega": omega, "kind": kind, "scores": sc, "residual_nnz": rnnz.value}


def coverage_host(n: int, row_ptr, col_idx, prune=False, deg1=False, deg2=False) -> dict:
    """Heuristics coverage over all sources (host only): sources, sweeps
    traversed, sources served by the 1-degree reduction, sources derived by
    the 2-degree heuristic, degree-2 traversal sources."""
    rp, ci = _i32(row_ptr), _i32(col_idx)
    lf = LOAD_PRUNE_TREES if prune == "trees" else (LOAD_PRUNE_DEG1 if prune else 0)
    out = np.zeros(5, np.int64)
    _check(lib().bc_coverage_host(n, _p(rp), _p(ci), lf, (H_DEG1 if deg1 else 0) | (H_DEG2 if deg2 else 0),
                                  _p(out)), "bc_coverage_host")
    return dict(zip(["sources", "traversed", "one_degree", "two_degree", "deg2_candidates"], (int(x) for x in out)))


def vertex_order_host(n: int, row_ptr, col_idx, order: str = "degree"):
    """The internal vertex order the library would load the graph in (host
    only): perm[v] = internal id of vertex v, for order "degree", "rcm" or
    "keep"; and the BFS depth from a highest-degree vertex."""
    rp, ci = _i32(row_ptr), _i32(col_idx)
    lf = {"degree": 0, "rcm": LOAD_ORDER_RCM, "keep": LOAD_KEEP_ORDER}[order]
    perm = np.zeros(n, np.int32)
    depth = ctypes.c_int64(0)
    _check(lib().bc_vertex_order_host(n, _p(rp), _p(ci), lf, _p(perm), ctypes.byref(depth)), "bc_vertex_order_host")
    return perm, int(depth.value)


class Context:
    def __init__(self, device: int = 0):
        self.h = ctypes.c_void_p()
        _check(lib().bc_context_create(device, ctypes.byref(self.h)), "bc_context_create")
        self.device = device

    def close(self):
        if self.h:
            lib().bc_context_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_opts(mode="batched", batch=256, deg1=False, deg2=False, sigma="auto", alpha=0.0, grid_per_cu=0, beta=0.0,
              graph_launches=0):
    o = ComputeOpts()
    o.mode = {v: k for k, v in MODE_NAMES.items()}[mode]
    o.batch = batch
    o.heuristics = (H_DEG1 if deg1 else 0) | (H_DEG2 if deg2 else 0)
    o.sigma_mode = {"auto": SIGMA_AUTO, "exact": SIGMA_EXACT_ONLY, "extended": SIGMA_EXTENDED}[sigma]
    o.alpha = alpha
    o.block = 0
    o.grid_per_cu = grid_per_cu
    o.beta = beta
    o.graph_launches = graph_launches
    return o


def _stream_handle(stream):
    if stream is None:
        return None
    return ctypes.c_void_p(int(stream.cuda_stream))


class Graph:
    """A graph resident in HBM.  `g` is anything with n, row_ptr, col_idx."""

    def __init__(self, ctx: Context, g, validate: bool = True, prune=False, keep_order: bool = False,
                 order: str = "degree"):
        """prune: False, True (one round of the 1-degree reduction) or "trees"
        (the reduction iterated until no degree-1 vertex is left); order: the
        internal vertex order, "degree" (decreasing degree) or "rcm" (reverse
        Cuthill-McKee, for long-diameter graphs); keep_order keeps the
        caller's."""
        self.ctx = ctx
        self.n = int(g.n)
        self.rp = _i32(g.row_ptr)
        self.ci = _i32(g.col_idx)
        flags = (LOAD_VALIDATE if validate else 0) | (LOAD_KEEP_ORDER if keep_order else 0)
        if order not in ("degree", "rcm"):
            raise ValueError(f"unknown vertex order {order!r}")
        if order == "rcm":
            flags |= LOAD_ORDER_RCM
        if prune == "trees":
            flags |= LOAD_PRUNE_TREES
        elif prune:
            flags |= LOAD_PRUNE_DEG1
        self.h = ctypes.c_void_p()
        _check(lib().bc_graph_load(ctx.h, self.n, _p(self.rp), _p(self.ci), int(self.rp[-1]), flags,
                                   ctypes.byref(self.h)), "bc_graph_load")

    def stats(self) -> dict:
        s = GraphStats()
        _check(lib().bc_graph_stats_get(self.h, ctypes.byref(s)), "bc_graph_stats_get")
        return {f: getattr(s, f) for f, _ in s._fields_}

    def workspace_size(self, **opts) -> int:
        o = make_opts(**opts)
        b = ctypes.c_size_t(0)
        _check(lib().bc_workspace_size(self.h, ctypes.byref(o), ctypes.byref(b)), "bc_workspace_size")
        return b.value

    def compute(self, sources=None, workspace=None, stream=None, **opts) -> dict:
        """Adds the RAW contributions of `sources` (None = all) to the scores.
        `workspace`: optional torch uint8 device tensor of workspace_size()
        bytes; `stream`: optional torch.cuda.Stream."""
        o = make_opts(**opts)
        st = RunStats()
        if sources is None:
            src, k = None, self.n
        else:
            src = _i32(sources)
            k = len(src)
        ws_ptr = ctypes.c_void_p(workspace.data_ptr()) if workspace is not None else None
        ws_bytes = workspace.numel() if workspace is not None else 0
        _check(lib().bc_compute(self.h, _p(src), k, ctypes.byref(o), ws_ptr, ws_bytes, _stream_handle(stream),
                                ctypes.byref(st)), "bc_compute")
        return st.as_dict()

    def compute_noalloc(self, sources=None, stream=None, **opts) -> dict:
        """compute() in the plain form through the entry point that makes no
        device allocation (workspace = the library's fixed scratch array)."""
        opts.setdefault("mode", "plain")
        o = make_opts(**opts)
        st = RunStats()
        if sources is None:
            src, k = None, self.n
        else:
            src = _i32(sources)
            k = len(src)
        _check(lib().bc_compute_noalloc(self.h, _p(src), k, ctypes.byref(o), _stream_handle(stream),
                                        ctypes.byref(st)), "bc_compute_noalloc")
        return st.as_dict()

    def autotune(self, sample, budget_ms: float = 0.0, **opts) -> dict:
        """Tune the batched mode on `sample` (scores untouched); later
        compute() calls with batch=0 use the result."""
        o = make_opts(**opts)
        src = _i32(sample)
        gt = ctypes.c_double(0.0)
        _check(lib().bc_autotune(self.h, _p(src), len(src), ctypes.byref(o), budget_ms, ctypes.byref(gt)),
               "bc_autotune")
        return {"batch": o.batch, "alpha": o.alpha, "beta": o.beta, "grid_per_cu": o.grid_per_cu, "gteps": gt.value}

    def scores(self, norm: str = "raw", out=None) -> np.ndarray:
        """Accumulated scores; `out` may be a torch float64 device tensor."""
        nv = {"raw": RAW, "undirected": UNDIRECTED}[norm]
        if out is not None:
            _check(lib().bc_scores(self.h, ctypes.c_void_p(out.data_ptr()), nv, 1), "bc_scores")
            return out
        a = np.zeros(self.n, np.float64)
        _check(lib().bc_scores(self.h, _p(a), nv, 0), "bc_scores")
        return a

    def reset(self) -> None:
        _check(lib().bc_scores_reset(self.h), "bc_scores_reset")

    def trace(self, sources, **opts) -> dict:
        """Per-source d, sigma (exact form), sigma significand/exponent,
        delta and overflow flags, computed by the chosen mode."""
        o = make_opts(**opts)
        src = _i32(sources)
        k, n = len(src), self.n
        d = np.zeros((k, n), np.int32)
        sig = np.zeros((k, n), np.uint64)
        sm = np.zeros((k, n), np.float64)
        se = np.zeros((k, n), np.int32)
        dl = np.zeros((k, n), np.float64)
        ovf = np.zeros(k, np.int32)
        _check(lib().bc_trace(self.h, _p(src), k, ctypes.byref(o), _p(d), _p(sig), _p(sm), _p(se), _p(dl), _p(ovf)),
               "bc_trace")
        return {"d": d, "sigma": sig, "sigma_mant": sm, "sigma_exp": se, "delta": dl, "overflow": ovf.astype(bool)}

    def close(self):
        if self.h:
            lib().bc_graph_free(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class Ticket:
    id: int
    out: np.ndarray


class Server:
    """Continuous-batching query server (see bc_server_create)."""

    def __init__(self, ctx: Context, hbm_budget_bytes: int = 0, max_inflight: int = 0, batch: int = 0,
                 queue_capacity: int = 0, deg1: bool = False):
        c = ServerConfig(hbm_budget_bytes, max_inflight, batch, queue_capacity, H_DEG1 if deg1 else 0)
        self.h = ctypes.c_void_p()
        _check(lib().bc_server_create(ctx.h, ctypes.byref(c), ctypes.byref(self.h)), "bc_server_create")

    def submit(self, graph: Graph, sources) -> Ticket:
        src = _i32(sources)
        out = np.zeros(graph.n, np.float64)
        t = ctypes.c_uint64(0)
        _check(lib().bc_submit(self.h, graph.h, _p(src), len(src), _p(out), ctypes.byref(t)), "bc_submit")
        return Ticket(t.value, out)

    def wait(self, ticket: Ticket, timeout_us: int = -1) -> dict:
        qs = QueryStats()
        st = lib().bc_wait(self.h, ticket.id, timeout_us, ctypes.byref(qs))
        d = {f: getattr(qs, f) for f, _ in qs._fields_}
        _check(st, "bc_wait")
        return d

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib().bc_server_stats_get(self.h, ctypes.byref(st)), "bc_server_stats_get")
        return {f: getattr(st, f) for f, _ in st._fields_}

    def close(self):
        if self.h:
            lib().bc_server_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
