"""Exact betweenness centrality (Brandes; arXiv:1602.00963 heuristics) on
one AMD Instinct MI355X, behind the C ABI of include/bc.h."""
from .bc import (BCError, Context, Graph, Server, lib, make_opts, prune_deg1_host,  # noqa: F401
                 coverage_host, prune_trees_host, validate_csr, vertex_order_host)
