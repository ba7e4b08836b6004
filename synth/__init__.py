"""Seeded synthetic inputs shared by the oracle side and the GPU side.

This package holds input generators and plain query descriptions only:
graphs of dictionary-encoded triples (the TripleID form of Sec. 3), triple
patterns with 0 standing for a free variable (Sec. 3), and postfix query
plans.  It computes no scan, join, union, filter or ordering result.
"""
from .graph import (ColSpec, GraphSpec, CONFIGS, make_graph, zipf_weights,
                    save_tid, load_tid)
from .plan import (Pattern, Plan, OP_SCAN, OP_JOIN, OP_UNION, OP_FILTER,
                   OP_PROJECT, OP_DISTINCT, OP_OPTIONAL, pat)

__all__ = [
    "ColSpec", "GraphSpec", "CONFIGS", "make_graph", "zipf_weights",
    "save_tid", "load_tid", "Pattern", "Plan", "OP_SCAN", "OP_JOIN",
    "OP_UNION", "OP_FILTER", "OP_PROJECT", "OP_DISTINCT", "OP_OPTIONAL", "pat",
]
