"""Run the oracle on several plans at once, one host thread per plan.

The oracle is single-threaded C called through ctypes, which releases the
interpreter lock for the length of each call, so independent plans evaluate
in parallel on the host's cores; each result is exactly what a lone call
returns."""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import oracle


def oracle_queries(g, plans, workers=None):
    workers = workers or min(16, os.cpu_count() or 1, max(1, len(plans)))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(lambda p: oracle.query(g, p), plans))
