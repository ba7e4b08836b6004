"""Tiny dictionary encoder: string triples -> TripleID rows (Sec. 3).

TEST INFRASTRUCTURE ONLY.  The paper converts an N-Triples file into ID
dictionaries and a binary file of 32-bit (SubjID, PredID, ObjID) rows in one
linear pass, with hash tables mapping keys to values (Sec. 3, Fig. 1).  Here
IDs are handed out from 1 in order of first appearance while the triples are
read left to right, s then p then o; 0 stays reserved for "?".

shared=True  one dictionary for all positions (the reading used throughout,
             so that joins may pair any two positions, Table 3);
shared=False one dictionary per position, as the paper's three ID files.
"""
from __future__ import annotations

from typing import Dict, Iterable, List, Sequence, Tuple

import numpy as np


def encode_graph(triples: Iterable[Sequence[str]], shared: bool = True
                 ) -> Tuple[np.ndarray, List[Dict[str, int]]]:
    """Return (rows, dictionaries).  With shared=True the three dictionaries
    are the same object."""
    if shared:
        d: Dict[str, int] = {}
        dicts = [d, d, d]
    else:
        dicts = [{}, {}, {}]
    rows = []
    for t in triples:
        if len(t) != 3:
            raise ValueError(f"not a triple: {t!r}")
        row = []
        for pos, term in enumerate(t):
            dd = dicts[pos]
            if term not in dd:
                dd[term] = len(dd) + 1
            row.append(dd[term])
        rows.append(row)
    arr = np.array(rows, dtype=np.uint32).reshape(-1, 3)
    return arr, dicts


def decode_row(row: Sequence[int], dicts: List[Dict[str, int]], positions: Sequence[int]
               ) -> Tuple[str, ...]:
    """Map IDs back to terms through the dictionary of each row value's position."""
    inv = [{v: k for k, v in d.items()} for d in dicts]
    return tuple(inv[pos][int(x)] for x, pos in zip(row, positions))
