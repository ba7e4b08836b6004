"""Seeded synthetic TripleID graphs.

A graph is an (N, 3) uint32 array of (subject, predicate, object) IDs in one
shared ID space starting at 1; 0 is reserved for the free variable (Sec. 3).
The paper's data sets (BTC-2009 and SP2Bench, Sec. 5.1 tables of data set
characteristics) are not available, so every workload is a synthetic stand-in
with independent columns drawn from bounded Zipf or uniform laws.

Sampling.  A column of `count` i.i.d. draws from a law over ranks 1..n is
produced as multinomial rank counts followed by a uniform random shuffle; the
result has exactly the distribution of i.i.d. draws, and is much faster in
numpy than inverse-CDF search over a large table.  Draws are made in chunks of
at most CHUNK rows, each chunk seeded from (seed, column, chunk index), so the
output does not depend on the machine.  Ranks map to IDs by identity for
subjects and predicates (rank 1 is the most frequent ID) and through a seeded
bijection of [1, n] for objects, so that the hub object is not also the hub
subject.
"""
from __future__ import annotations

import hashlib
import json
import os
from dataclasses import dataclass, field, replace

import numpy as np

CHUNK = 1 << 26


@dataclass(frozen=True)
class ColSpec:
    dist: str          # "uniform" or "zipf"
    n_ids: int         # law over ranks 1..n_ids
    exponent: float = 0.0
    permute: bool = False


@dataclass(frozen=True)
class GraphSpec:
    name: str
    n: int
    seed: int
    s: ColSpec
    p: ColSpec
    o: ColSpec

    def with_n(self, n: int) -> "GraphSpec":
        """Same laws, fewer or more triples (for tests at reduced size)."""
        return replace(self, n=int(n))

    def as_dict(self) -> dict:
        d = {"name": self.name, "n": self.n, "seed": self.seed}
        for k in ("s", "p", "o"):
            c = getattr(self, k)
            d[k] = {"dist": c.dist, "n_ids": c.n_ids, "exponent": c.exponent,
                    "permute": c.permute}
        return d


CONFIGS = {
    # 100k triples; s ~ U[1,1e4], p ~ U[1,50], o ~ Zipf(1.1) over 2e4.
    "small": GraphSpec("small", 100_000, 1,
                       ColSpec("uniform", 10_000),
                       ColSpec("uniform", 50),
                       ColSpec("zipf", 20_000, 1.1, True)),
    # 50M triples; s Zipf(1.0)/5e6, p Zipf(1.2)/1e3, o Zipf(1.1)/1e7.
    "medium": GraphSpec("medium", 50_000_000, 2,
                        ColSpec("zipf", 5_000_000, 1.0),
                        ColSpec("zipf", 1_000, 1.2),
                        ColSpec("zipf", 10_000_000, 1.1, True)),
    # 500M triples; same laws scaled to 5e7 subjects, 1e8 objects.
    "large": GraphSpec("large", 500_000_000, 3,
                       ColSpec("zipf", 50_000_000, 1.0),
                       ColSpec("zipf", 1_000, 1.2),
                       ColSpec("zipf", 100_000_000, 1.1, True)),
    # 200M triples for the batched workload (laws between medium and large).
    "batched": GraphSpec("batched", 200_000_000, 4,
                         ColSpec("zipf", 20_000_000, 1.0),
                         ColSpec("zipf", 1_000, 1.2),
                         ColSpec("zipf", 40_000_000, 1.1, True)),
    # 1B triples for the serving workload.
    "serving": GraphSpec("serving", 1_000_000_000, 5,
                         ColSpec("zipf", 100_000_000, 1.0),
                         ColSpec("zipf", 1_000, 1.2),
                         ColSpec("zipf", 200_000_000, 1.1, True)),
}


def zipf_weights(n: int, s: float) -> np.ndarray:
    """P(r) proportional to r**-s for r = 1..n, normalised (float64)."""
    r = np.arange(1, n + 1, dtype=np.float64)
    w = r ** (-float(s))
    return w / w.sum()


def _rank_counts(rng: np.random.Generator, col: ColSpec, count: int) -> np.ndarray:
    if col.dist == "uniform":
        pv = None
    elif col.dist == "zipf":
        pv = zipf_weights(col.n_ids, col.exponent)
    else:
        raise ValueError(f"unknown law {col.dist!r}")
    if pv is None:
        return rng.multinomial(count, np.full(col.n_ids, 1.0 / col.n_ids))
    return rng.multinomial(count, pv)


def _col_ids(spec: GraphSpec, which: int, col: ColSpec) -> np.ndarray:
    ids = np.arange(1, col.n_ids + 1, dtype=np.uint32)
    if col.permute:
        prng = np.random.Generator(np.random.PCG64(
            np.random.SeedSequence([spec.seed, which, 0xB1])))
        ids = prng.permutation(ids)
    return ids


def _chunk_values(spec: GraphSpec, which: int, col: ColSpec, ids: np.ndarray, ci: int,
                  cnt: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([spec.seed, which, ci])))
    if col.dist == "uniform":
        ranks = rng.integers(1, col.n_ids + 1, size=cnt, dtype=np.int64)
        return ids[ranks - 1]
    counts = _rank_counts(rng, col, cnt)
    vals = np.repeat(ids, counts)
    rng.shuffle(vals)
    return vals


def _draw_column(spec: GraphSpec, which: int, col: ColSpec, out: np.ndarray) -> None:
    ids = _col_ids(spec, which, col)
    for ci, start in enumerate(range(0, spec.n, CHUNK)):
        cnt = min(CHUNK, spec.n - start)
        out[start:start + cnt] = _chunk_values(spec, which, col, ids, ci, cnt)


def _worker(args):
    """Fill one (column, chunk) of a shared-memory graph (process pool)."""
    shm_name, n, spec, which, ci = args
    from multiprocessing import shared_memory
    shm = shared_memory.SharedMemory(name=shm_name)
    try:
        g = np.ndarray((n, 3), dtype=np.uint32, buffer=shm.buf)
        col = (spec.s, spec.p, spec.o)[which]
        start = ci * CHUNK
        cnt = min(CHUNK, n - start)
        g[start:start + cnt, which] = _chunk_values(spec, which, col, _col_ids(spec, which, col),
                                                    ci, cnt)
        del g
    finally:
        shm.close()
    return ci


def _gpu_initialised() -> bool:
    import sys
    torch = sys.modules.get("torch")
    try:
        return bool(torch is not None and torch.cuda.is_initialized())
    except Exception:  # noqa: BLE001
        return True


def make_graph(spec: GraphSpec, workers: int | None = None) -> np.ndarray:
    """Return the (N, 3) uint32 row-major triple array for `spec`.

    Each (column, chunk) is drawn from its own seed, so the result is the
    same whether chunks are drawn in one process or by a pool of forked
    workers (used for graphs of more than two chunks).  A process that has
    already initialised a GPU draws serially, so no GPU state is forked."""
    nchunks = (spec.n + CHUNK - 1) // CHUNK
    if workers is None:
        workers = min(16, os.cpu_count() or 1)
    if _gpu_initialised():
        workers = 1
    if nchunks <= 2 or workers <= 1:
        g = np.empty((spec.n, 3), dtype=np.uint32)
        for which, col in enumerate((spec.s, spec.p, spec.o)):
            tmp = np.empty(spec.n, dtype=np.uint32)
            _draw_column(spec, which, col, tmp)
            g[:, which] = tmp
            del tmp
        return g
    from concurrent.futures import ProcessPoolExecutor
    from multiprocessing import get_context, shared_memory
    shm = shared_memory.SharedMemory(create=True, size=spec.n * 12)
    try:
        jobs = [(shm.name, spec.n, spec, which, ci) for which in range(3) for ci in range(nchunks)]
        with ProcessPoolExecutor(max_workers=workers, mp_context=get_context("fork")) as ex:
            list(ex.map(_worker, jobs))
        g = np.empty((spec.n, 3), dtype=np.uint32)
        g[:] = np.ndarray((spec.n, 3), dtype=np.uint32, buffer=shm.buf)
    finally:
        shm.close()
        shm.unlink()
    return g


def save_tid(path: str, g: np.ndarray, spec: GraphSpec | None = None) -> dict:
    """Write the raw TripleID file (N x 12 bytes, little-endian, no header)
    and a JSON manifest beside it with the SHA-256 of the bytes."""
    g = np.ascontiguousarray(g, dtype="<u4")
    raw = g.tobytes()
    with open(path, "wb") as f:
        f.write(raw)
    man = {"n": int(g.shape[0]), "sha256": hashlib.sha256(raw).hexdigest(),
           "spec": spec.as_dict() if spec else None}
    with open(path + ".json", "w") as f:
        json.dump(man, f, indent=1)
    return man


def load_tid(path: str) -> np.ndarray:
    raw = np.fromfile(path, dtype="<u4")
    if raw.size % 3:
        raise ValueError(f"{path}: size is not a multiple of 12 bytes")
    return raw.reshape(-1, 3)
