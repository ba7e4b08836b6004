"""Seeded synthetic RDF graphs with an RDFS vocabulary, for the entailment
rules of Sec. 5.7 (rules 2, 3, 5, 7, 9 and 11 of its rule table).

IDs 1..5 are rdf:type, rdfs:subClassOf, rdfs:subPropertyOf, rdfs:domain and
rdfs:range; then come the class IDs, the property IDs and the resource IDs.
The schema part holds a class hierarchy (each class below the roots has one
or two superclasses among the classes before it), a property hierarchy (a
share of the properties has a superproperty), and domain and range
declarations for a share of the properties.  The data part holds
(resource, property, resource) triples with Zipf-distributed subjects and
properties, and rdf:type triples for a share of the resources.  Rows are
shuffled.  The paper's data (BTC-2009) is not available; this stands in for
it with the same kinds of triples.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

TYPE, SUBCLASS, SUBPROP, DOMAIN, RANGE = 1, 2, 3, 4, 5
VOCAB = (TYPE, SUBCLASS, SUBPROP, DOMAIN, RANGE)
FIRST_FREE = 6


@dataclass(frozen=True)
class RdfsSpec:
    n_data: int = 200_000        # (resource, property, resource) triples
    n_classes: int = 2_000
    n_props: int = 500
    n_resources: int = 100_000
    typed_share: float = 0.5     # resources with an rdf:type triple
    subprop_share: float = 0.5
    domain_share: float = 0.3
    range_share: float = 0.3
    seed: int = 7


def _zipf_ids(rng, n_ids, count, s):
    w = np.arange(1, n_ids + 1, dtype=np.float64) ** -s
    return rng.choice(n_ids, size=count, p=w / w.sum())


def make_rdfs_graph(spec: RdfsSpec = RdfsSpec()) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([spec.seed, 0x5D75])))
    c0 = FIRST_FREE
    p0 = c0 + spec.n_classes
    r0 = p0 + spec.n_props
    rows = []
    # class hierarchy: class i > 4 has one or two superclasses among the classes before it
    for i in range(5, spec.n_classes):
        for _ in range(1 + int(rng.random() < 0.3)):
            rows.append((c0 + i, SUBCLASS, c0 + int(rng.integers(0, i))))
    # property hierarchy, domains and ranges
    for j in range(spec.n_props):
        if j > 2 and rng.random() < spec.subprop_share:
            rows.append((p0 + j, SUBPROP, p0 + int(rng.integers(0, j))))
        if rng.random() < spec.domain_share:
            rows.append((p0 + j, DOMAIN, c0 + int(rng.integers(0, spec.n_classes))))
        if rng.random() < spec.range_share:
            rows.append((p0 + j, RANGE, c0 + int(rng.integers(0, spec.n_classes))))
    schema = np.array(rows, dtype=np.uint32).reshape(-1, 3)
    # data: Zipf subjects and properties, uniform objects
    s = r0 + _zipf_ids(rng, spec.n_resources, spec.n_data, 1.0)
    p = p0 + _zipf_ids(rng, spec.n_props, spec.n_data, 1.1)
    o = r0 + rng.integers(0, spec.n_resources, spec.n_data)
    data = np.stack([s, p, o], axis=1).astype(np.uint32)
    typed = np.nonzero(rng.random(spec.n_resources) < spec.typed_share)[0]
    types = np.stack([r0 + typed, np.full(typed.size, TYPE),
                      c0 + _zipf_ids(rng, spec.n_classes, typed.size, 0.8)], axis=1)
    g = np.concatenate([schema, data, types.astype(np.uint32)])
    return g[rng.permutation(g.shape[0])]
