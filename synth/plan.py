"""Plain descriptions of triple patterns and postfix query plans.

A triple pattern holds one ID per position (subject, predicate, object); 0
marks a free variable (Sec. 3).  Each free position may name a variable by a
non-negative integer id; positions that share an id must hold equal values,
and each distinct id becomes one output column, in s, p, o order.  A free
position with id -1 is unconstrained and not projected.  An optional half-open
ID range [lo, hi) may be attached to one position.

A plan is a list of patterns plus a postfix op stream of int32 words:

  OP_SCAN i               push the bindings of pattern i
  OP_JOIN v               pop R, pop L, push the inner join of L and R on
                          variable v (other shared variables must agree)
  OP_UNION k d            pop k tables, push their union (d=1: distinct)
  OP_FILTER v lo hi       keep rows whose variable v lies in [lo, hi)
  OP_PROJECT n v1 .. vn   keep the listed variables, in that order
  OP_DISTINCT             drop duplicate rows
  OP_OPTIONAL v           pop R, pop L, push the left outer join of L and R on
                          variable v (SPARQL OPTIONAL; L and R share no other
                          variable); R's cells of an L row with no partner are 0

The final result is always returned in lexicographic row order.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Sequence

OP_SCAN = 1
OP_JOIN = 2
OP_UNION = 3
OP_FILTER = 4
OP_PROJECT = 5
OP_DISTINCT = 6
OP_OPTIONAL = 7

UINT32_MAX = 0xFFFFFFFF


@dataclass(frozen=True)
class Pattern:
    s: int = 0
    p: int = 0
    o: int = 0
    vs: int = -1
    vp: int = -1
    vo: int = -1
    range_pos: int = -1
    lo: int = 0
    hi: int = 0

    def __post_init__(self):
        for k in (self.s, self.p, self.o, self.lo, self.hi):
            if not (0 <= int(k) <= UINT32_MAX):
                raise ValueError(f"ID {k} out of uint32 range")
        for c, v in ((self.s, self.vs), (self.p, self.vp), (self.o, self.vo)):
            if c != 0 and v != -1:
                raise ValueError("a bound position cannot name a variable")
            if v < -1:
                raise ValueError("variable ids are >= -1")
        if self.range_pos not in (-1, 0, 1, 2):
            raise ValueError("range_pos must be -1, 0, 1 or 2")

    @property
    def consts(self):
        return (self.s, self.p, self.o)

    @property
    def vars(self):
        return (self.vs, self.vp, self.vo)

    def out_vars(self) -> List[int]:
        """Distinct named variables in s, p, o order (the output schema)."""
        out: List[int] = []
        for v in self.vars:
            if v >= 0 and v not in out:
                out.append(v)
        return out


def pat(text: str, names: dict | None = None, range_pos: int = -1,
        lo: int = 0, hi: int = 0) -> Pattern:
    """Build a Pattern from text such as "?s 7 ?o" or "? 3 ?".

    "?name" names a variable (ids are assigned through `names`, which is
    updated in place); a bare "?" is an unprojected free position; digits are
    constant IDs."""
    if names is None:
        names = {}
    toks = text.split()
    if len(toks) != 3:
        raise ValueError(f"pattern needs three terms: {text!r}")
    consts, vars_ = [], []
    for t in toks:
        if t == "?":
            consts.append(0)
            vars_.append(-1)
        elif t.startswith("?"):
            if t not in names:
                names[t] = len(names)
            consts.append(0)
            vars_.append(names[t])
        else:
            consts.append(int(t))
            vars_.append(-1)
    return Pattern(*consts, *vars_, range_pos=range_pos, lo=lo, hi=hi)


@dataclass
class Plan:
    patterns: List[Pattern] = field(default_factory=list)
    ops: List[int] = field(default_factory=list)

    # builder helpers -------------------------------------------------
    def scan(self, p: Pattern) -> "Plan":
        self.patterns.append(p)
        self.ops += [OP_SCAN, len(self.patterns) - 1]
        return self

    def join(self, var: int) -> "Plan":
        self.ops += [OP_JOIN, var]
        return self

    def union(self, k: int, dedupe: bool) -> "Plan":
        self.ops += [OP_UNION, k, int(bool(dedupe))]
        return self

    def filter(self, var: int, lo: int, hi: int) -> "Plan":
        self.ops += [OP_FILTER, var, lo, hi]
        return self

    def project(self, vars_: Sequence[int]) -> "Plan":
        self.ops += [OP_PROJECT, len(vars_), *vars_]
        return self

    def optional(self, var: int) -> "Plan":
        self.ops += [OP_OPTIONAL, var]
        return self

    def distinct(self) -> "Plan":
        self.ops += [OP_DISTINCT]
        return self

    # plain-data form (query-mix files) --------------------------------
    def to_dict(self) -> dict:
        return {"patterns": [[p.s, p.p, p.o, p.vs, p.vp, p.vo, p.range_pos, p.lo, p.hi]
                             for p in self.patterns],
                "ops": [int(x) for x in self.ops]}

    @staticmethod
    def from_dict(d: dict) -> "Plan":
        return Plan([Pattern(*map(int, p)) for p in d["patterns"]], [int(x) for x in d["ops"]])
