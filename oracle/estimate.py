"""Algorithm 1 end to end: level sums T_u and the approximations A(l') for l' <= l.

For u = 0..l, every term of level u is evaluated (``literal`` = both networks
as dense state vectors, or ``network`` = one network per term) and summed into
T_u in enumeration order with Neumaier's compensated summation; A(l') is the
compensated sum of T_0..T_l'.  ``exact`` is the full density-matrix value
(small n only).
"""
from __future__ import annotations

import math
from typing import Optional

import numpy as np

from . import dense, literal, network, terms


class Neumaier:
    """Neumaier's variant of Kahan summation."""

    def __init__(self):
        self.s = 0.0
        self.c = 0.0

    def add(self, x: float):
        t = self.s + x
        if abs(self.s) >= abs(x):
            self.c += (self.s - t) + x
        else:
            self.c += (x - t) + self.s
        self.s = t

    @property
    def value(self) -> float:
        return self.s + self.c


def estimate(circ, level: Optional[int] = None, method: str = "network",
             term_list=None, reduce: bool = True):
    """Returns dict with keys terms, X (float64 per term), T (per level),
    A (cumulative per level), method."""
    if level is None:
        level = circ.level
    n_noise = circ.n_noises
    level = min(level, n_noise)
    tl = terms.enumerate_terms(n_noise, level) if term_list is None else list(term_list)
    xs = np.zeros(len(tl), dtype=np.float64)
    if method == "literal":
        sp = literal.splits(circ)
        for j, t in enumerate(tl):
            x, _, _ = literal.term_value(circ, t, sp)
            xs[j] = x.real
    elif method == "network":
        net = network.KetNetwork(circ, reduce=reduce)
        sp = network.slot_split(circ)
        for j, t in enumerate(tl):
            xs[j], _ = network.term_value(net, sp, t)
    else:
        raise ValueError(method)
    sums = [Neumaier() for _ in range(level + 1)]
    for t, x in zip(tl, xs):
        sums[terms.term_level(t)].add(float(x))
    tu = [s.value for s in sums]
    acc = Neumaier()
    a = []
    for v in tu:
        acc.add(v)
        a.append(acc.value)
    return {"terms": tl, "X": xs, "T": tu, "A": a, "method": method, "level": level}


def exact(circ) -> float:
    return dense.exact_value(circ)
