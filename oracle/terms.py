"""Term enumeration of the level-l approximation (Section IV, Algorithm 1).

A term is a tuple c of length N (one entry per noise, in circuit order);
c[s] = 0 means noise s is replaced by U_0 (x) V_0, c[s] = i in {1,2,3} means it
is replaced by U_i (x) V_i.  Level u collects the terms with exactly u non-zero
entries.  Order (the order Algorithm 1 loops in): level u ascending; inside a
level the position sets p_1 < ... < p_u in lexicographic order; inside a
position set the corrections (i_1..i_u) in {1,2,3}^u in lexicographic order.

Parity pinned by: brute force over all 4^N patterns, and the count
sum_{u<=l} C(N,u) 3^u of Theorem 1 (tests/test_oracle_terms.py).
"""
from __future__ import annotations

import itertools
import math
from typing import Iterator, List, Tuple


def enumerate_level(n_noise: int, u: int) -> Iterator[Tuple[int, ...]]:
    for pos in itertools.combinations(range(n_noise), u):
        for corr in itertools.product((1, 2, 3), repeat=u):
            c = [0] * n_noise
            for p, i in zip(pos, corr):
                c[p] = i
            yield tuple(c)


def enumerate_terms(n_noise: int, level: int) -> List[Tuple[int, ...]]:
    out: List[Tuple[int, ...]] = []
    for u in range(min(level, n_noise) + 1):
        out.extend(enumerate_level(n_noise, u))
    return out


def term_level(c) -> int:
    return sum(1 for x in c if x != 0)


def count_terms(n_noise: int, level: int) -> int:
    return sum(math.comb(n_noise, u) * 3 ** u for u in range(min(level, n_noise) + 1))
