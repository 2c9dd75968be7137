"""Pins of the oracle's term enumeration (Algorithm 1 loops; Theorem 1 count)."""
import itertools
import math
import os

import numpy as np
import pytest

from oracle import bounds, terms

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def brute_force(n_noise, level):
    pats = [p for p in itertools.product(range(4), repeat=n_noise)
            if sum(1 for x in p if x) <= level]

    def key(p):
        pos = tuple(i for i, x in enumerate(p) if x)
        cor = tuple(x for x in p if x)
        return (len(pos), pos, cor)
    return sorted(pats, key=key)


@pytest.mark.parametrize("n,l", [(1, 1), (3, 0), (3, 2), (4, 1), (4, 2), (4, 4), (5, 3), (6, 2)])
def test_enumeration_matches_brute_force(n, l):
    assert terms.enumerate_terms(n, l) == brute_force(n, l)


@pytest.mark.parametrize("n,l,t", [(4, 1, 13), (4, 2, 67), (4, 4, 256), (10, 1, 31), (10, 2, 436),
                                   (10, 3, 3676), (20, 2, 1771), (20, 3, 32551)])
def test_term_counts(n, l, t):
    assert terms.count_terms(n, l) == t
    if n <= 10:
        assert len(terms.enumerate_terms(n, l)) == t


def test_fig5_contraction_counts():
    rows = np.loadtxt(os.path.join(GOLD, "fig5_counts.txt"), dtype=np.int64)
    assert len(rows) == 31
    for n, cnt in rows:
        assert bounds.contraction_count(int(n), 1) == cnt


def test_full_level_has_every_pattern_once():
    for n in range(1, 6):
        t = terms.enumerate_terms(n, n)
        assert len(t) == 4 ** n == len(set(t))


def test_level_is_clamped_to_noise_count():
    assert terms.enumerate_terms(3, 7) == terms.enumerate_terms(3, 3)
    assert terms.count_terms(3, 7) == 64
    assert math.comb(3, 0) == 1
