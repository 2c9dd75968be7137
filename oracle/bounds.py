"""Theorem 1: contraction count and error bounds.

* ``contraction_count``: 2 sum_{i<=l} C(N,i) 3^i, two networks per term.
* ``paper_bound``: the theorem's printed bound
  (1+8p)^N - sum_{i<=l} C(N,i) (4p)^i (1+4p)^(N-i).
* ``rigorous_bound``: what the proof's own chain establishes once each factor
  is bounded by its actual norm: the remainder F - A(l) is the sum over noise
  subsets S with |S| > l of products with Mbar_s on S and M'_s elsewhere, and
  unitary superoperators have norm 1, so
  |F - A(l)| <= sum_{|S|>l} prod_{s in S} ||Mbar_s|| prod_{s not in S} ||M'_s||.
  Computed with the generating polynomial prod_s (||M'_s|| + x ||Mbar_s||).
  (The printed constants use ||M'|| <= 1 + 4p, which Lemma 2 does not give;
  this form avoids that step.)
"""
from __future__ import annotations

import math

import numpy as np

from . import channels


def contraction_count(n_noise: int, level: int) -> int:
    return 2 * sum(math.comb(n_noise, i) * 3 ** i for i in range(min(level, n_noise) + 1))


def paper_bound(n_noise: int, level: int, p: float) -> float:
    tail = sum(math.comb(n_noise, i) * (4 * p) ** i * (1 + 4 * p) ** (n_noise - i)
               for i in range(min(level, n_noise) + 1))
    return (1 + 8 * p) ** n_noise - tail


def split_norms(kraus):
    d, u, v = channels.svd_split(channels.superoperator(kraus))
    main = np.linalg.norm(np.kron(u[0], v[0]), 2)
    bar = np.linalg.norm(channels.reconstruct(u, v, (1, 2, 3)), 2)
    return float(main), float(bar)


def rigorous_bound(norms, level: int) -> float:
    """norms: list of (||M'_s||, ||Mbar_s||)."""
    poly = np.array([1.0])
    for a, b in norms:
        poly = np.convolve(poly, np.array([a, b]))
    return float(np.sum(poly[level + 1:]))
