"""Level sums by factoring the ket network over independent clusters.

When the (light-cone reduced) ket network falls into independent connected
parts, a term's amplitude is the product of the parts' amplitudes and its
weight the product of the parts' singular values, so X = |s|^2 prod_c X_c (s
the factor of the qubits the network no longer touches) and the level sums of
Algorithm 1 are the coefficients of a product of per-part polynomials:
    A(l) = |s|^2 sum_{k<=l} [prod_c g_c](k),
    g_c(k) = sum over the part's own patterns with k corrections of
             (prod_{s in c} d_{c_s}) |a_c|^2.
Each part is contracted on its own (its tensors only, one greedy order per
part), once per local pattern, in complex128.

Parity pinned by (tests/test_oracle_factored.py): the global enumeration of
``estimate.estimate`` on circuits that split into several parts, the stored
full-enumeration sums of the 225-qubit workload, and the density-matrix value
at level N.
"""
from __future__ import annotations

import itertools

import numpy as np

from . import network, terms
from .estimate import Neumaier


def parts(net: network.KetNetwork):
    """Connected parts of the network: lists of tensor indices (shared legs)."""
    n = len(net.tensors)
    parent = list(range(n))

    def find(i):
        while parent[i] != i:
            parent[i] = parent[parent[i]]
            i = parent[i]
        return i

    owner = {}
    for i, (_, legs) in enumerate(net.tensors):
        for e in legs:
            if e in owner:
                parent[find(i)] = find(owner[e])
            else:
                owner[e] = i
    groups = {}
    for i in range(n):
        groups.setdefault(find(i), []).append(i)
    return [groups[k] for k in sorted(groups)]


def _part_path(net, idx):
    legs = [list(net.tensors[i][1]) for i in idx]
    return network.hyper_greedy_path(legs, trials=1) if net.diagonal else network.greedy_path(legs)


def _part_value(net, idx, path, slot_mats):
    arrs, legs = [], []
    for i in idx:
        t, lg = net.tensors[i]
        arrs.append(np.asarray(slot_mats[t[1]], dtype=np.complex128) if isinstance(t, tuple) else t)
        legs.append(list(lg))
    if net.diagonal:
        return network.contract_hyper(arrs, legs, path)
    return network.contract_path(arrs, legs, path)


def factored_levels(circ, level: int, diagonal: bool = True):
    """{"g": per-part level polynomials, "A": A(0..level)}."""
    net = network.KetNetwork(circ, diagonal=diagonal)
    sp = network.slot_split(circ)
    level = min(level, circ.n_noises)
    poly = np.zeros(level + 1)
    poly[0] = abs(net.scalar) ** 2
    gs = []
    for idx in parts(net):
        slots = sorted(net.tensors[i][0][1] for i in idx if isinstance(net.tensors[i][0], tuple))
        g = [Neumaier() for _ in range(level + 1)]
        path = _part_path(net, idx)
        for k in range(min(level, len(slots)) + 1):
            for pos in itertools.combinations(range(len(slots)), k):
                for corr in itertools.product((1, 2, 3), repeat=k):
                    mats = {}
                    w = 1.0
                    for j, s in enumerate(slots):
                        ch = corr[pos.index(j)] if j in pos else 0
                        d, kk, _ = sp[s]
                        w *= d[ch]
                        mats[s] = kk[ch]
                    if w == 0.0:
                        continue
                    a = _part_value(net, idx, path, mats)
                    g[k].add(w * (a.real * a.real + a.imag * a.imag))
        gv = np.array([x.value for x in g])
        gs.append(gv)
        new = np.zeros(level + 1)
        for a in range(level + 1):
            for b in range(level + 1 - a):
                new[a + b] += poly[a] * gv[b]
        poly = new
    acc = Neumaier()
    A = []
    for v in poly:
        acc.add(float(v))
        A.append(acc.value)
    return {"g": gs, "A": A, "level": level}
