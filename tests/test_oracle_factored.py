"""Pins of the oracle's factored level sums (independent parts of the network).

Independent of the factoring: Algorithm 1's global enumeration
(``estimate.estimate``), the stored full-enumeration sums of the 225-qubit
workload, and the density-matrix value at level N.
"""
import dataclasses
import os

import numpy as np
import pytest

import workloads as W
from oracle import dense, estimate, factored, network

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def two_blocks(seed, n1=3, n2=3, kind="random"):
    """Two tiny random circuits on disjoint qubits: the network splits."""
    rng = np.random.default_rng(seed)
    a = W.tiny_random_circuit(rng, n1, 10, 3, noise=kind, level=2)
    b = W.tiny_random_circuit(rng, n2, 10, 2, noise=kind, level=2)
    ops = list(a.ops) + [dataclasses.replace(o, qubits=tuple(q + n1 for q in o.qubits)) for o in b.ops]
    return W.Circuit(n1 + n2, ops, np.concatenate([a.psi, b.psi]), "circuit_output",
                     np.concatenate([a.v, b.v]), 3)


@pytest.mark.parametrize("seed,kind", [(101, "random"), (102, "adpd"), (103, "depol")])
def test_factored_equals_global_enumeration(seed, kind):
    c = two_blocks(seed, kind=kind)
    assert len(factored.parts(network.KetNetwork(c, diagonal=True))) >= 2
    f = factored.factored_levels(c, 4)
    g = estimate.estimate(c, 4, "network")
    for u in range(5):
        assert abs(f["A"][u] - g["A"][u]) <= 1e-13, (u, f["A"][u], g["A"][u])


def test_factored_full_level_equals_density_matrix():
    c = two_blocks(104)
    f = factored.factored_levels(c, c.n_noises)
    assert abs(f["A"][-1] - dense.exact_value(c)) <= 1e-12


def test_factored_config5_equals_stored_full_sums():
    c = W.config(5)
    f = factored.factored_levels(c, 3)
    gold = np.loadtxt(os.path.join(GOLD, "config5_oracle.txt"))
    assert len(f["g"]) >= 2
    for u in range(4):
        assert abs(f["A"][u] - gold[u]) <= 1e-13 * gold[u], (u, f["A"][u], gold[u])


def test_dropped_cross_terms_are_caught():
    # summing the parts' corrections instead of multiplying their polynomials
    # misses the products of corrections in different parts (from level 2 on)
    c = two_blocks(105)
    f = factored.factored_levels(c, 2)
    x0 = f["A"][0]
    additive = x0 * (1 + sum(g[1] / g[0] for g in f["g"] if len(g) > 1) + sum(g[2] / g[0] for g in f["g"] if len(g) > 2))
    assert abs(additive - f["A"][2]) > 1e-10
