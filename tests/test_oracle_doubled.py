"""Pins of the oracle's doubled-network contraction (the exact baseline).

What fixes the answer independently of the doubled network:
* the dense density-matrix evolution of Section II (``dense.exact_value``);
* one depolarizing qubit: <0| E(|0><0|) |0> = 1 - 2p/3 (Kraus sqrt(1-p) I,
  sqrt(p/3) X, Y, Z); one amplitude-damping qubit: <1| E(|1><1|) |1> = 1 - g;
* the full expansion A(N) of Algorithm 1 (every term), which is exact.
Planted slips (a bra half left unconjugated, a superoperator without its
conjugate, transposed superoperator legs) must break these pins.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import dense, doubled, estimate


def tiny(seed, n=3, gates=10, noise=3, kind="random", target="circuit_output"):
    rng = np.random.default_rng(seed)
    return W.tiny_random_circuit(rng, n, gates, noise, noise=kind, level=1, target=target)


CASES = [(21, "random", "circuit_output"), (22, "adpd", "product"), (23, "depol", "dense"),
         (24, "random", "product"), (25, "random", "dense"), (26, "adpd", "circuit_output")]


@pytest.mark.parametrize("seed,kind,target", CASES)
@pytest.mark.parametrize("reduce", [True, False])
def test_doubled_equals_density_matrix(seed, kind, target, reduce):
    c = tiny(seed, n=4, gates=14, noise=5, kind=kind, target=target)
    f = dense.exact_value(c)
    val = doubled.doubled_value(c, reduce=reduce)
    assert abs(val.real - f) <= 1e-12 * max(1.0, abs(f))
    assert abs(val.imag) <= 1e-12


@pytest.mark.parametrize("seed,target", [(31, "circuit_output"), (32, "product")])
def test_doubled_with_diagonal_hyperedges(seed, target):
    c = tiny(seed, n=5, gates=20, noise=6, kind="random", target=target)
    f = dense.exact_value(c)
    assert abs(doubled.doubled_value(c, diagonal=True).real - f) <= 1e-12 * max(1.0, abs(f))


def _one_qubit(kraus, state):
    psi = np.array([state], dtype=np.complex128)
    return W.Circuit(1, [W.Op("noise", (0,), kraus=kraus)], psi, "product", psi.copy(), 1)


@pytest.mark.parametrize("p", [0.0, 0.01, 0.3, 0.75])
def test_one_depolarizing_qubit_closed_form(p):
    c = _one_qubit(W.kraus_depolarizing(p), [1.0, 0.0])
    assert math.isclose(doubled.doubled_value(c).real, 1.0 - 2.0 * p / 3.0, rel_tol=0, abs_tol=1e-15)


@pytest.mark.parametrize("g", [0.05, 0.5])
def test_one_amplitude_damping_qubit_closed_form(g):
    c = _one_qubit(W.kraus_ad_pd(g, 0.0), [0.0, 1.0])
    assert math.isclose(doubled.doubled_value(c).real, 1.0 - g, rel_tol=0, abs_tol=1e-15)


def test_doubled_equals_full_expansion():
    c = tiny(41, n=4, gates=16, noise=5, kind="random", target="circuit_output")
    r = estimate.estimate(c, 5, "network")
    assert abs(doubled.doubled_value(c).real - r["A"][-1]) <= 1e-12


def test_doubled_on_config1():
    c = W.config(1)
    f = dense.exact_value(c)
    assert abs(doubled.doubled_value(c).real - f) <= 1e-12


def _pins_hold():
    for seed, kind, target in CASES[:3]:
        c = tiny(seed, n=3, gates=10, noise=3, kind=kind, target=target)
        if abs(doubled.doubled_value(c).real - dense.exact_value(c)) > 1e-10:
            return False
    c = _one_qubit(W.kraus_depolarizing(0.3), [1.0, 0.0])
    return abs(doubled.doubled_value(c).real - 0.8) <= 1e-12


def test_unpatched_doubled_passes_the_pins():
    assert _pins_hold()


def test_superoperator_without_conjugate_is_caught(monkeypatch):
    def wrong(kraus):
        e = np.asarray(kraus, dtype=np.complex128).reshape(-1, 2, 2)
        return np.einsum("kab,kcd->abcd", e, e)
    monkeypatch.setattr(doubled, "superoperator_tensor", wrong)
    assert not _pins_hold()


def test_transposed_superoperator_legs_are_caught(monkeypatch):
    right = doubled.superoperator_tensor
    monkeypatch.setattr(doubled, "superoperator_tensor", lambda k: right(k).transpose(1, 0, 3, 2))
    assert not _pins_hold()


def test_unconjugated_bra_half_is_caught(monkeypatch):
    monkeypatch.setattr(doubled, "bra_tensor", lambda t: np.asarray(t))
    assert not _pins_hold()
