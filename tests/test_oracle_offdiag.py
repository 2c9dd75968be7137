"""Pins of the oracle's off-diagonal elements <x| E(|psi><psi|) |y>.

Independent of the cross form: the density matrix of Section II and its
graded recursion; the diagonal estimate (x = y); Hermitian symmetry; the
polarization identity on dense matrices (which also fixes the bond-2 target
vectors |p> + c|q> and the order of x and y in v_k = y + i^k x).
"""
import numpy as np
import pytest

import workloads as W
from oracle import dense, estimate, offdiag


def tiny(seed, n=4, gates=14, noise=4, kind="random", target="circuit_output"):
    rng = np.random.default_rng(seed)
    return W.tiny_random_circuit(rng, n, gates, noise, noise=kind, level=2, target=target)


def rand_product(rng, n):
    z = rng.standard_normal((n, 2)) + 1j * rng.standard_normal((n, 2))
    return z / np.linalg.norm(z, axis=1, keepdims=True)


CASES = [(71, "random", True), (72, "adpd", False), (73, "depol", True), (74, "random", False)]


@pytest.mark.parametrize("seed,kind,output", CASES)
def test_cross_form_equals_graded_density_matrix(seed, kind, output):
    c = tiny(seed, kind=kind)
    rng = np.random.default_rng(seed + 100)
    x, y = rand_product(rng, c.n_qubits), rand_product(rng, c.n_qubits)
    g = offdiag.element_graded(c, 3, x, y, output)
    r = offdiag.element_cross(c, 3, x, y, output)
    for u in range(4):
        assert abs(r["T"][u] - g[u]) <= 1e-12, (u, r["T"][u], g[u])


@pytest.mark.parametrize("seed,kind,output", CASES[:2])
def test_full_expansion_equals_density_matrix_element(seed, kind, output):
    c = tiny(seed, kind=kind)
    rng = np.random.default_rng(seed + 200)
    x, y = rand_product(rng, c.n_qubits), rand_product(rng, c.n_qubits)
    r = offdiag.element_cross(c, c.n_noises, x, y, output)
    assert abs(r["A"][-1] - offdiag.element_exact(c, x, y, output)) <= 1e-12


def test_equal_targets_give_the_diagonal_estimate():
    c = tiny(75, kind="adpd")
    r = offdiag.element_cross(c, 2, c.v, c.v, True)
    e = estimate.estimate(c, 2, "network")
    for u in range(3):
        assert abs(r["A"][u] - e["A"][u]) <= 1e-13


def test_hermitian_symmetry():
    c = tiny(76, kind="random", target="product")
    rng = np.random.default_rng(176)
    x, y = rand_product(rng, c.n_qubits), rand_product(rng, c.n_qubits)
    a = offdiag.element_cross(c, 2, x, y, False)["A"]
    b = offdiag.element_cross(c, 2, y, x, False)["A"]
    assert all(abs(p - np.conj(q)) <= 1e-14 for p, q in zip(a, b))


def _polarized(c, x, y, output, swap=False):
    tot = np.zeros(3, dtype=np.complex128)
    for (p, q, cc), wt in offdiag.polarization_targets(y, x) if swap else offdiag.polarization_targets(x, y):
        tot += wt * np.array(dense.graded_levels(offdiag.sum2_circuit(c, p, q, cc, output), 2))
    return tot


@pytest.mark.parametrize("output", [True, False])
def test_polarization_identity_on_the_graded_matrices(output):
    c = tiny(77, kind="random")
    rng = np.random.default_rng(177)
    x, y = rand_product(rng, c.n_qubits), rand_product(rng, c.n_qubits)
    want = offdiag.element_graded(c, 2, x, y, output)
    got = _polarized(c, x, y, output)
    assert np.allclose(got, want, rtol=0, atol=1e-13)
    # the roles of x and y matter: the swapped targets give the conjugate element
    assert not np.allclose(_polarized(c, x, y, output, swap=True), want, rtol=0, atol=1e-6)
    exact = sum(wt * dense.exact_value(offdiag.sum2_circuit(c, p, q, cc, output))
                for (p, q, cc), wt in offdiag.polarization_targets(x, y))
    assert abs(exact - offdiag.element_exact(c, x, y, output)) <= 1e-13


def test_cross_form_with_diagonal_hyperedges_is_the_same():
    c = tiny(78, n=5, gates=20, noise=4, kind="random")
    rng = np.random.default_rng(178)
    x, y = rand_product(rng, c.n_qubits), rand_product(rng, c.n_qubits)
    a = offdiag.element_cross(c, 2, x, y, True)["A"]
    b = offdiag.element_cross(c, 2, x, y, True, diagonal=True)["A"]
    assert np.allclose(a, b, rtol=0, atol=1e-14)
