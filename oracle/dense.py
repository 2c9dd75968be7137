"""Exact references on dense matrices (small n only).

* ``exact_value``: the quantity of Problem 1, <v| E_N(|psi><psi|) |v>, by
  evolving the full density matrix: rho <- G rho G^dagger for a gate and
  rho <- sum_k E_k rho E_k^dagger for a noise (Section II).
* ``graded_levels``: every level sum T_u at once without enumerating terms.
  One density-like matrix rho^(k) is kept per correction count k <= l; at a
  noise with split M = sum_i U_i (x) V_i (Section IV),
      rho^(k) <- U_0 rho^(k) V_0^T + sum_{i>=1} U_i rho^(k-1) V_i^T,
  and every gate maps rho^(k) <- G rho^(k) G^dagger.  Then
  T_k = <v| rho^(k) |v>.  Expanding the product of the N sums M = M' + Mbar
  by the number of Mbar factors gives exactly the T_u of Section IV, so this
  is an enumeration-free reference for the level sums.
"""
from __future__ import annotations

import numpy as np

from . import channels


def product_state(amps: np.ndarray) -> np.ndarray:
    """Kronecker product of per-qubit amplitudes, qubit 0 most significant."""
    out = np.ones(1, dtype=np.complex128)
    for q in range(amps.shape[0]):
        out = np.kron(out, np.asarray(amps[q], dtype=np.complex128))
    return out


def apply_to_axes(t: np.ndarray, mat: np.ndarray, axes) -> np.ndarray:
    """Apply a (2^k x 2^k) matrix to k axes of a tensor with all dims 2."""
    k = len(axes)
    g = np.asarray(mat, dtype=np.complex128).reshape((2,) * (2 * k))
    out = np.tensordot(g, t, axes=(list(range(k, 2 * k)), list(axes)))
    return np.moveaxis(out, list(range(k)), list(axes))


def ideal_state(circ, start: np.ndarray) -> np.ndarray:
    """U_ideal |start> (noises removed), as a flat vector."""
    n = circ.n_qubits
    st = start.reshape((2,) * n)
    for op in circ.ops:
        if op.kind == "gate":
            st = apply_to_axes(st, op.mat, op.qubits)
    return st.reshape(-1)


def target_vector(circ) -> np.ndarray:
    """The target |v> as a dense vector."""
    if circ.target == "circuit_output":
        return ideal_state(circ, product_state(circ.v))
    if circ.target == "product":
        return product_state(circ.v)
    if circ.target == "dense":
        return np.asarray(circ.v, dtype=np.complex128).reshape(-1)
    if circ.target in ("sum2", "circuit_output_sum2"):
        # |p> + c |q>: v holds p (n x 2), q (n x 2), then c
        n = circ.n_qubits
        flat = np.asarray(circ.v, dtype=np.complex128).reshape(-1)
        p, q, c = flat[:2 * n].reshape(n, 2), flat[2 * n:4 * n].reshape(n, 2), flat[4 * n]
        st = product_state(p) + c * product_state(q)
        return ideal_state(circ, st) if circ.target == "circuit_output_sum2" else st
    raise ValueError(circ.target)


def exact_value(circ) -> float:
    """<v| E_N(|psi><psi|) |v> from the full 2^n x 2^n density matrix."""
    n = circ.n_qubits
    psi = product_state(circ.psi)
    rho = np.outer(psi, psi.conj()).reshape((2,) * (2 * n))
    for op in circ.ops:
        ket = list(op.qubits)
        bra = [n + q for q in op.qubits]
        if op.kind == "gate":
            rho = apply_to_axes(rho, op.mat, ket)
            rho = apply_to_axes(rho, np.conj(op.mat), bra)
        else:
            acc = np.zeros_like(rho)
            for e in op.kraus:
                t = apply_to_axes(rho, e, ket)
                acc += apply_to_axes(t, np.conj(e), bra)
            rho = acc
    v = target_vector(circ)
    rho = rho.reshape(2 ** n, 2 ** n)
    val = np.vdot(v, rho @ v)
    return float(val.real)


def graded_levels(circ, level: int):
    """[T_0, ..., T_level] by the graded density-matrix recursion."""
    n = circ.n_qubits
    vv = target_vector(circ)
    return [np.vdot(vv, m @ vv) for m in graded_matrices(circ, level)]


def graded_matrices(circ, level: int):
    """The graded density matrices rho^(0..level) as 2^n x 2^n arrays."""
    n = circ.n_qubits
    psi = product_state(circ.psi)
    rho0 = np.outer(psi, psi.conj()).reshape((2,) * (2 * n))
    grades = [rho0] + [np.zeros_like(rho0) for _ in range(level)]
    for op in circ.ops:
        ket = list(op.qubits)
        bra = [n + q for q in op.qubits]
        if op.kind == "gate":
            grades = [apply_to_axes(apply_to_axes(g, op.mat, ket), np.conj(op.mat), bra)
                      for g in grades]
        else:
            d, u, v = channels.svd_split(channels.superoperator(op.kraus))
            new = []
            for k in range(level + 1):
                acc = apply_to_axes(apply_to_axes(grades[k], u[0], ket), v[0], bra)
                if k >= 1:
                    for i in (1, 2, 3):
                        acc = acc + apply_to_axes(apply_to_axes(grades[k - 1], u[i], ket), v[i], bra)
                new.append(acc)
            grades = new
    return [g.reshape(2 ** n, 2 ** n) for g in grades]


def exact_matrix(circ) -> np.ndarray:
    """E_N(|psi><psi|) as a 2^n x 2^n array (Kraus evolution, Section II)."""
    n = circ.n_qubits
    psi = product_state(circ.psi)
    rho = np.outer(psi, psi.conj()).reshape((2,) * (2 * n))
    for op in circ.ops:
        ket = list(op.qubits)
        bra = [n + q for q in op.qubits]
        if op.kind == "gate":
            rho = apply_to_axes(apply_to_axes(rho, op.mat, ket), np.conj(op.mat), bra)
        else:
            acc = np.zeros_like(rho)
            for e in op.kraus:
                acc += apply_to_axes(apply_to_axes(rho, e, ket), np.conj(e), bra)
            rho = acc
    return rho.reshape(2 ** n, 2 ** n)
