"""Off-diagonal elements <x| E(|psi><psi|) |y> and their level-l approximations.

The paper extends Problem 1 to every density-matrix element through the
polarization identity (Section III, after Problem 1): for any operator A,
    <x| A |y> = 1/4 sum_{k=0..3} i^k <v_k| A |v_k>,   v_k = y + i^k x,
so four diagonal-type values with the bond-2 targets v_k give one element,
and since every term of Algorithm 1 is linear in the target's outer product,
the same combination of the four level sums gives the element's level sums.

Routes here (x, y are product states, or the circuit's ideal outputs of
product states when ``output`` is set, as the circuit-output target of
Problem 1):
* ``element_exact`` / ``element_graded``: the density matrix of Section II and
  its graded form, <X| rho^(u) |Y> (small n);
* ``element_cross``: Algorithm 1's terms with the two targets in the two
  halves: a term is w_c <X|K_c psi> conj(<Y|K_c psi>), one ket network per
  target (``network.KetNetwork``), no polarization;
* ``sum2_circuit``: the circuit with the bond-2 target p + c q, for the
  polarization route (``dense.target_vector`` evaluates it densely).

Parity pinned by (tests/test_oracle_offdiag.py): the cross form equals the
graded density matrix level by level and the density-matrix element at level
N; x = y reduces to the diagonal estimate; Hermitian symmetry
<x|E|y> = conj(<y|E|x>); the polarization identity holds on the dense
matrices.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import dense, network, terms
from .estimate import Neumaier


def _target_circuit(circ, amps, output: bool):
    return dataclasses.replace(circ, target="circuit_output" if output else "product",
                               v=np.asarray(amps, dtype=np.complex128))


def sum2_circuit(circ, p, q, c, output: bool):
    """The circuit with target |p> + c|q> (p, q product amplitudes, n x 2), or
    U_ideal(|p> + c|q>) when ``output``."""
    flat = np.concatenate([np.asarray(p, dtype=np.complex128).reshape(-1),
                           np.asarray(q, dtype=np.complex128).reshape(-1), [complex(c)]])
    return dataclasses.replace(circ, target="circuit_output_sum2" if output else "sum2", v=flat)


def polarization_targets(x, y):
    """(p, q, c) of the four targets v_k = y + i^k x and the weights i^k / 4."""
    return [((y, x, 1j ** k), (1j ** k) / 4.0) for k in range(4)]


def element_exact(circ, x, y, output: bool) -> complex:
    X = dense.target_vector(_target_circuit(circ, x, output))
    Y = dense.target_vector(_target_circuit(circ, y, output))
    return complex(np.vdot(X, dense.exact_matrix(circ) @ Y))


def element_graded(circ, level: int, x, y, output: bool):
    X = dense.target_vector(_target_circuit(circ, x, output))
    Y = dense.target_vector(_target_circuit(circ, y, output))
    return [complex(np.vdot(X, m @ Y)) for m in dense.graded_matrices(circ, level)]


def element_cross(circ, level: int, x, y, output: bool, reduce: bool = True, diagonal: bool = False):
    """Level sums T_u and A(u) (complex) of <x|E|y> by the cross form
    (``diagonal``: diagonal gates as shared indices, same values)."""
    cx, cy = _target_circuit(circ, x, output), _target_circuit(circ, y, output)
    nx = network.KetNetwork(cx, reduce=reduce, diagonal=diagonal)
    ny = network.KetNetwork(cy, reduce=reduce, diagonal=diagonal)
    sp = network.slot_split(circ)
    level = min(level, circ.n_noises)
    re = [Neumaier() for _ in range(level + 1)]
    im = [Neumaier() for _ in range(level + 1)]
    vals = []
    for t in terms.enumerate_terms(circ.n_noises, level):
        w = 1.0
        mats = []
        for s, ch in enumerate(t):
            d, k, _ = sp[s]
            w *= d[ch]
            mats.append(k[ch])
        v = 0j if w == 0.0 else w * nx.value(mats) * np.conj(ny.value(mats))
        vals.append(v)
        u = terms.term_level(t)
        re[u].add(float(v.real))
        im[u].add(float(v.imag))
    tu = [complex(a.value, b.value) for a, b in zip(re, im)]
    ar, ai = Neumaier(), Neumaier()
    a = []
    for v in tu:
        ar.add(v.real)
        ai.add(v.imag)
        a.append(complex(ar.value, ai.value))
    return {"T": tu, "A": a, "values": np.array(vals)}
