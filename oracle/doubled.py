"""Exact value of Problem 1 by contracting the doubled network (any n).

The paper's exact baseline ("accuracy algorithm", Section IV around Fig. 2)
contracts one network holding both the ket and the bra of the density
matrix: every gate G acts on the ket wires and conj(G) on the bra wires, and
every noise is its full 4 x 4 superoperator M = sum_k E_k (x) conj(E_k)
(Section III), a tensor joining a ket wire and its bra wire.  Its value is
<v| E(|psi><psi|) |v> with no approximation.

Here the doubled network is the ket network of ``network.KetNetwork`` (the
same light-cone reduction when the target is the circuit's own output: a gate
with no noise in its causal future cancels on the ket side and, conjugated,
on the bra side), its complex conjugate as the bra half on fresh edge ids, and
at every noise slot the tensor
    T[ko, ki, bo, bi] = sum_k E_k[ko, ki] conj(E_k[bo, bi])
from the Kraus matrices themselves (no SVD).  Contracted pairwise by the
oracle's own greedy order, in complex128.

Parity pinned by (tests/test_oracle_doubled.py): the dense density-matrix
value ``dense.exact_value`` on small circuits of every target kind and
channel, the closed form of one depolarizing qubit, and the full expansion
A(N) of Algorithm 1 at level N (every term).
"""
from __future__ import annotations

import numpy as np

from . import network


def superoperator_tensor(kraus) -> np.ndarray:
    """T[ko, ki, bo, bi] = sum_k E_k[ko, ki] conj(E_k[bo, bi])."""
    e = np.asarray(kraus, dtype=np.complex128).reshape(-1, 2, 2)
    return np.einsum("kab,kcd->abcd", e, e.conj())


def bra_tensor(t) -> np.ndarray:
    """A tensor of the bra half: the complex conjugate of its ket tensor."""
    return np.conj(t)


def doubled_network(circ, reduce: bool = True, diagonal: bool = False):
    """(arrays, legs, scalar) of the doubled network of ``circ``."""
    net = network.KetNetwork(circ, reduce=reduce, diagonal=diagonal)
    kraus = [op.kraus for op in circ.noise_ops()]
    top = 1 + max((e for _, lg in net.tensors for e in lg), default=-1)
    arrs, legs = [], []
    slot_legs = {}
    for t, lg in net.tensors:
        if isinstance(t, tuple):
            slot_legs[t[1]] = list(lg)
            continue
        arrs.append(t)
        legs.append(list(lg))
        arrs.append(bra_tensor(t))
        legs.append([e + top for e in lg])
    for s, lg in sorted(slot_legs.items()):
        ko, ki = lg
        arrs.append(superoperator_tensor(kraus[s]))
        legs.append([ko, ki, ko + top, ki + top])
    scalar = net.scalar * np.conj(net.scalar)
    return arrs, legs, scalar


def doubled_value(circ, reduce: bool = True, diagonal: bool = False) -> complex:
    """Value of the doubled network (real up to rounding)."""
    arrs, legs, scalar = doubled_network(circ, reduce=reduce, diagonal=diagonal)
    if diagonal:
        path = network.hyper_greedy_path(legs)
        return complex(scalar * network.contract_hyper(arrs, legs, path))
    path = network.greedy_path(legs)
    return complex(scalar * network.contract_path(arrs, legs, path))
