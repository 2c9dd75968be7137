"""Algorithm 1 taken literally, for small n.

For one term c: every noise s is replaced by U_{c_s} (x) V_{c_s} (Section IV).
The doubled network then splits into a ket network (gates G, slot tensors
U_{c_s}, input |psi>, output <v|) and a bra network (gates conj(G), slot
tensors V_{c_s}, input |psi*>, output <v*|); both are contracted here as dense
state-vector simulations and multiplied (Algorithm 1, "contract both tensor
networks, and multiply").
"""
from __future__ import annotations

import numpy as np

from . import channels, dense


def splits(circ):
    """(d, U, V) for each noise of the circuit, in circuit order."""
    out = []
    for op in circ.noise_ops():
        out.append(channels.svd_split(channels.superoperator(op.kraus)))
    return out


def term_value(circ, term, split=None):
    """(X, a, b): X = a * b with a the ket and b the bra network value."""
    if split is None:
        split = splits(circ)
    n = circ.n_qubits
    ket = dense.product_state(circ.psi).reshape((2,) * n)
    bra = dense.product_state(circ.psi).conj().reshape((2,) * n)
    s = 0
    for op in circ.ops:
        if op.kind == "gate":
            ket = dense.apply_to_axes(ket, op.mat, op.qubits)
            bra = dense.apply_to_axes(bra, np.conj(op.mat), op.qubits)
        else:
            d, u, v = split[s]
            i = term[s]
            ket = dense.apply_to_axes(ket, u[i], op.qubits)
            bra = dense.apply_to_axes(bra, v[i], op.qubits)
            s += 1
    vv = dense.target_vector(circ)
    a = np.vdot(vv, ket.reshape(-1))            # <v| ...
    b = np.sum(vv * bra.reshape(-1))            # <v*| ... = v^T ...
    return a * b, a, b
