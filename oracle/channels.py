"""Channel representation and the SVD split of a noise superoperator (FP64).

Parity pinned by: the printed permutation of the 2-qubit identity (Section IV,
Fig. 3a), reconstruction M = sum_i U_i (x) V_i (Section IV), Lemmas 1 and 2 as
properties, closed forms of depolarizing / amplitude damping / phase damping
(tests/test_oracle_channels.py).
"""
from __future__ import annotations

import numpy as np


def superoperator(kraus) -> np.ndarray:
    """Matrix representation M = sum_k E_k (x) conj(E_k) (Section III).

    Row index (a, b) = 2a + b, a the ket index and b the bra index, so that
    M vec(rho) = vec(sum_k E_k rho E_k^dagger) with row-major vec."""
    m = np.zeros((4, 4), dtype=np.complex128)
    for e in kraus:
        e = np.asarray(e, dtype=np.complex128)
        m += np.kron(e, e.conj())
    return m


def tp_residual(kraus) -> float:
    """Spectral norm of sum_k E_k^dagger E_k - I (trace preservation,
    Section II)."""
    s = np.zeros((2, 2), dtype=np.complex128)
    for e in kraus:
        e = np.asarray(e, dtype=np.complex128)
        s += e.conj().T @ e
    return float(np.linalg.norm(s - np.eye(2), 2))


def permute(m: np.ndarray) -> np.ndarray:
    """Tensor permutation of Fig. 3a: M has edges (1,2) as rows and (3,4) as
    columns; the permuted matrix has edges (1,3) as rows and (2,4) as columns,
    i.e. Mt[(a,c),(b,d)] = M[(a,b),(c,d)]."""
    return np.asarray(m).reshape(2, 2, 2, 2).transpose(0, 2, 1, 3).reshape(4, 4)


def svd_split(m: np.ndarray):
    """SVD split of Section IV / Fig. 3b-c.

    Mt = S D T^dagger with d descending (LAPACK).  Ut_i = d_i S|i>,
    Vt_i = T|i>, so Mt = sum_i Ut_i Vt_i^dagger.  Permuting back gives
    M = sum_i U_i (x) V_i with U_i[a,c] = Ut_i[(a,c)] and
    V_i[b,d] = conj(Vt_i[(b,d)]).

    Returns (d[4], U[4,2,2], V[4,2,2])."""
    mt = permute(m)
    s, d, th = np.linalg.svd(mt)
    t = th.conj().T
    u = np.zeros((4, 2, 2), dtype=np.complex128)
    v = np.zeros((4, 2, 2), dtype=np.complex128)
    for i in range(4):
        u[i] = (d[i] * s[:, i]).reshape(2, 2)
        v[i] = t[:, i].conj().reshape(2, 2)
    return d, u, v


def reconstruct(u: np.ndarray, v: np.ndarray, idx=range(4)) -> np.ndarray:
    """sum over i in idx of U_i (x) V_i."""
    out = np.zeros((4, 4), dtype=np.complex128)
    for i in idx:
        out += np.kron(u[i], v[i])
    return out


def noise_rate(m: np.ndarray) -> float:
    """||M - I||_2, the noise rate defined in Section IV."""
    return float(np.linalg.norm(np.asarray(m) - np.eye(4), 2))


def apply_superop(m: np.ndarray, rho: np.ndarray) -> np.ndarray:
    """M acting on a 2x2 density matrix through row-major vec."""
    return (np.asarray(m) @ np.asarray(rho).reshape(4)).reshape(2, 2)
