"""Quantum-trajectories estimate of Problem 1 with one tensor network per sample.

The paper's main comparison (Section V, Fig. 5 / Table III) is the quantum
trajectories method: each noise is replaced by one of its Kraus operators,
drawn at random, and the value is averaged over samples.  Written here for
networks: noise s draws Kraus index k with the state-independent probability
    q_{s,k} = tr(E_k^dagger E_k) / 2        (sum_k q_{s,k} = 1 by Section II),
and a sample's network carries E_k / sqrt(q_{s,k}) at slot s; its score is
X = |<v| ... |psi>|^2.  Then E[X] = sum over all index choices of
prod_s q_{s,k_s} |<v| prod E_{k_s} / sqrt(q_{s,k_s}) |psi>|^2
= sum_k |<v| E_k... |psi>|^2 = <v| E(|psi><psi|) |v>: the mean is unbiased.

The uniforms that drive the draws are inputs (one per sample and noise): index
k is the first with u < q_{s,0} + ... + q_{s,k} over the Kraus operators with
q > 0.

Parity pinned by (tests/test_oracle_trajectories.py): the q-weighted sum of
X over every index choice equals the density-matrix value (exact, no
sampling); the draw frequencies follow q; a long run's mean lies within its
standard error band of the exact value.
"""
from __future__ import annotations

import itertools

import numpy as np

from . import network


def probabilities(kraus) -> np.ndarray:
    e = np.asarray(kraus, dtype=np.complex128).reshape(-1, 2, 2)
    return np.real(np.einsum("kab,kab->k", e.conj(), e)) / 2.0


def draw(q: np.ndarray, u: float) -> int:
    acc = 0.0
    last = 0
    for k, qk in enumerate(q):
        if qk <= 0.0:
            continue
        acc += qk
        last = k
        if u < acc:
            return k
    return last


def sample_indices(circ, uniforms: np.ndarray) -> np.ndarray:
    """(n_samples, n_noise) Kraus indices from (n_samples, n_noise) uniforms."""
    qs = [probabilities(op.kraus) for op in circ.noise_ops()]
    out = np.zeros(uniforms.shape, dtype=np.int8)
    for i in range(uniforms.shape[0]):
        for s, q in enumerate(qs):
            out[i, s] = draw(q, float(uniforms[i, s]))
    return out


def sample_value(net: network.KetNetwork, circ, idx) -> float:
    mats = []
    for s, op in enumerate(circ.noise_ops()):
        q = probabilities(op.kraus)
        k = int(idx[s])
        mats.append(np.asarray(op.kraus[k], dtype=np.complex128) / np.sqrt(q[k]))
    a = net.value(mats)
    return float(a.real * a.real + a.imag * a.imag)


def estimate(circ, uniforms: np.ndarray, diagonal: bool = True):
    """{"X": per-sample scores, "mean": their mean, "stderr": standard error}."""
    net = network.KetNetwork(circ, diagonal=diagonal)
    idx = sample_indices(circ, uniforms)
    xs = np.array([sample_value(net, circ, row) for row in idx])
    return {"X": xs, "idx": idx, "mean": float(xs.mean()),
            "stderr": float(xs.std(ddof=1) / np.sqrt(len(xs))) if len(xs) > 1 else float("nan")}


def expectation(circ) -> float:
    """sum over every index choice of prod q * X (the estimator's mean, exactly)."""
    net = network.KetNetwork(circ)
    qs = [probabilities(op.kraus) for op in circ.noise_ops()]
    tot = 0.0
    for idx in itertools.product(*[range(len(q)) for q in qs]):
        p = float(np.prod([q[k] for q, k in zip(qs, idx)]))
        if p > 0.0:
            tot += p * sample_value(net, circ, idx)
    return tot
