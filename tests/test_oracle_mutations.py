"""Planted mistakes in the oracle must be caught by its pins.

Each case patches one oracle function with a plausible slip (wrong axis order,
a missing conjugate, a dropped term, a transposed operand) and checks that at
least one of the independent pins fails.  The patch lives only inside the test.
"""
import numpy as np
import pytest

import workloads as W
from oracle import channels, dense, estimate, literal, network, terms


def pins_hold():
    """A compact selection of the pins; False as soon as one fails."""
    printed = np.array([[1, 0, 0, 1], [0, 0, 0, 0], [0, 0, 0, 0], [1, 0, 0, 1]], dtype=float)
    if not np.array_equal(channels.permute(np.eye(4)).real, printed):
        return False
    rng = np.random.default_rng(7)
    for nk in (2, 4):
        kr = W.random_isometry_kraus(rng, nk)
        m = channels.superoperator(kr)
        d, u, v = channels.svd_split(m)
        if np.linalg.norm(channels.reconstruct(u, v) - m) > 1e-12:
            return False
    if len(terms.enumerate_terms(4, 2)) != 67:
        return False
    c = W.tiny_random_circuit(np.random.default_rng(8), 3, 10, 3, noise="random",
                              target="product")
    f = dense.exact_value(c)
    for method in ("literal", "network"):
        r = estimate.estimate(c, 3, method)
        if abs(r["A"][-1] - f) > 1e-10:
            return False
    g = dense.graded_levels(c, 2)
    r = estimate.estimate(c, 2, "network")
    if any(abs(g[u].real - r["T"][u]) > 1e-12 for u in range(3)):
        return False
    return True


def test_unpatched_oracle_passes_the_pins():
    assert pins_hold()


def _wrong_permute(m):
    return np.asarray(m).reshape(2, 2, 2, 2).transpose(0, 3, 1, 2).reshape(4, 4)


def _superop_missing_conj(kraus):
    m = np.zeros((4, 4), dtype=np.complex128)
    for e in kraus:
        m += np.kron(e, e)
    return m


def _split_without_conj(m):
    mt = channels.permute(m)
    s, d, th = np.linalg.svd(mt)
    t = th.conj().T
    u = np.stack([(d[i] * s[:, i]).reshape(2, 2) for i in range(4)])
    v = np.stack([t[:, i].reshape(2, 2) for i in range(4)])
    return d, u, v


def _enumerate_dropping_last(n, l):
    out = []
    for u in range(min(l, n) + 1):
        out.extend(terms.enumerate_level(n, u))
    return out[:-1]


def _apply_transposed(t, mat, axes):
    k = len(axes)
    g = np.asarray(mat, dtype=np.complex128).T.reshape((2,) * (2 * k))
    o = np.tensordot(g, t, axes=(list(range(k, 2 * k)), list(axes)))
    return np.moveaxis(o, list(range(k)), list(axes))


@pytest.mark.parametrize("target,attr,bad", [
    (channels, "permute", _wrong_permute),
    (channels, "superoperator", _superop_missing_conj),
    (channels, "svd_split", _split_without_conj),
    (terms, "enumerate_terms", _enumerate_dropping_last),
    (dense, "apply_to_axes", _apply_transposed),
])
def test_planted_mistake_is_caught(monkeypatch, target, attr, bad):
    monkeypatch.setattr(target, attr, bad)
    assert not pins_hold()
