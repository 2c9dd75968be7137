"""Pins of the oracle's channel layer (superoperator, permutation, SVD split).

Each test checks the oracle against something other than itself: the matrix
printed in Section IV, textbook closed forms of the channels, trace
preservation (Section II), and Lemmas 1 and 2 as properties.
"""
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import channels

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def basis_rho(a, b):
    r = np.zeros((2, 2), dtype=np.complex128)
    r[a, b] = 1.0
    return r


def test_identity_permutation_matches_printed_matrix():
    printed = np.loadtxt(os.path.join(GOLD, "identity_permutation.txt"))
    got = channels.permute(np.eye(4))
    assert np.array_equal(got.real, printed)
    assert np.all(got.imag == 0)


def test_permutation_is_an_involution_and_keeps_frobenius_norm():
    rng = np.random.default_rng(1)
    for _ in range(20):
        a = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
        assert np.array_equal(channels.permute(channels.permute(a)), a)
        assert math.isclose(np.linalg.norm(channels.permute(a)), np.linalg.norm(a), rel_tol=1e-14)


def test_permutation_moves_single_entries_as_stated():
    # M has edges (1,2) as rows and (3,4) as columns; Mt has (1,3) as rows and
    # (2,4) as columns: entry M[(a,b),(c,d)] lands on Mt[(a,c),(b,d)].
    for a in range(2):
        for b in range(2):
            for c in range(2):
                for d in range(2):
                    m = np.zeros((4, 4))
                    m[2 * a + b, 2 * c + d] = 1
                    mt = channels.permute(m)
                    assert mt[2 * a + c, 2 * b + d] == 1 and mt.sum() == 1


@pytest.mark.parametrize("p", [0.0, 1e-4, 1e-3, 0.05, 0.3])
def test_depolarizing_closed_form(p):
    # E(rho) = (1 - p) rho + p/3 (X rho X + Y rho Y + Z rho Z)
    #        = (1 - 4p/3) rho + (2p/3) tr(rho) I
    m = channels.superoperator(W.kraus_depolarizing(p))
    for a in range(2):
        for b in range(2):
            rho = basis_rho(a, b)
            want = (1 - 4 * p / 3) * rho + (2 * p / 3) * np.trace(rho) * np.eye(2)
            assert np.allclose(channels.apply_superop(m, rho), want, atol=1e-15)


@pytest.mark.parametrize("g,lam", [(0.0, 0.0), (1e-3, 5e-3), (0.2, 0.0), (0.0, 0.3), (0.1, 0.4)])
def test_amplitude_phase_damping_closed_form(g, lam):
    m = channels.superoperator(W.kraus_ad_pd(g, lam))
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))
    rho = x @ x.conj().T
    rho /= np.trace(rho)
    out = channels.apply_superop(m, rho)
    assert np.isclose(out[0, 0], rho[0, 0] + g * rho[1, 1], atol=1e-15)
    assert np.isclose(out[1, 1], (1 - g) * rho[1, 1], atol=1e-15)
    assert np.isclose(out[0, 1], math.sqrt((1 - g) * (1 - lam)) * rho[0, 1], atol=1e-15)
    assert np.isclose(out[1, 0], math.sqrt((1 - g) * (1 - lam)) * rho[1, 0], atol=1e-15)


def test_trace_preservation_identity():
    # sum_k E_k^dagger E_k = I  <=>  vec(I)^dagger M = vec(I)^dagger
    rng = np.random.default_rng(3)
    veci = np.eye(2).reshape(4)
    for nk in (1, 2, 3, 4):
        kr = W.random_isometry_kraus(rng, nk)
        assert channels.tp_residual(kr) < 1e-14
        m = channels.superoperator(kr)
        assert np.allclose(veci @ m, veci, atol=1e-14)
    bad = [1.01 * np.eye(2)]
    assert channels.tp_residual(bad) > 1e-3
    assert not np.allclose(veci @ channels.superoperator(bad), veci)


def _channels_for_tests():
    rng = np.random.default_rng(4)
    out = [W.kraus_depolarizing(1e-3), W.kraus_depolarizing(0.2), W.kraus_ad_pd(1e-3, 2e-3),
           W.kraus_ad_pd(0.3, 0.1), [np.eye(2, dtype=np.complex128)]]
    for nk in (1, 2, 3, 4, 4, 4):
        out.append(W.random_isometry_kraus(rng, nk))
    return out


def test_svd_split_reconstructs_the_superoperator():
    for kr in _channels_for_tests():
        m = channels.superoperator(kr)
        d, u, v = channels.svd_split(m)
        assert np.all(np.diff(d) <= 1e-15)  # descending
        assert np.linalg.norm(channels.reconstruct(u, v) - m) < 1e-14


def test_split_of_psd_permuted_matrix_has_conjugate_factors():
    # Mt = sum_k vec(E_k) vec(E_k)^dagger is Hermitian PSD, so S = T on the
    # non-zero singular subspace: V_i = conj(U_i) / d_i.
    for kr in _channels_for_tests():
        m = channels.superoperator(kr)
        mt = channels.permute(m)
        assert np.allclose(mt, mt.conj().T, atol=1e-15)
        assert np.min(np.linalg.eigvalsh(mt)) > -1e-14
        d, u, v = channels.svd_split(m)
        for i in range(4):
            if d[i] > 1e-12:
                assert np.allclose(v[i], np.conj(u[i]) / d[i], atol=1e-12)


def test_depolarizing_singular_values_and_rank_of_adpd():
    p = 1e-3
    d, _, _ = channels.svd_split(channels.superoperator(W.kraus_depolarizing(p)))
    assert np.allclose(d, [2 * (1 - p), 2 * p / 3, 2 * p / 3, 2 * p / 3], atol=1e-15)
    d2, _, _ = channels.svd_split(channels.superoperator(W.kraus_ad_pd(1e-3, 2e-3)))
    assert d2[3] < 1e-16 and d2[2] > 1e-4      # Kraus rank 3


def test_lemma1_permutation_at_most_doubles_spectral_distance():
    rng = np.random.default_rng(5)
    for _ in range(200):
        a = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
        b = a + 0.1 * (rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4)))
        lhs = np.linalg.norm(channels.permute(a) - channels.permute(b), 2)
        assert lhs <= 2 * np.linalg.norm(a - b, 2) * (1 + 1e-12)


def test_lemma2_dominant_term_within_four_noise_rates():
    rng = np.random.default_rng(6)
    for _ in range(100):
        kind = rng.integers(3)
        if kind == 0:
            kr = W.kraus_depolarizing(rng.uniform(0, 0.2))
        elif kind == 1:
            kr = W.kraus_ad_pd(rng.uniform(0, 0.2), rng.uniform(0, 0.2))
        else:
            kr = W.random_isometry_kraus(rng, int(rng.integers(1, 5)))
        m = channels.superoperator(kr)
        d, u, v = channels.svd_split(m)
        lhs = np.linalg.norm(m - np.kron(u[0], v[0]), 2)
        assert lhs <= 4 * channels.noise_rate(m) + 1e-14


def test_noise_rate_of_depolarizing_is_four_thirds_p():
    # From the closed form, M - I vanishes on vec(I) and is -(4p/3) on the
    # traceless directions, so ||M - I|| = 4p/3 (the text of Section IV says
    # 2p; the definition is what is implemented).
    for p in (1e-4, 1e-3, 0.01):
        m = channels.superoperator(W.kraus_depolarizing(p))
        assert math.isclose(channels.noise_rate(m), 4 * p / 3, rel_tol=1e-10)
