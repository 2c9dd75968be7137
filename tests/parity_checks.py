"""Checks of a computed estimate against the stored oracle values (test
infrastructure; no GPU).  Used by the GPU parity tests on the kernels'
results, and by CPU tests on the host replay of the same schedules, including
replays with planted mistakes that the checks must catch.

Per term: an FP32 term value X = w |a|^2 is compared within fp32_term_tol.
The amplitude a is a contraction of unitary gates, unit states and the slot
matrices K_c, so |a| <= prod ||K_c||_2 and its FP32 rounding error is a
multiple of the unit roundoff times prod ||K_c||_2 (not of |a|: small terms
come from cancellation).  With B = w prod ||K_c||_2^2 and eta = 2^-18 (64
units of FP32 rounding): |X_gpu - X| <= 2e-5 X + 2 eta sqrt(X B) + eta^2 B.
The all-dominant term is computed in FP64 and compared at 1e-12.

Per level (Algorithm 1's T_u): within 2e-5 T_u plus the sum of the level's
per-term bounds.  Degenerate channels (depolarizing: d_1 = d_2 = d_3) make
single terms basis dependent, so sums over each noise-position set are
compared instead, within the summed bounds of their terms.

FP64 sums (a8): the reported T_u equals math.fsum of the same computed X_t of
level u within 1e-12 relative.
"""
import math

import numpy as np

ETA32 = 2.0 ** -18


def term_bound(split, term):
    """B = w prod ||K_c||_2^2 of one term (split: oracle.network.slot_split)."""
    b = 1.0
    for s, c in enumerate(term):
        d, k, _ = split[s]
        b *= d[c] * np.linalg.norm(k[c], 2) ** 2
    return b


def fp32_term_tol(split, term, ref):
    b = term_bound(split, term)
    return 2e-5 * ref + 2 * ETA32 * math.sqrt(max(ref, 0.0) * b) + ETA32 ** 2 * b


def term_tols(split, pat, ref, fp64_first=True):
    """fp32_term_tol of every term; with fp64_first the first entry is the
    all-dominant term, computed in FP64 (1e-12 relative)."""
    pat = np.asarray(pat, dtype=np.int64)
    ref = np.asarray(ref, dtype=np.float64)
    fac = np.array([[split[s][0][c] * np.linalg.norm(split[s][1][c], 2) ** 2 for c in range(4)]
                    for s in range(len(split))])
    b = np.ones(len(pat))
    for s in range(pat.shape[1]):
        b *= fac[s][pat[:, s]]
    tol = 2e-5 * ref + 2 * ETA32 * np.sqrt(np.maximum(ref, 0.0) * b) + ETA32 ** 2 * b
    if fp64_first and len(tol):
        tol[0] = 1e-12 * ref[0]
    return tol


def check_terms(x, ref, pat, split, degenerate, fp64_first=True):
    """Every term (or, for degenerate channels, every noise-position group)
    within its FP32 bound; returns the per-term tolerances."""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert x.shape == ref.shape, (x.shape, ref.shape)
    tol = term_tols(split, pat, ref, fp64_first)
    if degenerate:
        keys = [tuple(np.flatnonzero(row)) for row in pat]
        groups = {}
        for j, k in enumerate(keys):
            groups.setdefault(k, []).append(j)
        for k, idx in groups.items():
            got, want, t = x[idx].sum(), ref[idx].sum(), tol[idx].sum()
            assert abs(got - want) <= t, ("position group", k, got, want, t)
    else:
        err = np.abs(x - ref)
        bad = np.flatnonzero(err > tol)
        assert bad.size == 0, ("terms", bad[:5], x[bad[:5]], ref[bad[:5]], tol[bad[:5]])
    return tol


def check_level_sums(T, x, pat, gold_T, tol):
    """T_u against the oracle's stored level sums (2e-5 T_u plus the level's
    summed per-term bounds), and against math.fsum of the same x (1e-12)."""
    lv = (np.asarray(pat) != 0).sum(axis=1)
    assert len(T) == len(gold_T), (len(T), len(gold_T))
    for u in range(len(gold_T)):
        sel = lv == u
        bound = 2e-5 * abs(gold_T[u]) + tol[sel].sum()
        assert abs(T[u] - gold_T[u]) <= bound, ("T_u vs oracle", u, T[u], gold_T[u], bound)
        fs = math.fsum(float(v) for v in np.asarray(x)[sel])
        assert abs(T[u] - fs) <= 1e-12 * abs(fs) + 1e-300, ("T_u vs fsum of the same X_t", u, T[u], fs)


def check_against_golden(T, x, pat, gold_T, gold_x, split, degenerate):
    """Terms, then level sums; raises AssertionError at the first failure."""
    tol = check_terms(x, gold_x, pat, split, degenerate)
    check_level_sums(T, x, pat, gold_T, tol)
