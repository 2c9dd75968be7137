"""Pins of the oracle's quantum-trajectories estimate.

Independent of sampling: the estimator's exact mean (every Kraus index
choice weighted by its probability) equals the density-matrix value of
Section II; the draws follow q; a long run lies within its error band.
"""
import numpy as np
import pytest

import workloads as W
from oracle import dense, trajectories


def tiny(seed, n=3, gates=10, noise=3, kind="random", target="circuit_output"):
    rng = np.random.default_rng(seed)
    return W.tiny_random_circuit(rng, n, gates, noise, noise=kind, level=1, target=target, scale=5.0)


@pytest.mark.parametrize("seed,kind,target", [(131, "random", "circuit_output"), (132, "adpd", "product"),
                                               (133, "depol", "dense"), (134, "random", "product")])
def test_exact_mean_equals_density_matrix(seed, kind, target):
    c = tiny(seed, kind=kind, target=target)
    assert abs(trajectories.expectation(c) - dense.exact_value(c)) <= 1e-12


def test_probabilities_sum_to_one_and_draws_follow_them():
    rng = np.random.default_rng(135)
    for kr in (W.random_isometry_kraus(rng, 3), W.kraus_ad_pd(0.3, 0.2), W.kraus_depolarizing(0.4)):
        q = trajectories.probabilities(kr)
        assert abs(q.sum() - 1.0) <= 1e-14 and np.all(q >= 0)
        u = np.random.default_rng(136).random(200000)
        counts = np.bincount([trajectories.draw(q, x) for x in u], minlength=len(q))
        sig = np.sqrt(q * (1 - q) / len(u))
        assert np.all(np.abs(counts / len(u) - q) <= 5 * sig + 1e-12)
    # boundaries: u below the first cumulative value picks 0, at it picks 1
    q = np.array([0.5, 0.0, 0.5])
    assert trajectories.draw(q, 0.4999) == 0 and trajectories.draw(q, 0.5) == 2 and trajectories.draw(q, 0.99) == 2


def test_long_run_within_its_error_band():
    c = tiny(137, kind="adpd")
    r = trajectories.estimate(c, W.trajectory_uniforms(4000, c.n_noises, 7))
    f = dense.exact_value(c)
    assert abs(r["mean"] - f) <= 5 * r["stderr"], (r["mean"], f, r["stderr"])


def test_wrong_normalisation_is_caught(monkeypatch):
    c = tiny(138, kind="random")
    f = dense.exact_value(c)

    def by_q(net, circ, idx):       # dividing the Kraus matrix by q instead of sqrt(q)
        mats = []
        for s, op in enumerate(circ.noise_ops()):
            q = trajectories.probabilities(op.kraus)
            mats.append(np.asarray(op.kraus[int(idx[s])]) / q[int(idx[s])])
        a = net.value(mats)
        return float(abs(a) ** 2)
    monkeypatch.setattr(trajectories, "sample_value", by_q)
    assert abs(trajectories.expectation(c) - f) > 1e-6
