"""Pins of the FP64 reference network: its analytic gradient against central
finite differences of its loss, and Adam against the update written out."""
import numpy as np

from oracle import mlp


def make_state(rng, n_in, width, depth):
    _, P = mlp.layout(n_in, width, depth)
    st = np.zeros(2 * n_in + 4 * P)
    st[:n_in] = rng.standard_normal(n_in) * 0.1
    st[n_in:2 * n_in] = 1.0 + rng.uniform(0, 0.5, n_in)
    st[2 * n_in:2 * n_in + P] = rng.standard_normal(P) * 0.5
    return st, P


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    n_in, width, depth = 5, 7, 2
    st, P = make_state(rng, n_in, width, depth)
    x = rng.standard_normal((11, n_in))
    t = rng.standard_normal(11)
    w = rng.uniform(0.5, 2.0, 11)
    g = mlp.gradients(st, x, t, w, n_in, width, depth)
    h = 1e-6
    for k in range(P):
        sp = st.copy()
        sm = st.copy()
        sp[2 * n_in + k] += h
        sm[2 * n_in + k] -= h
        fd = (mlp.loss(sp, x, t, w, n_in, width, depth) - mlp.loss(sm, x, t, w, n_in, width, depth)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(fd)), (k, fd, g[k])


def test_adam_first_step_moves_by_lr_times_sign():
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -0.1, 0.0])
    p2, m, v = mlp.adam(p, g, np.zeros(3), np.zeros(3), lr=0.01, step=1)
    # first step: m_hat = g, v_hat = g^2 -> update lr * g / (|g| + eps)
    assert np.allclose(p2[:2], p[:2] - 0.01 * np.sign(g[:2]), atol=1e-9)
    assert p2[2] == p[2]
