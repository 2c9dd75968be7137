"""Reference (FP64, numpy) of the term-pruning network, for checking the GPU
kernels: same state layout, forward pass, weighted squared-error loss, its
gradient by explicit backpropagation, and the Adam update.

Pinned by central finite differences of the loss (tests/test_oracle_mlp.py).

State layout (as the library's): [mean | inv_std | params | grads | m | v],
params per layer: W (out x in, row-major) then b (out); layers
n_in -> width (ReLU) -> ... -> width (ReLU) -> 1.
"""
import numpy as np


def layout(n_in, width, depth):
    dims = [n_in] + [width] * depth + [1]
    layers = []
    off = 0
    for l in range(len(dims) - 1):
        din, dout = dims[l], dims[l + 1]
        layers.append((din, dout, off, off + din * dout))
        off += din * dout + dout
    return layers, off


def unpack(state, n_in, width, depth):
    layers, P = layout(n_in, width, depth)
    mean = state[:n_in]
    istd = state[n_in:2 * n_in]
    params = state[2 * n_in:2 * n_in + P]
    Ws, bs = [], []
    for din, dout, wo, bo in layers:
        Ws.append(params[wo:wo + din * dout].reshape(dout, din))
        bs.append(params[bo:bo + dout])
    return mean, istd, Ws, bs


def forward(state, x, n_in, width, depth):
    mean, istd, Ws, bs = unpack(np.asarray(state, np.float64), n_in, width, depth)
    a = (np.asarray(x, np.float64) - mean) * istd
    acts = [a]
    for l, (W, b) in enumerate(zip(Ws, bs)):
        z = a @ W.T + b
        a = z if l == len(Ws) - 1 else np.maximum(z, 0.0)
        acts.append(a)
    return a[:, 0], acts


def loss(state, x, t, w, n_in, width, depth):
    y, _ = forward(state, x, n_in, width, depth)
    w = np.ones_like(y) if w is None else np.asarray(w, np.float64)
    return float(np.mean(w * (y - np.asarray(t, np.float64)) ** 2))


def gradients(state, x, t, w, n_in, width, depth):
    """Gradient of `loss` with respect to params (flat, layout order)."""
    state = np.asarray(state, np.float64)
    y, acts = forward(state, x, n_in, width, depth)
    n = y.shape[0]
    w = np.ones_like(y) if w is None else np.asarray(w, np.float64)
    _, _, Ws, bs = unpack(state, n_in, width, depth)
    layers, P = layout(n_in, width, depth)
    g = np.zeros(P)
    dz = (2.0 * w * (y - np.asarray(t, np.float64)) / n)[:, None]
    for l in range(len(Ws) - 1, -1, -1):
        din, dout, wo, bo = layers[l]
        a_prev = acts[l]
        g[wo:wo + din * dout] = (dz.T @ a_prev).reshape(-1)
        g[bo:bo + dout] = dz.sum(axis=0)
        if l > 0:
            dz = (dz @ Ws[l]) * (a_prev > 0)
    return g


def adam(params, grads, m, v, lr, step, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * grads
    v = b2 * v + (1 - b2) * grads * grads
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v
