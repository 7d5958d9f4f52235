"""FP64 CPU reference of the surrogate MLP: forward, loss and gradients.

TEST INFRASTRUCTURE ONLY (called by tests to check the GPU kernels).  Written
from the definition of the network, with back-propagation by hand:
    x' = (x - x_mean) / x_std for the 6 features, then the derived input
         log10(max(x_5, 1e-4)) + 1.5 (x_5 = r / R_out, unnormalised), then
         zeros up to 32 inputs,
    h_0 = SiLU(W_0 x' + b_0),  h_l = SiLU(W_l h_{l-1} + b_l)  (l = 1 .. depth-1),
    out = w_out . h_{depth-1} + b_out,
    loss = mean over rows of (out - (y - y_mean) / y_std)^2,
SiLU(z) = z / (1 + e^-z).  Parameters of one member are a flat vector:
W_0 [256 x 32], W_1..W_{depth-1} [256 x 256] (row-major [out][in]), the depth
hidden biases [256 each], w_out [256], b_out.
"""
from __future__ import annotations

import numpy as np

WIDTH = 256
N_IN = 32
N_FEAT = 6


def param_count(depth: int) -> int:
    return WIDTH * N_IN + (depth - 1) * WIDTH * WIDTH + depth * WIDTH + WIDTH + 1


def unpack(p: np.ndarray, depth: int):
    p = np.asarray(p, np.float64)
    Ws = [p[:WIDTH * N_IN].reshape(WIDTH, N_IN)]
    o = WIDTH * N_IN
    for _ in range(depth - 1):
        Ws.append(p[o:o + WIDTH * WIDTH].reshape(WIDTH, WIDTH))
        o += WIDTH * WIDTH
    bs = [p[o + l * WIDTH:o + (l + 1) * WIDTH] for l in range(depth)]
    o += depth * WIDTH
    wout = p[o:o + WIDTH]
    bout = p[o + WIDTH]
    return Ws, bs, wout, bout


def _sig(z):
    return 1.0 / (1.0 + np.exp(-z))


def inputs(X, x_mean, x_std):
    X = np.asarray(X, np.float64)
    xs = (X - np.asarray(x_mean, np.float64)) / np.asarray(x_std, np.float64)
    out = np.zeros((len(X), N_IN))
    out[:, :N_FEAT] = xs
    out[:, N_FEAT] = np.log10(np.maximum(X[:, N_FEAT - 1], 1e-4)) + 1.5
    return out


def forward(p, depth, X, x_mean, x_std):
    """Network output (standardised target units) and the layer values for back-propagation."""
    Ws, bs, wout, bout = unpack(p, depth)
    h = inputs(X, x_mean, x_std)
    hs, zs = [h], []
    for W, b in zip(Ws, bs):
        z = h @ W.T + b
        h = z * _sig(z)
        zs.append(z)
        hs.append(h)
    return h @ wout + bout, hs, zs


def predict_logT(p, depth, X, x_mean, x_std, y_mean, y_std):
    out, _, _ = forward(p, depth, X, x_mean, x_std)
    return y_mean + y_std * out


def loss_and_grad(p, depth, X, y, x_mean, x_std, y_mean, y_std):
    out, hs, zs = forward(p, depth, X, x_mean, x_std)
    n = len(out)
    t = (np.asarray(y, np.float64) - y_mean) / y_std
    r = out - t
    loss = float(np.mean(r * r))
    g = 2.0 * r / n                                       # d loss / d out
    Ws, bs, wout, bout = unpack(p, depth)
    gW, gb = [None] * depth, [None] * depth
    gwout = hs[-1].T @ g
    gbout = g.sum()
    dh = np.outer(g, wout)                                # d loss / d h_{depth-1}
    for l in range(depth - 1, -1, -1):
        s = _sig(zs[l])
        dz = dh * (s * (1.0 + zs[l] * (1.0 - s)))         # SiLU'(z) = s (1 + z (1 - s))
        gW[l] = dz.T @ hs[l]
        gb[l] = dz.sum(axis=0)
        dh = dz @ Ws[l]
    flat = np.concatenate([w.ravel() for w in gW] + gb + [gwout, [gbout]])
    return loss, flat
