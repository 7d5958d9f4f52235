"""Pins of the FP64 MLP reference: analytical gradients against central finite
differences of the loss, and the closed form of a network with zero weights."""
import numpy as np

from oracle import mlp_ref


def _setup(depth, seed=0, n=6):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.08, mlp_ref.param_count(depth))
    X = rng.normal(0, 1, (n, 6))
    y = rng.normal(1.3, 0.2, n)
    return p, X, y


def test_gradients_match_finite_differences():
    depth = 2
    p, X, y = _setup(depth)
    xm, xs, ym, ys = np.zeros(6), np.ones(6), 1.2, 0.3
    loss, g = mlp_ref.loss_and_grad(p, depth, X, y, xm, xs, ym, ys)
    rng = np.random.default_rng(1)
    # first layer inputs beyond the 6 features and the derived log-radius input
    # never see a nonzero input: zero gradient
    W0 = g[:256 * 32].reshape(256, 32)
    assert np.all(W0[:, 7:] == 0) and np.any(W0[:, 6] != 0)
    idx = np.concatenate([rng.integers(0, 256 * 32, 20) // 32 * 32 + rng.integers(0, 7, 20),
                          rng.integers(256 * 32, len(p), 60)])
    h = 1e-6
    for i in idx:
        q = p.copy()
        q[i] += h
        lp, _ = mlp_ref.loss_and_grad(q, depth, X, y, xm, xs, ym, ys)
        q[i] -= 2 * h
        lm, _ = mlp_ref.loss_and_grad(q, depth, X, y, xm, xs, ym, ys)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (i, fd, g[i])


def test_zero_network_outputs_bias():
    depth = 3
    p = np.zeros(mlp_ref.param_count(depth))
    p[-1] = 0.7                               # output bias
    X = np.random.default_rng(2).normal(size=(5, 6))
    out = mlp_ref.predict_logT(p, depth, X, np.zeros(6), np.ones(6), 1.0, 2.0)
    assert np.allclose(out, 1.0 + 2.0 * 0.7)
    # SiLU(0) = 0 so every hidden activation vanishes; only b_out moves the output
    loss, g = mlp_ref.loss_and_grad(p, depth, X, np.full(5, 1.0 + 2.0 * 0.7), np.zeros(6), np.ones(6), 1.0, 2.0)
    assert loss == 0.0 and np.all(g == 0)


def test_derived_log_radius_input():
    X = np.zeros((3, 6))
    X[:, 5] = [1.0, 1e-2, 0.0]
    x = mlp_ref.inputs(X, np.zeros(6), np.ones(6))
    assert np.allclose(x[:, 6], [1.5, -0.5, -2.5]) and np.all(x[:, 7:] == 0)
