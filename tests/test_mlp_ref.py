"""Pins of the FP64 MLP oracle (CPU): finite differences and closed forms."""
import numpy as np

from oracle import mlp_ref as M


def _case(seed, B=37, k=6):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.3, M.n_params(k))
    x = rng.normal(0, 1, (B, M.NI))
    t = rng.normal(0, 1, (B, k))
    return p, x, t, k


def test_gradient_matches_central_differences():
    p, x, t, k = _case(1)
    g = M.grad(p, x, t, k)
    rng = np.random.default_rng(2)
    idx = rng.choice(len(p), 300, replace=False)
    fd = M.fd_grad(p, x, t, k, idx)
    assert np.max(np.abs(fd - g[idx])) <= 1e-6 * max(1.0, np.max(np.abs(fd)))


def test_bias3_gradient_closed_form():
    # d loss / d b3_k = 2 / (B K) * sum_b (y_bk - t_bk)
    p, x, t, k = _case(3)
    y, _ = M.forward(p, x, k)
    g = M.grad(p, x, t, k)
    want = 2.0 * (y - t).sum(axis=0) / (x.shape[0] * k)
    assert np.allclose(g[-k:], want, rtol=1e-12, atol=1e-14)


def test_zero_weights_output_is_bias():
    k = 4
    p = np.zeros(M.n_params(k))
    p[-k:] = [1.0, -2.0, 3.0, 0.5]
    x = np.random.default_rng(4).normal(0, 1, (5, M.NI))
    y, _ = M.forward(p, x, k)
    assert np.array_equal(y, np.tile(p[-k:], (5, 1)))


def test_linear_regime_is_affine_least_squares_gradient():
    # with all hidden pre-activations positive the network is the affine map
    # x -> x A + c, A = W1 W2 W3; the W3 gradient is the textbook least-squares
    # gradient 2 / (B K) * h2^T (Y - T)
    rng = np.random.default_rng(5)
    k = 3
    p = np.abs(rng.normal(0, 0.1, M.n_params(k)))
    x = np.abs(rng.normal(0, 1, (20, M.NI)))
    t = rng.normal(0, 1, (20, k))
    W1, b1, W2, b2, W3, b3 = M.unpack(p, k)
    y, (_, z1, h1, z2, h2) = M.forward(p, x, k)
    assert (z1 > 0).all() and (z2 > 0).all()
    A = W1 @ W2 @ W3
    c = b1 @ W2 @ W3 + b2 @ W3 + b3
    assert np.allclose(y, x @ A + c, rtol=1e-12, atol=1e-12)
    g = M.grad(p, x, t, k)
    off = M.NI * M.H + M.H + M.H * M.H + M.H
    gW3 = g[off:off + M.H * k].reshape(M.H, k)
    assert np.allclose(gW3, 2.0 * h2.T @ (y - t) / (20 * k), rtol=1e-12, atol=1e-14)
