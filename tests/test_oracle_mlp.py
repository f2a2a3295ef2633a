"""Pins of the binary64 cost-model oracle (CPU only)."""
import numpy as np
import pytest

import synth
from oracle import mlp


def _net(n_in=3, hidden=4, depth=2, B=5, seed=0):
    rng = np.random.default_rng(seed)
    p = synth.mlp_init(n_in, hidden, depth, 100 + seed).double().numpy()
    p = p + rng.normal(0, 0.1, p.size)      # non-zero biases too
    X = rng.normal(0, 1, (B, n_in))
    y = rng.normal(0, 1, B)
    return p, X, y, (n_in, hidden, depth)


def fd_grad(f, p, h=1e-6):
    g = np.zeros_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        g[i] = (f(p + e) - f(p - e)) / (2 * h)
    return g


@pytest.mark.parametrize("seed,depth", [(0, 1), (1, 2), (2, 3)])
def test_gradient_matches_central_differences(seed, depth):
    p, X, y, arch = _net(depth=depth, seed=seed)
    arch = (arch[0], arch[1], depth)
    p = p[:mlp.param_count(*arch)] if p.size >= mlp.param_count(*arch) else \
        synth.mlp_init(*arch, 7).double().numpy()
    g = mlp.grad(p, X, y, *arch)
    fd = fd_grad(lambda q: mlp.loss(q, X, y, *arch), p)
    assert np.max(np.abs(g - fd)) <= 1e-6 * max(1.0, np.max(np.abs(fd)))


def test_param_layout_and_count():
    assert mlp.param_count(16, 64, 3) == 16 * 64 + 64 + 2 * (64 * 64 + 64) \
        + 64 + 1
    assert synth.mlp_init(16, 64, 3, 0).numel() == mlp.param_count(16, 64, 3)


def test_zero_weights_closed_form():
    n_in, hidden, depth = 5, 6, 3
    p = np.zeros(mlp.param_count(n_in, hidden, depth))
    p[-1] = 0.75                                  # output bias
    rng = np.random.default_rng(3)
    X = rng.normal(size=(9, n_in))
    y = rng.normal(size=9)
    out, _ = mlp.forward(p, X, n_in, hidden, depth)
    assert np.all(out == 0.75)
    assert mlp.loss(p, X, y, n_in, hidden, depth) == pytest.approx(
        np.mean((0.75 - y) ** 2), rel=1e-15)
    g = mlp.grad(p, X, y, n_in, hidden, depth)
    assert g[-1] == pytest.approx(2 * np.mean(0.75 - y), rel=1e-14)
    # every hidden unit is dead (input 0 to the ReLU's kink from the left):
    # all other gradients vanish
    assert np.all(g[:-1] == 0)


def test_linear_regime_collapses_to_matrix_product():
    """With non-negative inputs, weights and biases every ReLU passes its
    input, so the network equals the collapsed affine map."""
    n_in, hidden, depth = 3, 4, 2
    rng = np.random.default_rng(4)
    p = rng.uniform(0.1, 1.0, mlp.param_count(n_in, hidden, depth))
    X = rng.uniform(0.0, 1.0, (6, n_in))
    (W1, b1), (W2, b2), (W3, b3) = mlp.unpack(p, n_in, hidden, depth)
    Wc = W3 @ W2 @ W1
    bc = W3 @ (W2 @ b1 + b2) + b3
    expect = X @ Wc.T + bc
    out, _ = mlp.forward(p, X, n_in, hidden, depth)
    assert np.allclose(out, expect[:, 0], rtol=1e-13, atol=0)


def test_adam_first_step_is_scaled_sign():
    rng = np.random.default_rng(5)
    p = rng.normal(size=20)
    g = rng.normal(size=20)
    lr, eps = 1e-2, 1e-8
    p1, m1, v1 = mlp.adam(p, g, np.zeros(20), np.zeros(20), 1, lr=lr, eps=eps)
    assert np.allclose(p1, p - lr * g / (np.abs(g) + eps), rtol=1e-14,
                       atol=1e-17)
    assert np.allclose(m1, 0.1 * g) and np.allclose(v1, 0.001 * g * g)


def test_planted_missing_relu_mask_fails_the_pin(monkeypatch):
    """A backward pass that forgets the ReLU mask disagrees with the finite
    differences (planted in a copy of the oracle on the CPU)."""
    p, X, y, arch = _net(depth=2, seed=9)

    def bad_grad(p, X, y, n_in, hidden, depth):
        layers = mlp.unpack(p, n_in, hidden, depth)
        out, acts = mlp.forward(p, X, n_in, hidden, depth)
        dZ = (2.0 / out.shape[0]) * (out - y)[:, None]
        grads = [None] * len(layers)
        for l in range(depth, -1, -1):
            W, _ = layers[l]
            grads[l] = (dZ.T @ acts[l], dZ.sum(axis=0))
            if l > 0:
                dZ = dZ @ W                      # mask dropped
        return np.concatenate([np.concatenate([g.ravel(), b])
                               for g, b in grads])
    fd = fd_grad(lambda q: mlp.loss(q, X, y, *arch), p)
    assert np.max(np.abs(bad_grad(p, X, y, *arch) - fd)) > 1e-4


def _adam_run(p, gs, m, v, t0, **hp):
    """Successive Adam steps t0, t0 + 1, ... with the gradients gs."""
    for i, g in enumerate(gs):
        p, m, v = mlp.adam(p, g, m, v, t0 + i, **hp)
    return p, m, v


def test_adam_constant_gradient_closed_form():
    """From zero moments a constant gradient g gives m_t = (1 - b1^t) g and
    v_t = (1 - b2^t) g^2, so both bias-corrected moments equal g and g^2 at
    every step and each step moves p by -lr g / (|g| + eps)."""
    rng = np.random.default_rng(6)
    p0 = rng.normal(size=16)
    g = rng.normal(size=16)
    lr, b1, b2, eps = 1e-2, 0.9, 0.999, 1e-8
    p, m, v = p0, np.zeros(16), np.zeros(16)
    for t in range(1, 13):
        p, m, v = mlp.adam(p, g, m, v, t, lr=lr, b1=b1, b2=b2, eps=eps)
        assert np.allclose(m, (1 - b1 ** t) * g, rtol=1e-13, atol=0)
        assert np.allclose(v, (1 - b2 ** t) * g * g, rtol=1e-12, atol=0)
        assert np.allclose(p, p0 - t * lr * g / (np.abs(g) + eps),
                           rtol=1e-12, atol=1e-15)


def test_adam_zero_gradient_decays_moments_geometrically():
    """With g = 0 the moments decay as m_t = b1^n m_0, v_t = b2^n v_0 after
    n steps, and each step moves p against the bias-corrected ratio."""
    rng = np.random.default_rng(7)
    p0 = rng.normal(size=12)
    m0 = rng.normal(size=12)
    v0 = rng.uniform(0.5, 2.0, 12)
    lr, b1, b2, eps = 1e-3, 0.8, 0.99, 1e-8
    n, t0 = 9, 4
    p, m, v = _adam_run(p0, [np.zeros(12)] * n, m0, v0, t0, lr=lr, b1=b1,
                        b2=b2, eps=eps)
    assert np.allclose(m, b1 ** n * m0, rtol=1e-13, atol=0)
    assert np.allclose(v, b2 ** n * v0, rtol=1e-13, atol=0)
    # p moved by sum over steps j = 1..n of lr * mhat_j / (sqrt(vhat_j) + eps)
    # with mhat_j = b1^j m0 / (1 - b1^(t0+j-1)), likewise vhat_j
    step = np.zeros(12)
    for j in range(1, n + 1):
        t = t0 + j - 1
        mh = b1 ** j * m0 / (1 - b1 ** t)
        vh = b2 ** j * v0 / (1 - b2 ** t)
        step += lr * mh / (np.sqrt(vh) + eps)
    assert np.allclose(p, p0 - step, rtol=1e-12, atol=1e-15)


def _adam_no_decay(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    m = (1 - b1) * g                      # planted: b1 * m dropped
    v = (1 - b2) * g * g                  # planted: b2 * v dropped
    return (p - lr * (m / (1 - b1 ** t)) / (np.sqrt(v / (1 - b2 ** t)) + eps),
            m, v)


def _adam_wrong_correction(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999,
                           eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1)                     # planted: b1 in place of b1**t
    vh = v / (1 - b2)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


@pytest.mark.parametrize("bad", [_adam_no_decay, _adam_wrong_correction])
def test_planted_adam_mistakes_fail_the_pins(monkeypatch, bad):
    """Each planted mistake (on the CPU, in a copy of the update) breaks the
    constant-gradient or the zero-gradient closed form."""
    monkeypatch.setattr(mlp, "adam", bad)
    failed = 0
    for pin in (test_adam_constant_gradient_closed_form,
                test_adam_zero_gradient_decays_moments_geometrically):
        try:
            pin()
        except AssertionError:
            failed += 1
    assert failed >= 1
