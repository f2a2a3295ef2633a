"""Binary64 oracle of the tile-picker cost model (test infrastructure only).

The model is a multilayer perceptron: `depth` hidden layers of `hidden`
ReLU units and one linear output, trained on mean squared error with Adam.
Parameters are one flat vector; per layer W (out x in, row-major) then
b (out); the output layer has out = 1.  Everything here is the plain
definition, evaluated in float64 with numpy; the gradient is derived by hand
(chain rule) and pinned by central finite differences in the tests.
"""
import numpy as np


def shapes(n_in, hidden, depth):
    dims, sh = [n_in] + [hidden] * depth + [1], []
    for l in range(depth + 1):
        sh.append((dims[l + 1], dims[l]))
    return sh


def param_count(n_in, hidden, depth):
    return sum(o * i + o for o, i in shapes(n_in, hidden, depth))


def unpack(p, n_in, hidden, depth):
    p = np.asarray(p, dtype=np.float64)
    out, off = [], 0
    for o, i in shapes(n_in, hidden, depth):
        W = p[off:off + o * i].reshape(o, i)
        off += o * i
        b = p[off:off + o]
        off += o
        out.append((W, b))
    assert off == p.size
    return out


def forward(p, X, n_in, hidden, depth):
    """(out (B,), activations [X, H1, ..., H_depth])."""
    layers = unpack(p, n_in, hidden, depth)
    H = np.asarray(X, dtype=np.float64)
    acts = [H]
    for l, (W, b) in enumerate(layers):
        Z = H @ W.T + b
        if l < depth:
            H = np.maximum(Z, 0.0)
            acts.append(H)
        else:
            H = Z
    return H[:, 0], acts


def loss(p, X, y, n_in, hidden, depth):
    out, _ = forward(p, X, n_in, hidden, depth)
    d = out - np.asarray(y, dtype=np.float64)
    return float(np.mean(d * d))


def grad(p, X, y, n_in, hidden, depth):
    """d loss / d p by the chain rule, same flat layout as p."""
    layers = unpack(p, n_in, hidden, depth)
    out, acts = forward(p, X, n_in, hidden, depth)
    Bn = out.shape[0]
    dZ = (2.0 / Bn) * (out - np.asarray(y, dtype=np.float64))[:, None]
    grads = [None] * len(layers)
    for l in range(depth, -1, -1):
        W, _ = layers[l]
        Hprev = acts[l]
        grads[l] = (dZ.T @ Hprev, dZ.sum(axis=0))
        if l > 0:
            dZ = (dZ @ W) * (Hprev > 0)
    return np.concatenate([np.concatenate([g.ravel(), b]) for g, b in grads])


def adam(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba, Algorithm 1) at step t >= 1."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
