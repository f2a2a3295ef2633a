"""Pins of the oracle's RMS normalisation (CPU): closed forms and
invariants that fix the definition y = x w / sqrt(mean(x^2) + eps)."""
import math

import numpy as np
import pytest

import oracle


def test_rms_norm_closed_forms():
    # a constant row c: mean square c^2, so y = c w / sqrt(c^2 + eps)
    w = np.array([1.0, -2.0, 0.5, 3.0])
    y = oracle.rms_norm(np.full((1, 4), 3.0), w, 0.25)
    assert np.allclose(y, 3.0 * w / math.sqrt(9.25), rtol=0, atol=1e-15)
    # (3, 4): mean square 12.5
    y = oracle.rms_norm([[3.0, 4.0]], [1.0, 1.0], 0.0)
    assert np.allclose(y, [[3 / math.sqrt(12.5), 4 / math.sqrt(12.5)]],
                       rtol=0, atol=1e-15)
    # one element: y = sign(x) w when eps = 0
    assert oracle.rms_norm([[-7.0]], [2.0], 0.0)[0, 0] == -2.0
    # a zero row stays zero for eps > 0
    assert np.all(oracle.rms_norm(np.zeros((1, 9)), np.ones(9), 1e-6) == 0)


def test_rms_norm_invariants():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((5, 77)) * rng.uniform(0.1, 10, (5, 1))
    ones = np.ones(77)
    y = oracle.rms_norm(x, ones, 0.0)
    # unit weights, eps 0: every row has mean square exactly 1
    assert np.allclose(np.mean(y * y, axis=1), 1.0, rtol=1e-13)
    # scale invariance per row, weights act per column
    assert np.allclose(oracle.rms_norm(x * 17.0, ones, 0.0), y, rtol=1e-13)
    w = rng.standard_normal(77)
    assert np.allclose(oracle.rms_norm(x, w, 0.0), y * w, rtol=1e-13)
    # rows are independent
    assert np.allclose(oracle.rms_norm(x[2:3], w, 0.3),
                       oracle.rms_norm(x, w, 0.3)[2:3], rtol=1e-15)
    # eps enters the mean square, not the root: the mean square of the
    # result is m / (m + eps) for unit weights
    m = np.mean(x * x, axis=1)
    y = oracle.rms_norm(x, ones, 0.5)
    assert np.allclose(np.mean(y * y, axis=1), m / (m + 0.5), rtol=1e-13)


def test_rms_norm_brute_force_small():
    rng = np.random.default_rng(2)
    x = rng.integers(-5, 6, (3, 6)).astype(float)
    w = rng.integers(-3, 4, 6).astype(float)
    y = oracle.rms_norm(x, w, 0.125)
    for r in range(3):
        s = 0.0
        for j in range(6):
            s += x[r, j] ** 2
        d = math.sqrt(s / 6 + 0.125)
        for j in range(6):
            assert abs(y[r, j] - x[r, j] * w[j] / d) <= 1e-15 * (1 + abs(y[r, j]))


def _norm_variant(kind):
    """Plausible mistakes in the RMS normalisation, planted on the CPU."""
    def f(x, w, eps):
        x = np.atleast_2d(np.asarray(x, dtype=np.float64))
        w = np.asarray(w, dtype=np.float64).reshape(-1)
        if kind == "sum_not_mean":
            return x * w / np.sqrt(np.sum(x * x, axis=1, keepdims=True) + eps)
        if kind == "eps_outside_root":
            return x * w / (np.sqrt(np.mean(x * x, axis=1, keepdims=True))
                            + eps)
        if kind == "no_weight":
            return x / np.sqrt(np.mean(x * x, axis=1, keepdims=True) + eps)
        if kind == "column_mean":
            return x * w / np.sqrt(np.mean(x * x, axis=0, keepdims=True) + eps)
        return oracle.rms_norm(x, w, eps)
    return f


@pytest.mark.parametrize("kind", ["sum_not_mean", "eps_outside_root",
                                  "no_weight", "column_mean"])
def test_planted_norm_mistakes_fail_a_pin(kind):
    f = _norm_variant(kind)
    rng = np.random.default_rng(1)
    x = rng.standard_normal((5, 77)) * rng.uniform(0.1, 10, (5, 1))
    ones = np.ones(77)
    w = rng.standard_normal(77)
    m = np.mean(x * x, axis=1)
    checks = [
        np.allclose(f(np.full((1, 4), 3.0), [1.0, -2.0, 0.5, 3.0], 0.25),
                    3.0 * np.array([1.0, -2.0, 0.5, 3.0]) / math.sqrt(9.25)),
        np.allclose(np.mean(f(x, ones, 0.0) ** 2, axis=1), 1.0),
        np.allclose(np.mean(f(x, ones, 0.5) ** 2, axis=1), m / (m + 0.5)),
        np.allclose(f(x, w, 0.0), f(x, ones, 0.0) * w),
        np.allclose(f(x[2:3], w, 0.3), f(x, w, 0.3)[2:3]),
    ]
    assert not all(checks)


# ------------------------------------------- fused normalisation + product

def test_fused_norm_matvec_equals_chain_when_rounding_is_exact():
    """With power-of-two normalisation weights and bf16 activations every
    x * nw is a bf16 value, so the fused definition reduces to the plain
    chain rms_norm(x, nw) . W^T (row scale factored out of the sum)."""
    rng = np.random.default_rng(11)
    M, K, N = 3, 40, 7
    x = oracle.decode_bf16(oracle.round_bf16(rng.standard_normal((M, K))))
    nw = 2.0 ** rng.integers(-2, 3, K)
    W = rng.standard_normal((N, K))
    sw = rng.uniform(0.5, 2.0, N)
    for eps in (0.0, 1e-3):
        got = oracle.rms_norm_matvec(x, nw, W, eps, sw)
        want = oracle.rms_norm(x, nw, eps) @ W.T * sw
        assert np.allclose(got, want, rtol=1e-13, atol=1e-15)


def test_fused_norm_matvec_small_integers_exact():
    """Rows of +-2^j (mean square 4^j, eps 0: row scale 2^-j exactly),
    power-of-two weights and small-integer W: an exact integer sum halved
    j times."""
    rng = np.random.default_rng(12)
    M, K, N = 4, 64, 5
    sign = np.where(rng.integers(0, 2, (M, K)) == 1, 1.0, -1.0)
    j = np.arange(M)[:, None]
    x = sign * 2.0 ** j
    nw = 2.0 ** rng.integers(-1, 3, K)
    W = rng.integers(-4, 5, (N, K)).astype(np.float64)
    got = oracle.rms_norm_matvec(x, nw, W, 0.0)
    want = (sign * nw) @ W.T           # x * nw / 2^j = sign * nw
    assert np.array_equal(got, want)


def test_fused_norm_matvec_worked_rounding_example():
    """K = 2, x = (1 + 2^-7, 1 + 2^-7), nw = (1 + 2^-7, 1), W = (1, 1):
    x0 nw0 = 1 + 2^-6 + 2^-14 rounds to the bf16 value 1 + 2^-6 (2^-14 is
    below half a bf16 unit at 1, 2^-8), x1 nw1 = 1 + 2^-7 is exact, and the
    mean square is (1 + 2^-7)^2, so y = (2 + 3 2^-7) / (1 + 2^-7)."""
    a = 1.0 + 2.0 ** -7
    got = oracle.rms_norm_matvec([[a, a]], [a, 1.0], [[1.0, 1.0]], 0.0)
    assert got[0, 0] == pytest.approx((2.0 + 3 * 2.0 ** -7) / a, rel=1e-15)
    # without the intermediate rounding the 2^-14 term would survive
    assert abs(got[0, 0] - (2.0 + 3 * 2.0 ** -7 + 2.0 ** -14) / a) > 1e-5


def test_planted_fused_scale_inside_rounding_fails(monkeypatch):
    """Applying the row scale before the bf16 rounding (round(x nw s))
    breaks the worked example (planted in a copy of the oracle)."""
    def bad(x, nw, W, eps, sw=None):
        x = np.atleast_2d(np.asarray(x, dtype=np.float64))
        nw = np.asarray(nw, dtype=np.float64).reshape(-1)
        s = 1.0 / np.sqrt(np.mean(x * x, axis=1, keepdims=True) + eps)
        xw = oracle.decode_bf16(oracle.round_bf16(x * nw * s))
        return oracle.gemm(xw, W, b_nk=True, sb=sw)
    monkeypatch.setattr(oracle, "rms_norm_matvec", bad)
    with pytest.raises(AssertionError):
        test_fused_norm_matvec_worked_rounding_example()


def test_residual_add_closes_the_layer():
    """The decode layer's output is its matvec result plus its input: with
    zero weights the layer returns the residual exactly, with a zero
    residual it returns the product, and scales act on the product only
    (W = I, output scales 2, residual 1: y = 2 x + 1, not 2 (x + 1))."""
    rng = np.random.default_rng(14)
    x = rng.integers(-8, 9, (3, 6)).astype(np.float64)
    R = rng.integers(-8, 9, (3, 6)).astype(np.float64)
    P0 = oracle.gemm(x, np.zeros((6, 6)), b_nk=True)
    assert np.array_equal(oracle.residual_add(P0, R), R)
    P = oracle.gemm(x, np.eye(6), b_nk=True, sb=np.full(6, 2.0))
    assert np.array_equal(oracle.residual_add(P, np.zeros((3, 6))), 2 * x)
    assert np.array_equal(oracle.residual_add(P, np.ones((3, 6))),
                          2 * x + 1)


def test_planted_scaled_residual_fails(monkeypatch):
    """Scaling the residual with the product (planted) fails the pin."""
    monkeypatch.setattr(oracle, "residual_add",
                        lambda P, R: 2.0 * (np.asarray(P) / 2.0 +
                                            np.asarray(R)))
    with pytest.raises(AssertionError):
        test_residual_add_closes_the_layer()
