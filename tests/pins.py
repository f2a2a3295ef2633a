"""Independent pins for a binary64 GEMM routine.

Each check compares a candidate `gemm(A, B) -> R` with something other than
itself: exact integer / rational brute force, closed forms of the product,
and the binary64 error bound of a length-K dot product.  `run_pins` returns
the list of failed checks, so the test-suite can show both that the oracle
passes every pin and that planted mistakes fail at least one.
"""
import itertools
from fractions import Fraction

import numpy as np


def brute_int(A, B):
    """Exact product of integer matrices with Python ints."""
    M, K = len(A), len(A[0]) if len(A) else 0
    N = len(B[0]) if len(B) else 0
    return [[sum(int(A[i][k]) * int(B[k][j]) for k in range(K))
             for j in range(N)] for i in range(M)]


def brute_frac(A, B):
    """Exact product of binary64 matrices as rationals."""
    M, K = A.shape
    N = B.shape[1]
    return [[sum((Fraction(float(A[i, k])) * Fraction(float(B[k, j]))
                  for k in range(K)), Fraction(0)) for j in range(N)]
            for i in range(M)]


def _ints(rng, shape, lo=-9, hi=9):
    return rng.integers(lo, hi + 1, size=shape).astype(np.float64)


def pin_brute_small(gemm, dims=range(1, 8), seed=0):
    rng = np.random.default_rng(seed)
    bad = []
    for M, N, K in itertools.product(dims, dims, dims):
        A, B = _ints(rng, (M, K)), _ints(rng, (K, N))
        R = gemm(A, B)
        E = np.array(brute_int(A.astype(int).tolist(),
                               B.astype(int).tolist()), dtype=np.float64)
        if R.shape != (M, N) or not np.array_equal(R, E.reshape(M, N)):
            bad.append(("brute_small", M, N, K))
    return bad


def pin_brute_edges(gemm, seed=1):
    rng = np.random.default_rng(seed)
    bad = []
    for M, N, K in [(31, 33, 32), (33, 31, 65), (64, 63, 31), (65, 64, 63),
                    (1, 65, 64), (63, 1, 33)]:
        A, B = _ints(rng, (M, K), -4, 4), _ints(rng, (K, N), -4, 4)
        R = gemm(A, B)
        E = np.array(brute_int(A.astype(int).tolist(),
                               B.astype(int).tolist()), dtype=np.float64)
        if R.shape != (M, N) or not np.array_equal(R, E.reshape(M, N)):
            bad.append(("brute_edges", M, N, K))
    return bad


def pin_closed_forms(gemm, seed=2):
    """ones.ones = K everywhere; A.I = A; I.B = B; diag(d).B = row scaling;
    B.diag(d) = column scaling.  Non-square shapes so that a transposed
    operand cannot pass."""
    rng = np.random.default_rng(seed)
    bad = []
    M, N, K = 7, 5, 11
    R = gemm(np.ones((M, K)), np.ones((K, N)))
    if R.shape != (M, N) or not np.all(R == K):
        bad.append("ones")
    A = rng.standard_normal((M, K))
    R = gemm(A, np.eye(K))
    if R.shape != (M, K) or not np.array_equal(R, A):
        bad.append("A.I")
    B = rng.standard_normal((K, N))
    R = gemm(np.eye(K), B)
    if R.shape != (K, N) or not np.array_equal(R, B):
        bad.append("I.B")
    d = rng.standard_normal(K)
    R = gemm(np.diag(d), B)
    if R.shape != (K, N) or not np.array_equal(R, d[:, None] * B):
        bad.append("diag.B")
    R = gemm(A, np.diag(d))
    if R.shape != (M, K) or not np.array_equal(R, A * d[None, :]):
        bad.append("A.diag")
    return bad


def pin_error_bound(gemm, seed=3):
    """|fl(A.B) - A.B| <= gamma_K |A||B| with unit roundoff 2^-53 (every
    binary64 dot product evaluated in any order satisfies it)."""
    rng = np.random.default_rng(seed)
    bad = []
    for M, N, K in [(3, 4, 5), (2, 3, 17), (4, 2, 40)]:
        A = rng.standard_normal((M, K))
        B = rng.standard_normal((K, N))
        R = gemm(A, B)
        E = brute_frac(A, B)
        u = 2.0 ** -53
        g = K * u / (1 - K * u)
        absAB = np.abs(A) @ np.abs(B)
        for i in range(M):
            for j in range(N):
                err = abs(Fraction(float(R[i, j])) - E[i][j])
                if err > Fraction(g * absAB[i, j] * (1 + 1e-12)):
                    bad.append(("bound", M, N, K, i, j))
    return bad


def run_pins(gemm):
    return (pin_brute_small(gemm) + pin_brute_edges(gemm) +
            pin_closed_forms(gemm) + pin_error_bound(gemm))
