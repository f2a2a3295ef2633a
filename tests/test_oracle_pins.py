"""Pins of the CPU oracle against facts other than itself (CPU only)."""
import math
from fractions import Fraction

import numpy as np
import pytest
import torch

from conftest import read_golden
import pins


def _oracle_gemm(o):
    return lambda A, B: o.gemm(A, B)


def test_oracle_passes_all_pins(oracle_mod):
    assert pins.run_pins(_oracle_gemm(oracle_mod)) == []


@pytest.mark.parametrize("mutant", ["drop_last_k", "transpose_b", "sign",
                                    "index_shift", "skip_row"])
def test_planted_mistakes_fail_a_pin(oracle_mod, mutant):
    """Plausible oracle mistakes, planted on the CPU, are caught by the pins."""
    o = oracle_mod

    def g(A, B):
        A = np.asarray(A, dtype=np.float64)
        B = np.asarray(B, dtype=np.float64)
        if mutant == "drop_last_k":
            return o.gemm(A[:, :-1], B[:-1, :]) if A.shape[1] > 1 else \
                np.zeros((A.shape[0], B.shape[1]))
        if mutant == "transpose_b":
            if B.shape[0] == B.shape[1]:
                return o.gemm(A, B.T)
            return o.gemm(A, B)[:, ::-1]
        if mutant == "sign":
            R = o.gemm(A, B)
            R[-1, -1] = -R[-1, -1]
            return R
        if mutant == "index_shift":
            return o.gemm(A, np.roll(B, 1, axis=0))
        if mutant == "skip_row":
            R = o.gemm(A, B)
            R[0, :] = 0.0
            return R
        raise AssertionError
    assert pins.run_pins(g) != []


def test_b_nk_layout_matches_brute_force(oracle_mod):
    rng = np.random.default_rng(11)
    for M, N, K in [(1, 5, 7), (3, 9, 4), (8, 17, 33)]:
        A = rng.integers(-5, 6, (M, K)).astype(np.float64)
        W = rng.integers(-5, 6, (N, K)).astype(np.float64)   # N x K
        R = oracle_mod.gemm(A, W, b_nk=True)
        E = pins.brute_int(A.astype(int).tolist(),
                           W.T.astype(int).tolist())
        assert np.array_equal(R, np.array(E, dtype=np.float64))


def test_scaled_matches_rational_brute_force(oracle_mod):
    rng = np.random.default_rng(12)
    M, N, K = 4, 6, 9
    A = rng.integers(-4, 5, (M, K)).astype(np.float64)
    B = rng.integers(-4, 5, (K, N)).astype(np.float64)
    sa = rng.uniform(0.5, 2.0, M)
    sb = rng.uniform(0.5, 2.0, N)
    R = oracle_mod.gemm(A, B, sa=sa, sb=sb)
    E = pins.brute_int(A.astype(int).tolist(), B.astype(int).tolist())
    for i in range(M):
        for j in range(N):
            exact = Fraction(sa[i]) * Fraction(sb[j]) * E[i][j]
            # two binary64 roundings of the scale product + one of the result
            assert abs(Fraction(R[i, j]) - exact) <= abs(exact) * Fraction(
                3 * 2.0 ** -53)
    # one scale only
    R1 = oracle_mod.gemm(A, B, sa=sa)
    assert np.allclose(R1, sa[:, None] * np.array(E), rtol=1e-15, atol=0)


def test_entries_match_rational_brute_force(oracle_mod):
    rng = np.random.default_rng(13)
    M, N, K = 9, 7, 13
    A = rng.integers(-6, 7, (M, K)).astype(np.float64)
    W = rng.integers(-6, 7, (N, K)).astype(np.float64)
    ii = rng.integers(0, M, 20)
    jj = rng.integers(0, N, 20)
    E = pins.brute_int(A.astype(int).tolist(), W.T.astype(int).tolist())
    out = oracle_mod.gemm_entries(A, W, ii, jj, b_nk=True)
    assert [float(v) for v in out] == [float(E[i][j]) for i, j in zip(ii, jj)]
    sb = rng.uniform(0.1, 3.0, N)
    out = oracle_mod.gemm_entries(A, W, ii, jj, b_nk=True, sb=sb)
    for v, i, j in zip(out, ii, jj):
        assert abs(v - sb[j] * E[i][j]) <= abs(sb[j] * E[i][j]) * 1e-15


def test_rel_fro_closed_forms(oracle_mod):
    rng = np.random.default_rng(14)
    R = rng.standard_normal(1000)
    # uniform relative perturbation delta -> error exactly |delta| (to fp64)
    for d in [1e-3, -2.5e-6, 0.5]:
        assert oracle_mod.rel_fro(R * (1 + d), R) == pytest.approx(
            abs(d), rel=1e-9)
    # one perturbed element
    C = R.copy()
    C[17] += 3.0
    assert oracle_mod.rel_fro(C, R) == pytest.approx(
        3.0 / math.sqrt(float(np.sum(R * R))), rel=1e-12)
    # zero reference -> absolute norm
    assert oracle_mod.rel_fro(np.array([3.0, 4.0]), np.zeros(2)) == 5.0
    assert oracle_mod.rel_fro(R, R) == 0.0


def test_e4m3fn_golden_values(oracle_mod):
    rows = read_golden("e4m3fn_values.txt")
    codes = [int(c, 16) for c, _ in rows]
    got = oracle_mod.decode_e4m3fn(codes)
    for (c, v), g in zip(rows, got):
        if v == "nan":
            assert math.isnan(g)
        else:
            assert g == float(v) and math.copysign(1, g) == math.copysign(
                1, float(v)), c


def test_e4m3fn_all_codes_match_torch(oracle_mod):
    codes = np.arange(256, dtype=np.uint8)
    got = oracle_mod.decode_e4m3fn(codes)
    ref = torch.from_numpy(codes).view(torch.float8_e4m3fn).to(
        torch.float64).numpy()
    nan = np.isnan(ref)
    assert np.array_equal(np.isnan(got), nan)
    assert np.array_equal(got[~nan], ref[~nan])
    finite = got[~nan]
    assert finite.max() == 448.0 and finite.min() == -448.0
    assert np.sum(nan) == 2


def test_bf16_golden_and_torch(oracle_mod):
    rows = read_golden("bf16_values.txt")
    got = oracle_mod.decode_bf16([int(c, 16) for c, _ in rows])
    assert [float(v) for _, v in rows] == [float(g) for g in got]
    rng = np.random.default_rng(15)
    bits = rng.integers(0, 65536, 4096).astype(np.uint16)
    # drop NaN patterns (exponent all ones, mantissa non-zero)
    keep = ~(((bits & 0x7F80) == 0x7F80) & ((bits & 0x7F) != 0))
    bits = bits[keep]
    ref = torch.from_numpy(bits.view(np.int16)).view(torch.bfloat16).to(
        torch.float64).numpy()
    assert np.array_equal(oracle_mod.decode_bf16(bits), ref)


def test_listing1_worked_example(oracle_mod):
    """The paper's element-wise example: 1024 elements, partition [128],
    8 programs, value 2.0.  Its GEMM analogue ones.ones = K is pinned above;
    here the partition of the example is painted."""
    g = {r[0]: r[1] for r in read_golden("listing1_add.txt")}
    n, part, progs = int(g["n"]), int(g["partition"]), int(g["programs"])
    st, counts = oracle_mod.partition_paint(1, n, 1, part)
    assert st == oracle_mod.PART_OK and counts.sum() == n
    assert (n + part - 1) // part == progs
    # one program per sub-tensor: every element painted exactly once
    assert np.all(counts == 1)
    # the example's arithmetic, ones + ones, through the oracle's product:
    # [1 1] . [[1],[1]] = 2 for every element
    R = oracle_mod.gemm(np.ones((n, 2)), np.ones((2, 1)))
    assert np.all(R == float(g["value"]))


def _race_map(B, H, M_tiles):
    """Program (b, h1, h2) of the racy head permute stores destination
    sub-tensors (b, m, h2) for every m.  The destination, viewed as a 2-D
    grid of (b*M_tiles + m) x h2 sub-tensors of 1 x 1, is what is painted."""
    offs, tiles = [0], []
    for b in range(B):
        for h1 in range(H):
            for h2 in range(H):
                for m in range(M_tiles):
                    tiles.append((b * M_tiles + m) * H + h2)
                offs.append(len(tiles))
    return offs, tiles


def test_listing5_race_is_overlap(oracle_mod):
    g = {r[0]: r[1] for r in read_golden("listing5_race.txt")}
    B, H, Mt = int(g["B"]), int(g["H"]), int(g["M_tiles"])
    offs, tiles = _race_map(B, H, Mt)
    st, counts = oracle_mod.partition_paint(B * Mt, H, 1, 1, offs, tiles)
    assert st == oracle_mod.PART_OVERLAP and g["expected"] == "OVERLAP"
    assert counts.max() == int(g["multiplicity"]) == counts.min()


def test_partition_paint_rules(oracle_mod):
    o = oracle_mod
    # clipped edge tiles still cover exactly once
    st, c = o.partition_paint(100, 70, 32, 32)
    assert st == o.PART_OK and np.all(c == 1)
    # a persistent map: 3 programs walking 12 tiles with stride 3
    offs, tiles = [0], []
    for p in range(3):
        tiles += list(range(p, 12, 3))
        offs.append(len(tiles))
    st, c = o.partition_paint(96, 128, 32, 32, offs, tiles)
    assert st == o.PART_OK and np.all(c == 1)
    # a tile given to two programs
    st, c = o.partition_paint(96, 128, 32, 32, [0, 2, 4], [0, 1, 1, 2])
    assert st == o.PART_OVERLAP
    # a missing tile
    st, c = o.partition_paint(64, 64, 32, 32, [0, 2, 3], [0, 1, 2])
    assert st == o.PART_NOCOVER and c.sum() == 3 * 32 * 32
    # out-of-grid tile id, bad shapes
    st, _ = o.partition_paint(64, 64, 32, 32, [0, 1], [4])
    assert st == o.PART_ARG
    st, _ = o.partition_paint(64, 64, 0, 32)
    assert st == o.PART_ARG


def test_ranges_intersect(oracle_mod):
    o = oracle_mod
    assert o.ranges_intersect(0, 10, 9, 5)
    assert not o.ranges_intersect(0, 10, 10, 5)
    assert not o.ranges_intersect(0, 0, 0, 5)
    assert o.ranges_intersect(100, 1, 50, 51)
