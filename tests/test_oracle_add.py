"""Pins of the oracle's element-wise add and its bfloat16 rounding (CPU).

The rounding is pinned to the bfloat16 format itself: every finite code
round-trips through the oracle's independent C decoder, every midpoint of
two neighbouring codes goes to the even one, random values go to their
nearest code by brute-force search, and values that the format's layout
fixes (1, -2, the largest finite value, the smallest subnormal, the overflow
tie) give their known bit patterns.  The binary32 add is pinned to numpy's
IEEE binary32 addition, which is correctly rounded by definition."""
import numpy as np
import pytest

import oracle

ALL = np.arange(65536, dtype=np.uint32).astype(np.uint16)
POS_FINITE = np.arange(0x7F80, dtype=np.uint32).astype(np.uint16)


def _dec(c):
    return oracle.decode_bf16(np.asarray(c, dtype=np.uint16))


@pytest.mark.parametrize("v,bits", [
    (1.0, 0x3F80), (-2.0, 0xC000), (0.5, 0x3F00), (3.0, 0x4040),
    ((2 - 2 ** -7) * 2.0 ** 127, 0x7F7F),        # largest finite
    (2.0 ** -126, 0x0080),                       # smallest normal
    (2.0 ** -133, 0x0001),                       # smallest subnormal
    (2.0 ** -134, 0x0000),                       # tie with 0 -> even (0)
    (3 * 2.0 ** -134, 0x0002),                   # tie 1|2 quanta -> 2
    (1 + 2.0 ** -8, 0x3F80),                     # tie -> even mantissa
    (1 + 3 * 2.0 ** -8, 0x3F82),                 # tie -> even mantissa
    (1 + 2.0 ** -8 + 2.0 ** -30, 0x3F81),        # just above the tie
    (2.0 ** 128 * (1 - 2.0 ** -9), 0x7F80),      # overflow tie -> inf
    (2.0 ** 128 * (1 - 2.0 ** -9) - 2.0 ** 100, 0x7F7F),
    (-0.0, 0x8000), (float("inf"), 0x7F80), (float("-inf"), 0xFF80),
    (1e300, 0x7F80), (-1e-300, 0x8000),
])
def test_round_bf16_known_patterns(v, bits):
    assert int(oracle.round_bf16(v)) == bits


def test_round_bf16_round_trips_every_code():
    dec = _dec(ALL)
    back = oracle.round_bf16(dec)
    nan = np.isnan(dec)
    assert nan.sum() == 2 * 127                  # exponent 255, mantissa != 0
    assert np.array_equal(back[~nan], ALL[~nan])
    assert np.all(np.isnan(_dec(back[nan])))


def test_round_bf16_midpoints_go_to_even_code():
    lo, hi = POS_FINITE[:-1], POS_FINITE[1:]
    mid = (_dec(lo) + _dec(hi)) / 2              # exact in binary64
    got = oracle.round_bf16(mid)
    want = np.where(lo % 2 == 0, lo, hi)
    assert np.array_equal(got, want)
    assert np.array_equal(oracle.round_bf16(-mid), want | np.uint16(0x8000))


def test_round_bf16_is_nearest_by_search():
    rng = np.random.default_rng(7)
    table = _dec(POS_FINITE)                     # increasing
    v = np.ldexp(rng.random(20000) + 0.5, rng.integers(-140, 128, 20000))
    v = v[v < table[-1]]
    got = _dec(oracle.round_bf16(v))
    i = np.searchsorted(table, v)                # table[i-1] < v <= table[i]
    below = table[np.maximum(i - 1, 0)]
    above = table[i]
    best = np.minimum(np.abs(v - below), np.abs(above - v))
    assert np.all(np.abs(got - v) == best)
    assert np.all((got == below) | (got == above))


def test_add_bf16_pinned_cases():
    b = lambda v: oracle.round_bf16(np.asarray(v, dtype=np.float64))
    add = lambda x, y: int(np.ravel(oracle.add_bf16(b(x), b(y)))[0])
    assert add(1.0, 2.0 ** -8) == 0x3F80          # tie -> 1
    assert add(1 + 2.0 ** -7, 2.0 ** -8) == 0x3F82  # tie -> 1 + 2^-6
    assert add(2.0 ** 100, 2.0 ** -100) == int(b(2.0 ** 100))
    assert add(2.0 ** -133, 2.0 ** -133) == 0x0002
    big = (2 - 2 ** -7) * 2.0 ** 127
    assert add(big, big) == 0x7F80
    assert add(-big, -big) == 0xFF80
    assert np.isnan(_dec(oracle.add_bf16(0x7F80, 0xFF80)))
    assert add(-0.0, -0.0) == 0x8000
    assert add(0.0, -0.0) == 0x0000


def test_add_bf16_small_integers_exact():
    ints = np.arange(-128, 129, dtype=np.float64)
    x, y = np.meshgrid(ints, ints)
    z = oracle.add_bf16(oracle.round_bf16(x), oracle.round_bf16(y))
    assert np.array_equal(_dec(z), x + y)        # |x + y| <= 256: 8 bits


def test_add_bf16_identities_over_every_code():
    dec = _dec(ALL)
    ok = ~np.isnan(dec)
    zero = np.zeros_like(ALL)
    plus0 = oracle.add_bf16(ALL, zero)
    want = np.where(ALL == 0x8000, np.uint16(0), ALL)   # -0 + +0 = +0
    assert np.array_equal(plus0[ok], want[ok])
    neg = ALL ^ np.uint16(0x8000)
    fin = ok & np.isfinite(dec)
    assert np.all(oracle.add_bf16(ALL, neg)[fin] == 0)  # x + (-x) = +0
    rng = np.random.default_rng(3)
    x, y = rng.integers(0, 65536, (2, 50000)).astype(np.uint16)
    a, c = oracle.add_bf16(x, y), oracle.add_bf16(y, x)
    okxy = ~np.isnan(_dec(a))
    assert np.array_equal(a[okxy], c[okxy])      # commutative


def test_add_f32_is_ieee_binary32_addition():
    rng = np.random.default_rng(11)
    bits = rng.integers(0, 2 ** 32, (2, 200000), dtype=np.uint64)
    x, y = bits.astype(np.uint32).view(np.float32)
    x = np.concatenate([x, rng.standard_normal(1000).astype(np.float32),
                        np.float32([3.4e38, -0.0, 1e-45, 1.0])])
    y = np.concatenate([y, rng.standard_normal(1000).astype(np.float32),
                        np.float32([3.4e38, -0.0, 1e-45, 2.0 ** -24])])
    with np.errstate(over="ignore", invalid="ignore"):
        want = x + y
    got = oracle.add_f32(x, y)
    nan = np.isnan(want)
    assert np.array_equal(np.isnan(got), nan)
    assert np.array_equal(got[~nan].view(np.uint32),
                          want[~nan].view(np.uint32))


def test_mul_bf16_pinned_cases():
    b = lambda v: oracle.round_bf16(np.asarray(v, dtype=np.float64))
    mul = lambda x, y: int(np.ravel(oracle.mul_bf16(b(x), b(y)))[0])
    ints = np.arange(-15, 16, dtype=np.float64)
    x, y = np.meshgrid(ints, ints)
    z = oracle.mul_bf16(oracle.round_bf16(x), oracle.round_bf16(y))
    assert np.array_equal(_dec(z), x * y)        # |x y| <= 225: 8 bits
    # (1 + 2^-7)^2 = 1 + 2^-6 + 2^-14: rounds to 1 + 2^-6
    assert mul(1 + 2.0 ** -7, 1 + 2.0 ** -7) == 0x3F82
    # (1 + 3 * 2^-7)(1 + 2^-7) = 1 + 2^-5 + 3 * 2^-14 -> 1 + 2^-5
    assert mul(1 + 3 * 2.0 ** -7, 1 + 2.0 ** -7) == 0x3F84
    assert mul(2.0 ** -70, 2.0 ** -70) == 0x0000    # 2^-140 < 2^-134
    assert mul(2.0 ** -66, 2.0 ** -67) == 0x0001    # 2^-133
    assert mul(2.0 ** 64, 2.0 ** 64) == 0x7F80      # 2^128 overflows
    assert mul(-0.0, 5.0) == 0x8000
    assert np.isnan(_dec(oracle.mul_bf16(0x7F80, 0x0000)))   # inf * 0


def test_mul_bf16_identities_over_every_code():
    dec = _dec(ALL)
    ok = ~np.isnan(dec)
    one = np.full_like(ALL, 0x3F80)
    assert np.array_equal(oracle.mul_bf16(ALL, one)[ok], ALL[ok])
    m1 = np.full_like(ALL, 0xBF80)
    assert np.array_equal(oracle.mul_bf16(ALL, m1)[ok],
                          (ALL ^ np.uint16(0x8000))[ok])
    two = np.full_like(ALL, 0x4000)
    fin = ok & (np.abs(dec) < 2.0 ** 127)
    assert np.array_equal(_dec(oracle.mul_bf16(ALL, two))[fin], 2 * dec[fin])


def test_mul_f32_is_ieee_binary32_multiplication():
    rng = np.random.default_rng(12)
    bits = rng.integers(0, 2 ** 32, (2, 200000), dtype=np.uint64)
    x, y = bits.astype(np.uint32).view(np.float32)
    with np.errstate(over="ignore", invalid="ignore", under="ignore"):
        want = x * y
    got = oracle.mul_f32(x, y)
    nan = np.isnan(want)
    assert np.array_equal(np.isnan(got), nan)
    assert np.array_equal(got[~nan].view(np.uint32),
                          want[~nan].view(np.uint32))


def _round_variant(kind):
    """Plausible mistakes in bf16 rounding, planted on the CPU."""
    def f(v):
        v = np.asarray(v, dtype=np.float64)
        _, e = np.frexp(v)
        shift = {"quantum_off_by_one": -7}.get(kind, -8)
        q = np.ldexp(1.0, np.maximum(e.astype(np.int64) + shift, -133))
        with np.errstate(over="ignore", invalid="ignore"):
            if kind == "ties_away":
                r = np.sign(v) * np.floor(np.abs(v) / q + 0.5) * q
            elif kind == "truncate":
                r = np.trunc(v / q) * q
            elif kind == "no_subnormal_floor":
                q = np.ldexp(1.0, e.astype(np.int64) - 8)
                r = np.round(v / q) * q
                r = np.where(np.abs(r) < 2.0 ** -126, 0.0, r)
            else:
                r = np.round(v / q) * q
            r = np.where(np.abs(r) >= 2.0 ** 128, np.copysign(np.inf, v), r)
            return (r.astype(np.float32).view(np.uint32) >> 16).astype(
                np.uint16)
    return f


@pytest.mark.parametrize("kind", ["ties_away", "truncate",
                                  "quantum_off_by_one", "no_subnormal_floor"])
def test_planted_rounding_mistakes_fail_a_pin(kind):
    f = _round_variant(kind)
    dec = _dec(ALL)
    fin = np.isfinite(dec)
    lo, hi = POS_FINITE[:-1], POS_FINITE[1:]
    mid = (_dec(lo) + _dec(hi)) / 2
    rng = np.random.default_rng(7)
    v = np.ldexp(rng.random(5000) + 0.5, rng.integers(-140, 128, 5000))
    caught = (not np.array_equal(f(dec[fin]), ALL[fin])
              or not np.array_equal(f(mid), np.where(lo % 2 == 0, lo, hi))
              or not np.array_equal(f(v), oracle.round_bf16(v)))
    assert caught
