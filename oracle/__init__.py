"""CPU oracle for the tile-partitioned GEMM  C = A.B  (binary64, plain loops).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  It shares no code
with the HIP path and never imports it.

What it computes (arxiv 2606.15991):
  * gemm / gemm_scaled / gemm_entries -- the plain definition of the
    product that the mapped-partition GEMM of Sec. 3.6 reaches: every owned
    output tile is a zero-initialised sum of tile products over K, stored
    once, i.e. R[i,j] = sum_k A[i,k] B[k,j].  Quantised (FP8) operands are
    decoded exactly and the per-row / per-column scales are applied to the
    binary64 sum.
  * rel_fro -- relative Frobenius error in binary64.
  * partition_paint -- the ownership rules of Sec. 3.4 and App. A
    (injective program -> sub-tensor map, covering grid) checked by painting
    every output element.
  * decode_bf16 / decode_e4m3fn -- exact decoding of the two 16/8-bit
    element formats from their published bit layouts.
  * round_bf16 / add_bf16 / add_f32 -- the element-wise add of Sec. 2 (the
    first listing; measured element-wise in Sec. 5.1): each output element
    is the exact sum of the two input elements rounded once to the storage
    format, to nearest with ties to even.  The binary64 sum of two bf16 or
    two binary32 values, rounded again to the 8- or 24-bit format, is that
    correctly rounded sum (53 >= 2p + 2, so the double rounding is
    innocuous).
  * mul_bf16 / mul_f32 -- the element-wise product of the execution-mode
    measurement of Sec. 5.2, correctly rounded.  The binary64 product of
    two bf16 values (8-bit significands, exponents within binary64's range)
    or two binary32 values (24-bit significands: 48 bits) is exact, so one
    rounding to the storage format is the definition.
  * rms_norm -- the RMS normalisation of the decode layer in Sec. 3.2's
    graph-scope listing, y = x * w / sqrt(mean(x^2) + eps) per row, in
    binary64 (the usual RMSNorm definition; the paper names the operation
    and its eps without writing the formula out).
  * residual_add -- the residual add that closes the decode layer of
    Sec. 3.2's graph-scope listing (layer output = matvec result + layer
    input), applied to a finished binary64 product: scales belong to the
    product, the residual is added unscaled, the sum is stored once.
  * mlp (submodule) -- binary64 forward/backward of the tile-picker MLP and
    its Adam update.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_i64 = ctypes.c_int64
_dp = ctypes.POINTER(ctypes.c_double)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.oracle_gemm.argtypes = [_i64, _i64, _i64, _dp, _i64, _dp, _i64,
                                ctypes.c_int, _dp, _i64]
    lib.oracle_gemm.restype = None
    lib.oracle_gemm_scaled.argtypes = [_i64, _i64, _i64, _dp, _i64, _dp,
                                       _i64, ctypes.c_int, _dp, _dp, _dp,
                                       _i64]
    lib.oracle_gemm_scaled.restype = None
    lib.oracle_gemm_entries.argtypes = [_i64, _dp, _i64, _dp, _i64,
                                        ctypes.c_int, _dp, _dp,
                                        ctypes.c_void_p, ctypes.c_void_p,
                                        _i64, _dp]
    lib.oracle_gemm_entries.restype = None
    lib.oracle_rel_fro.argtypes = [_dp, _dp, _i64]
    lib.oracle_rel_fro.restype = ctypes.c_double
    lib.oracle_partition_paint.argtypes = [_i64, _i64, _i64, _i64, _i64,
                                           ctypes.c_void_p, ctypes.c_void_p,
                                           ctypes.c_void_p]
    lib.oracle_partition_paint.restype = ctypes.c_int
    lib.oracle_ranges_intersect.argtypes = [ctypes.c_uint64] * 4
    lib.oracle_ranges_intersect.restype = ctypes.c_int
    lib.oracle_decode_bf16.argtypes = [ctypes.c_void_p, _dp, _i64]
    lib.oracle_decode_bf16.restype = None
    lib.oracle_decode_e4m3fn.argtypes = [ctypes.c_void_p, _dp, _i64]
    lib.oracle_decode_e4m3fn.restype = None
    lib.oracle_num_threads.argtypes = []
    lib.oracle_num_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def decode_bf16(bits) -> np.ndarray:
    """bfloat16 bit patterns (any integer array of 16-bit codes) -> float64."""
    b = np.ascontiguousarray(np.asarray(bits).astype(np.uint16))
    out = np.empty(b.shape, dtype=np.float64)
    _load().oracle_decode_bf16(b.ctypes.data, out.ctypes.data_as(_dp), b.size)
    return out


def decode_e4m3fn(codes) -> np.ndarray:
    """OCP E4M3 (e4m3fn) byte codes -> float64 (NaN for S.1111.111)."""
    b = np.ascontiguousarray(np.asarray(codes).astype(np.uint8))
    out = np.empty(b.shape, dtype=np.float64)
    _load().oracle_decode_e4m3fn(b.ctypes.data, out.ctypes.data_as(_dp),
                                 b.size)
    return out


def gemm(A, B, b_nk: bool = False, sa=None, sb=None) -> np.ndarray:
    """R = diag(sa) . A . B . diag(sb) in binary64.

    A: (M, K).  B: (K, N), or (N, K) when b_nk.  sa: (M,) or None,
    sb: (N,) or None.
    """
    A, pa = _f64(A)
    B, pb = _f64(B)
    M, K = A.shape
    N = B.shape[0] if b_nk else B.shape[1]
    assert (B.shape[1] if b_nk else B.shape[0]) == K
    R = np.empty((M, N), dtype=np.float64)
    lib = _load()
    if sa is None and sb is None:
        lib.oracle_gemm(M, N, K, pa, K, pb, B.shape[1], int(b_nk),
                        R.ctypes.data_as(_dp), N)
    else:
        sa_a, psa = _f64(sa) if sa is not None else (None, None)
        sb_a, psb = _f64(sb) if sb is not None else (None, None)
        lib.oracle_gemm_scaled(M, N, K, pa, K, pb, B.shape[1], int(b_nk),
                               psa, psb, R.ctypes.data_as(_dp), N)
    return R


def gemm_entries(A, B, ii, jj, b_nk: bool = False, sa=None,
                 sb=None) -> np.ndarray:
    """Entries R[ii[t], jj[t]] of diag(sa) . A . B . diag(sb)."""
    A, pa = _f64(A)
    B, pb = _f64(B)
    K = A.shape[1]
    ii = np.ascontiguousarray(ii, dtype=np.int64)
    jj = np.ascontiguousarray(jj, dtype=np.int64)
    out = np.empty(ii.shape, dtype=np.float64)
    sa_a, psa = _f64(sa) if sa is not None else (None, None)
    sb_a, psb = _f64(sb) if sb is not None else (None, None)
    _load().oracle_gemm_entries(K, pa, K, pb, B.shape[1], int(b_nk), psa, psb,
                                ii.ctypes.data, jj.ctypes.data, ii.size,
                                out.ctypes.data_as(_dp))
    return out


def rel_fro(C, R) -> float:
    """||C - R||_F / ||R||_F in binary64 (||C||_F when R is all zero)."""
    C, pc = _f64(C)
    R, pr = _f64(R)
    assert C.size == R.size
    return float(_load().oracle_rel_fro(pc, pr, C.size))


PART_OK, PART_ARG, PART_OVERLAP, PART_NOCOVER = 0, 1, 4, 5


def round_bf16(v) -> np.ndarray:
    """binary64 values -> bfloat16 bit patterns (uint16), round to nearest,
    ties to even, overflow to infinity, NaN -> 0x7FC0 (sign kept).

    bfloat16 keeps 8 significant bits and binary32's exponent range, so the
    spacing of representable values around |v| in [2^(e-1), 2^e) is
    2^(e-8), and never below the subnormal spacing 2^-133."""
    v = np.asarray(v, dtype=np.float64)
    _, e = np.frexp(v)
    q = np.ldexp(1.0, np.maximum(e.astype(np.int64) - 8, -133))
    with np.errstate(over="ignore", invalid="ignore"):
        r = np.round(v / q) * q                  # np.round: ties to even
        r = np.where(np.abs(r) >= 2.0 ** 128, np.copysign(np.inf, v), r)
        r = np.where(np.isinf(v), v, r)
        bits = (r.astype(np.float32).view(np.uint32) >> 16).astype(np.uint16)
    nan = np.isnan(v)
    if nan.any():
        sign = np.signbit(v).astype(np.uint16) << 15
        bits = np.where(nan, sign | np.uint16(0x7FC0), bits)
    return bits.astype(np.uint16)


def add_bf16(x_bits, y_bits) -> np.ndarray:
    """z = x + y for bfloat16 bit patterns: the correctly rounded sum."""
    with np.errstate(invalid="ignore"):          # inf + (-inf) -> NaN
        return round_bf16(decode_bf16(x_bits) + decode_bf16(y_bits))


def add_f32(x, y) -> np.ndarray:
    """z = x + y for binary32 arrays: the correctly rounded sum."""
    with np.errstate(over="ignore", invalid="ignore"):
        s = np.asarray(x, np.float64) + np.asarray(y, np.float64)
        return s.astype(np.float32)


def rms_norm(x, w, eps: float) -> np.ndarray:
    """binary64 y[r, j] = x[r, j] w[j] / sqrt(mean_j(x[r, j]^2) + eps)."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    w = np.asarray(w, dtype=np.float64).reshape(-1)
    ms = np.mean(x * x, axis=1, keepdims=True)
    return x * w / np.sqrt(ms + float(eps))


def mul_bf16(x_bits, y_bits) -> np.ndarray:
    """z = x * y for bfloat16 bit patterns: the correctly rounded product
    (the binary64 product of two 8-bit significands is exact)."""
    with np.errstate(invalid="ignore", over="ignore", under="ignore"):
        return round_bf16(decode_bf16(x_bits) * decode_bf16(y_bits))


def mul_f32(x, y) -> np.ndarray:
    """z = x * y for binary32 arrays: the correctly rounded product (the
    binary64 product of two 24-bit significands is exact)."""
    with np.errstate(over="ignore", invalid="ignore", under="ignore"):
        s = np.asarray(x, np.float64) * np.asarray(y, np.float64)
        return s.astype(np.float32)


def partition_paint(M, N, bm, bn, prog_offsets=None, prog_tiles=None):
    """Paint an M x N output with per-element owner counts.

    Returns (status, counts) where status is PART_OK, PART_OVERLAP,
    PART_NOCOVER or PART_ARG.  With no map, one program per sub-tensor.
    """
    counts = np.zeros((max(M, 0), max(N, 0)), dtype=np.int32)
    if prog_offsets is None:
        st = _load().oracle_partition_paint(M, N, bm, bn, 0, None, None,
                                            counts.ctypes.data)
    else:
        po = np.ascontiguousarray(prog_offsets, dtype=np.int32)
        pt = np.ascontiguousarray(prog_tiles, dtype=np.int32)
        if pt.size == 0:
            pt = np.zeros(1, dtype=np.int32)
        st = _load().oracle_partition_paint(M, N, bm, bn, po.size - 1,
                                            po.ctypes.data, pt.ctypes.data,
                                            counts.ctypes.data)
    return int(st), counts


def ranges_intersect(a: int, na: int, b: int, nb: int) -> bool:
    return bool(_load().oracle_ranges_intersect(a, na, b, nb))


def rms_norm_matvec(x, nw, W, eps: float, sw=None) -> np.ndarray:
    """The decode layer's normalisation fused into its product (Sec. 3.2,
    graph-scope listing: rms_norm, then the matvec), binary64:

        y[m, n] = s_m * sum_k round_bf16(x[m, k] * nw[k]) * W[n, k] * sw[n]
        s_m     = 1 / sqrt(mean_k x[m, k]^2 + eps)

    W is stored N x K.  Reading: the weighted activation x * nw is held at
    the width of the stored normalised buffer of the unfused chain (bf16,
    round to nearest even) before the contraction, and the row scale s_m
    multiplies the finished sum; sw (N,) or None are per-output scales."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    nw = np.asarray(nw, dtype=np.float64).reshape(-1)
    xw = decode_bf16(round_bf16(x * nw))
    s = 1.0 / np.sqrt(np.mean(x * x, axis=1) + float(eps))
    return gemm(xw, W, b_nk=True, sa=s, sb=sw)


def residual_add(P, R) -> np.ndarray:
    """out = P + R in binary64: the decode layer's residual add (Sec. 3.2,
    graph-scope listing) on a finished product P (scales already applied to
    P; the residual R is added as it is).  Rounding the result to the
    output format is the caller's one rounding."""
    return np.asarray(P, dtype=np.float64) + np.asarray(R, dtype=np.float64)
