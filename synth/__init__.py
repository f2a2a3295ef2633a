"""Seeded synthetic inputs for the tile-partitioned GEMM workloads.

This module is shared by the tests, the benchmark and the smoke check.  It
only draws random numbers and rounds them to the storage formats the
workloads are defined in (bfloat16 by round-to-nearest-even, OCP E4M3 with
per-channel scales); it holds none of the GEMM arithmetic.  All draws come
from torch's CPU generator so they are identical on every machine.

Workloads (shapes and value distributions):
  * plain FP32 product, 256^3, entries uniform in [-1, 1), output split into
    32 x 32 sub-tensors; a small-integer variant with entries in [-4, 4];
  * BF16 product 8192^3 with entries N(0, 1) rounded to bf16; the split
    precision variant keeps the fp32 N(0, 1) draws;
  * decode-shaped products, M in {1, 8}, (N, K) in {(5120, 5120),
    (51200, 5120), (5120, 25600)}, weights N(0, 0.02) stored N x K in bf16 or
    E4M3 with per-output-channel fp32 scales, activations N(0, 1) in bf16;
  * a batch of 64 independent bf16 products, M uniform in [1, 2048], N and K
    uniform multiples of 128 in [1024, 8192], entries N(0, 1);
  * tile-picker shapes: M, N, K log-uniform in [1, 16384], dtype bf16 or fp8.
"""
import math

import torch

E4M3_MAX = 448.0


def gen(seed: int) -> torch.Generator:
    g = torch.Generator(device="cpu")
    g.manual_seed(int(seed))
    return g


def uniform_pm1(shape, seed: int) -> torch.Tensor:
    """fp32 entries uniform in [-1, 1)."""
    return torch.rand(shape, generator=gen(seed), dtype=torch.float32) * 2 - 1


def small_int(shape, seed: int, lo: int = -4, hi: int = 4) -> torch.Tensor:
    """fp32 tensor of integers uniform in [lo, hi] (exact in fp32/bf16/e4m3)."""
    return torch.randint(lo, hi + 1, shape, generator=gen(seed)).to(
        torch.float32)


def normal(shape, seed: int, std: float = 1.0) -> torch.Tensor:
    """fp32 entries N(0, std^2)."""
    return torch.randn(shape, generator=gen(seed), dtype=torch.float32) * std


def to_bf16(x: torch.Tensor) -> torch.Tensor:
    """Round to bfloat16 (round-to-nearest-even)."""
    return x.to(torch.bfloat16)


def quant_e4m3_rows(w: torch.Tensor):
    """Quantise each row of w to OCP E4M3 with one fp32 scale per row.

    scale_r = amax_r / 448 (1 when the row is all zero); codes are
    round-to-nearest-even of w / scale, saturated to +-448.
    Returns (codes as torch.float8_e4m3fn, scales fp32 of shape (rows,)).
    """
    w = w.to(torch.float32)
    amax = w.abs().amax(dim=1)
    scale = torch.where(amax > 0, amax / E4M3_MAX, torch.ones_like(amax))
    q = (w / scale[:, None]).clamp(-E4M3_MAX, E4M3_MAX)
    return q.to(torch.float8_e4m3fn), scale.to(torch.float32)


def quant_e4m3_cols(w: torch.Tensor):
    """Per-column version of quant_e4m3_rows (scales of shape (cols,))."""
    q, s = quant_e4m3_rows(w.t().contiguous())
    return q.t().contiguous(), s


def ceil_to(x: int, m: int) -> int:
    return (x + m - 1) // m * m


def grouped_shapes(seed: int = 4, n: int = 64):
    """n problems (M, N, K): M ~ U{1..2048}, N, K ~ 128 * U{8..64}."""
    g = gen(seed)
    m = torch.randint(1, 2049, (n,), generator=g)
    nn = torch.randint(8, 65, (n,), generator=g) * 128
    kk = torch.randint(8, 65, (n,), generator=g) * 128
    return [(int(a), int(b), int(c)) for a, b, c in zip(m, nn, kk)]


def picker_shapes(seed: int, n: int, lo: int = 1, hi: int = 16384):
    """n shapes (M, N, K, dtype) with M, N, K log-uniform in [lo, hi] and
    dtype 'bf16' or 'fp8' with equal probability."""
    g = gen(seed)
    u = torch.rand((n, 3), generator=g, dtype=torch.float64)
    d = torch.randint(0, 2, (n,), generator=g)
    lo_l, hi_l = math.log(lo), math.log(hi)
    dims = torch.round(torch.exp(lo_l + u * (hi_l - lo_l))).to(torch.int64)
    dims = dims.clamp(lo, hi)
    return [(int(a), int(b), int(c), "fp8" if int(t) else "bf16")
            for (a, b, c), t in zip(dims.tolist(), d)]


DECODE_SHAPES = [(5120, 5120), (51200, 5120), (5120, 25600)]


def mlp_init(n_in: int, hidden: int, depth: int, seed: int) -> torch.Tensor:
    """Initial cost-model parameters (float32, flat): per layer W (out x in)
    drawn uniform in +-sqrt(6 / in) (He-uniform), then b = 0; the output
    layer has one unit."""
    g = gen(seed)
    dims = [n_in] + [hidden] * depth + [1]
    parts = []
    for l in range(depth + 1):
        i, o = dims[l], dims[l + 1]
        lim = math.sqrt(6.0 / i)
        parts.append((torch.rand((o, i), generator=g, dtype=torch.float64)
                      * 2 - 1).mul(lim).reshape(-1))
        parts.append(torch.zeros(o, dtype=torch.float64))
    return torch.cat(parts).to(torch.float32)


def random_codes16(shape, seed: int) -> torch.Tensor:
    """Uniformly random 16-bit patterns (int16): as bfloat16 they cover every
    exponent, both zeros, subnormals, infinities and NaNs."""
    return torch.randint(-32768, 32768, shape, generator=gen(seed),
                         dtype=torch.int32).to(torch.int16)


def bimodal_sizes(seed: int, n: int = 2000, p_big: float = 0.2,
                  small: int = 512, big: int = 2048):
    """n square GEMM sizes: `big` with probability p_big, else `small`."""
    u = torch.rand(n, generator=gen(seed))
    return [big if float(v) < p_big else small for v in u]
