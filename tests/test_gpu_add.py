"""Parity of the element-wise add z = x + y with the oracle (needs a GPU).

Every element is compared bit for bit: the oracle's sum is the exact sum
rounded once to the storage format, which is also what the kernel computes
(one binary32 add, then round to nearest even), so no tolerance applies.
NaN results compare as NaN (their payload is not fixed by the format).
Inputs: uniformly random 16/32-bit patterns (every exponent, zeros,
subnormals, infinities, NaNs) and normal-distributed values."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import note

pytestmark = pytest.mark.gpu

tg = pytest.importorskip("paper_2606_15991_amd")
DEV = "cuda:0"


def codes_bf16(shape, seed):
    return synth.random_codes16(shape, seed).view(torch.bfloat16)


def codes_f32(shape, seed):
    lo = synth.random_codes16(shape, seed).to(torch.int32) & 0xFFFF
    hi = synth.random_codes16(shape, seed + 1).to(torch.int32)
    return ((hi << 16) | lo).view(torch.float32)


def bits16(t):
    return t.detach().cpu().contiguous().view(torch.int16).numpy() \
        .view(np.uint16)


def expect(x, y):
    if x.dtype == torch.bfloat16:
        return oracle.add_bf16(bits16(x), bits16(y))
    return oracle.add_f32(x.cpu().numpy(), y.cpu().numpy())


def assert_same(z, want):
    z = z.detach().cpu().contiguous()
    if z.dtype == torch.bfloat16:
        got = bits16(z)
        nan_g = np.isnan(oracle.decode_bf16(got))
        nan_w = np.isnan(oracle.decode_bf16(want))
    else:
        got = z.numpy().view(np.uint32)
        want = np.asarray(want, np.float32)
        nan_g, nan_w = np.isnan(z.numpy()), np.isnan(want)
        want = want.view(np.uint32)
    assert np.array_equal(nan_g, nan_w)
    bad = np.argwhere((got != want) & ~nan_w)
    assert bad.size == 0, f"{len(bad)} mismatches, first at {bad[:4]}"


def run_add(x, y, bm=0, bn=0, count=False, **kw):
    xd, yd = x.to(DEV), y.to(DEV)
    z = torch.full(x.shape, 7.0, dtype=x.dtype, device=DEV)
    wc = torch.zeros(x.shape, dtype=torch.int32, device=DEV) if count else None
    tg.tile_add(xd, yd, z, bm, bn, write_count=wc, **kw)
    torch.cuda.synchronize()
    return z, wc


SHAPES = [(1, 1), (1, 7), (3, 1000), (257, 1031), (64, 4096), (2, 70000),
          (5, 131072)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("dt", ["bf16", "f32"])
def test_add_random_codes_bit_exact(shape, dt):
    note("add codes", dt, shape)
    mk = codes_bf16 if dt == "bf16" else codes_f32
    x, y = mk(shape, 11), mk(shape, 29)
    z, _ = run_add(x, y)
    assert_same(z, expect(x, y))


@pytest.mark.parametrize("bm,bn", [(7, 24), (16, 8), (3, 5), (1, 1024),
                                   (300, 2000), (1, 1), (64, 64)])
def test_add_partitions_each_element_stored_once(bm, bn):
    note("add partition", bm, bn)
    x, y = codes_bf16((257, 1031), 3), codes_bf16((257, 1031), 4)
    z, wc = run_add(x, y, bm, bn, count=True)
    assert tg.tile_add.last_partition == (bm, bn)
    assert_same(z, expect(x, y))
    assert int(wc.min()) == 1 and int(wc.max()) == 1


@pytest.mark.parametrize("dt", [torch.bfloat16, torch.float32])
@pytest.mark.parametrize("off", [0, 1, 3])
def test_add_strided_and_unaligned_views(dt, off):
    note("add views", dt, off)
    rows, cols, ld = 129, 1000, 1037
    base = [synth.normal((rows, ld + 8), s).to(dt).to(DEV) for s in (5, 6, 7)]
    x = base[0][:, off:off + cols]
    y = base[1][:, 2:2 + cols]
    zbuf = base[2].clone()
    z = zbuf[:, off:off + cols]
    tg.tile_add(x, y, z)
    torch.cuda.synchronize()
    want = expect(x.cpu(), y.cpu()) if dt == torch.bfloat16 else \
        oracle.add_f32(x.cpu().numpy(), y.cpu().numpy())
    assert_same(z, want)
    # the bytes of the buffer outside the view are untouched
    keep = torch.ones_like(zbuf, dtype=torch.bool)
    keep[:, off:off + cols] = False
    assert torch.equal(zbuf[keep].cpu(), base[2][keep].cpu())


def test_add_normal_values_workload_distribution():
    note("add normal 4096x4096")
    x = synth.to_bf16(synth.normal((4096, 4096), 41))
    y = synth.to_bf16(synth.normal((4096, 4096), 42))
    z, _ = run_add(x, y)
    assert_same(z, expect(x, y))


def test_add_full_size_sampled():
    """2^28 bf16 elements (the measured size): sampled elements, and the
    first and last row whole, against the oracle."""
    n = 16384
    note("add 2^28 sampled")
    x = codes_bf16((n, n), 51).to(DEV)
    y = synth.to_bf16(synth.normal((n, n), 52)).to(DEV)
    z = torch.empty_like(x)
    tg.tile_add(x, y, z)
    torch.cuda.synchronize()
    g = torch.Generator().manual_seed(5)
    idx = torch.randint(0, n * n, (1 << 20,), generator=g)
    xs, ys, zs = (t.view(-1)[idx.to(DEV)].cpu() for t in (x, y, z))
    assert_same(zs, expect(xs, ys))
    for r in (0, n - 1):
        assert_same(z[r], expect(x[r].cpu(), y[r].cpu()))


@pytest.mark.parametrize("shape", [(0, 5), (5, 0), (0, 0)])
def test_add_empty(shape):
    note("add empty", shape)
    x = torch.zeros(shape, dtype=torch.bfloat16, device=DEV)
    z = torch.empty_like(x)
    tg.tile_add(x, x.clone(), z)
    torch.cuda.synchronize()


def test_add_rejects_aliasing_and_mismatch():
    note("add argument errors")
    x = torch.ones((64, 64), dtype=torch.bfloat16, device=DEV)
    y = torch.ones_like(x)
    with pytest.raises(tg.TileGemmError):
        tg.tile_add(x, y, x)                    # z is an input
    buf = torch.ones((64, 128), dtype=torch.bfloat16, device=DEV)
    with pytest.raises(tg.TileGemmError):
        tg.tile_add(buf[:, :64], y, buf[:, 32:96])   # z overlaps x
    with pytest.raises(tg.TileGemmError):
        tg.tile_add(x, y.float(), torch.empty_like(x))
    with pytest.raises(tg.TileGemmError):
        tg.tile_add(x, y[:, :32], torch.empty_like(x))
    e = torch.ones((64, 64), dtype=torch.float8_e4m3fn, device=DEV)
    with pytest.raises(tg.TileGemmError):
        tg.tile_add(e, e.clone(), torch.empty_like(e))
    torch.cuda.synchronize()
    assert float(x.float().sum()) == 64 * 64


# ------------------------------------------------------------ z = x * y

def run_mul(x, y, bm=0, bn=0, count=False):
    xd, yd = x.to(DEV), y.to(DEV)
    z = torch.full(x.shape, 7.0, dtype=x.dtype, device=DEV)
    wc = torch.zeros(x.shape, dtype=torch.int32, device=DEV) if count else None
    tg.tile_mul(xd, yd, z, bm, bn, write_count=wc)
    torch.cuda.synchronize()
    return z, wc


@pytest.mark.parametrize("shape", [(1, 2048), (3, 1000), (257, 1031),
                                   (2, 70000)])
def test_mul_bf16_random_codes(shape):
    """Bit-exact where the exact product is 0, infinite, NaN or at least
    2^-126 in magnitude; below that the product is first rounded to the
    binary32 subnormal grid, and the result is within 2^-133 (one bf16
    subnormal step) of the exact product."""
    note("mul codes bf16", shape)
    x, y = codes_bf16(shape, 13), codes_bf16(shape, 31)
    z, _ = run_mul(x, y)
    xb, yb = bits16(x), bits16(y)
    exact = oracle.decode_bf16(xb) * oracle.decode_bf16(yb)
    want = oracle.mul_bf16(xb, yb)
    got = bits16(z)
    dg = oracle.decode_bf16(got)
    small = (np.abs(exact) < 2.0 ** -126) & (exact != 0)
    nan_w = np.isnan(oracle.decode_bf16(want))
    assert np.array_equal(np.isnan(dg), nan_w)
    big = ~small & ~nan_w
    assert np.array_equal(got[big], want[big])
    assert np.all(np.abs(dg[small] - exact[small]) <= 2.0 ** -133)


@pytest.mark.parametrize("shape", [(1, 2048), (257, 1031)])
def test_mul_f32_random_codes_bit_exact(shape):
    note("mul codes f32", shape)
    x, y = codes_f32(shape, 17), codes_f32(shape, 37)
    z, _ = run_mul(x, y)
    assert_same(z, oracle.mul_f32(x.numpy(), y.numpy()))


def test_mul_normal_values_partition_bit_exact():
    note("mul normal, partition 5 x 40")
    x = synth.to_bf16(synth.normal((129, 1000), 43))
    y = synth.to_bf16(synth.normal((129, 1000), 44))
    z, wc = run_mul(x, y, 5, 40, count=True)
    assert_same(z, oracle.mul_bf16(bits16(x), bits16(y)))
    assert int(wc.min()) == 1 and int(wc.max()) == 1
