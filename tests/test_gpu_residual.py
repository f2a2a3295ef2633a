"""The residual epilogue of the decode product: y = s (x W^T) + r, stored
once by the program (or the merge program of a split product) that owns each
element -- the residual add that closes the decode layer of Sec. 3.2's
graph-scope listing, folded into the product's store.

Tolerances (the definition is oracle.residual_add on the binary64 product):
  * binary32 output: relative Frobenius 1e-5 (binary32 accumulation of the
    product, one binary32 add of the residual);
  * bf16 output: relative Frobenius 4e-3 (one bf16 rounding, unit roundoff
    2^-8);
  * small integers (x, W, r integers, every partial sum below 2^24):
    bit-exact, with and without the K split, for both residual types and
    both output types."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import exact64, note, rel_err

pytestmark = pytest.mark.gpu

tg = pytest.importorskip("paper_2606_15991_amd")
DEV = "cuda:0"


def want(x, W, r, sw=None):
    P = oracle.gemm(exact64(x), exact64(W), b_nk=True,
                    sb=None if sw is None else exact64(sw))
    return oracle.residual_add(P, exact64(r))


def run(x, W, y, r, split, sw=None, wc=None, fused=None):
    """One call.  split False: one program per sub-tensor; True: K split
    over three programs per sub-tensor and the merge launch (the fused
    product splits by its own rule when given a workspace)."""
    if fused is not None:
        nw, eps = fused
        return tg.tile_rms_norm_matvec(x, nw, W, y, eps, scale_w=sw,
                                       residual=r, write_count=wc,
                                       workspace=None if split else False)
    return tg.tile_gemm(x, W, y, b_trans=True, scale_b=sw, residual=r,
                        write_count=wc,
                        config={"kind": "skinny", "splitk": 3 if split
                                else 1})


@pytest.mark.parametrize("M,N,K", [(1, 5120, 5120), (8, 1000, 1536),
                                   (3, 264, 200), (16, 48, 4096)])
@pytest.mark.parametrize("out", [torch.float32, torch.bfloat16])
@pytest.mark.parametrize("rdt", [torch.float32, torch.bfloat16])
@pytest.mark.parametrize("split", [False, True])
def test_residual_matches_definition(M, N, K, out, rdt, split):
    note("residual", M, N, K, out, rdt, split)
    x = synth.to_bf16(synth.normal((M, K), 41))
    W = synth.to_bf16(synth.normal((N, K), 42, std=0.02))
    r = synth.normal((M, N), 43).to(rdt)
    y = torch.full((M, N), float("nan"), dtype=out, device=DEV)
    wc = torch.zeros((M, N), dtype=torch.int32, device=DEV)
    run(x.to(DEV), W.to(DEV), y, r.to(DEV), split, wc=wc)
    torch.cuda.synchronize()
    assert torch.all(wc == 1)
    R = want(x, W, r)
    assert rel_err(y.cpu(), R) <= (1e-5 if out == torch.float32 else 4e-3)


@pytest.mark.parametrize("wdt", ["bf16", "e4m3"])
@pytest.mark.parametrize("out", [torch.float32, torch.bfloat16])
@pytest.mark.parametrize("rdt", [torch.float32, torch.bfloat16])
@pytest.mark.parametrize("split", [False, True])
def test_residual_small_integers_exact(wdt, out, rdt, split):
    M, N, K = 5, 1040, 2560
    note("residual exact", wdt, out, rdt, split)
    x = synth.to_bf16(synth.small_int((M, K), 44))
    r = synth.small_int((M, N), 46).to(rdt)
    if wdt == "bf16":
        W, sw = synth.to_bf16(synth.small_int((N, K), 45)), None
    else:
        W = synth.small_int((N, K), 45).to(torch.float8_e4m3fn)
        sw = torch.full((N,), 2.0)
    y = torch.empty((M, N), dtype=out, device=DEV)
    run(x.to(DEV), W.to(DEV), y, r.to(DEV), split,
        sw=None if sw is None else sw.to(DEV))
    torch.cuda.synchronize()
    R = want(x, W, r, sw)
    if out == torch.bfloat16:
        R = oracle.decode_bf16(oracle.round_bf16(R))
    assert np.array_equal(exact64(y.cpu()), R)


@pytest.mark.parametrize("split", [False, True])
def test_fused_norm_matvec_residual_exact(split):
    """Rows of +-1 (eps 0: row scale exactly 1), power-of-two nw, small
    integer W and residual: the fused layer output is exact."""
    M, N, K = 3, 520, 1024
    note("fused residual exact", split)
    rng = np.random.default_rng(47)
    x = torch.from_numpy(np.where(rng.integers(0, 2, (M, K)) == 1, 1.0,
                                  -1.0)).to(torch.bfloat16)
    nw = torch.from_numpy(2.0 ** rng.integers(-1, 2, K)).to(torch.bfloat16)
    W = synth.to_bf16(synth.small_int((N, K), 48))
    r = synth.small_int((M, N), 49).to(torch.bfloat16)
    y = torch.empty((M, N), device=DEV)
    wc = torch.zeros((M, N), dtype=torch.int32, device=DEV)
    run(x.to(DEV), W.to(DEV), y, r.to(DEV), split, wc=wc,
        fused=(nw.to(DEV), 0.0))
    torch.cuda.synchronize()
    assert torch.all(wc == 1)
    P = oracle.rms_norm_matvec(exact64(x), exact64(nw), exact64(W), 0.0)
    assert np.array_equal(exact64(y.cpu()),
                          oracle.residual_add(P, exact64(r)))


def test_decode_layer_with_folded_residual():
    """rms_norm -> matvec with the residual folded in (two launches, and
    one fused launch) against the oracle's layer: one bf16 rounding of
    (matvec + input); graph replays bitwise equal to the eager call."""
    d = 5120
    note("layer folded residual", d)
    h = synth.to_bf16(synth.normal((1, d), 50))
    nw = (1.0 + synth.normal((d,), 51, std=0.1)).to(torch.bfloat16)
    W = synth.to_bf16(synth.normal((d, d), 52, std=0.02))
    hd, nwd, Wd = h.to(DEV), nw.to(DEV), W.to(DEV)
    norm = torch.empty((1, d), dtype=torch.bfloat16, device=DEV)
    out2 = torch.empty((1, d), dtype=torch.bfloat16, device=DEV)
    out1 = torch.empty((1, d), dtype=torch.bfloat16, device=DEV)
    tg.tile_rms_norm(hd, nwd, norm, 1e-6)
    tg.tile_gemm(norm, Wd, out2, b_trans=True, residual=hd)
    tg.tile_rms_norm_matvec(hd, nwd, Wd, out1, 1e-6, residual=hd)
    torch.cuda.synchronize()
    n64 = exact64(norm.cpu())
    R2 = oracle.residual_add(oracle.gemm(n64, exact64(W), b_nk=True),
                             exact64(h))
    assert rel_err(out2.cpu(), R2) <= 4e-3
    R1 = oracle.residual_add(
        oracle.rms_norm_matvec(exact64(h), exact64(nw), exact64(W), 1e-6),
        exact64(h))
    assert rel_err(out1.cpu(), R1) <= 4e-3
    eager = out1.clone()
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    ws = torch.empty(tg.tile_rms_norm_matvec_workspace_size(hd, Wd, out1) +
                     256, dtype=torch.uint8, device=DEV)
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            tg.tile_rms_norm_matvec(hd, nwd, Wd, out1, 1e-6, residual=hd,
                                    workspace=ws, checked=False, stream=s)
    for rep in range(3):
        out1.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out1, eager), rep


def test_residual_errors():
    M, N, K = 2, 256, 512
    x = synth.to_bf16(synth.normal((M, K), 53)).to(DEV)
    W = synth.to_bf16(synth.normal((N, K), 54)).to(DEV)
    y = torch.empty((M, N), device=DEV)
    with pytest.raises(tg.TileGemmError) as e:     # the output itself
        tg.tile_gemm(x, W, y, b_trans=True, residual=y)
    assert e.value.status == tg.TG_E_ALIAS
    with pytest.raises(tg.TileGemmError) as e:     # wrong shape
        tg.tile_gemm(x, W, y, b_trans=True,
                     residual=torch.zeros((M, N + 1), device=DEV))
    assert e.value.status == tg.TG_E_SHAPE
    with pytest.raises(tg.TileGemmError) as e:     # not a float type
        tg.tile_gemm(x, W, y, b_trans=True,
                     residual=torch.zeros((M, N), dtype=torch.int32,
                                          device=DEV))
    assert e.value.status in (tg.TG_E_DTYPE, tg.TG_E_ARG)
    A = synth.to_bf16(synth.normal((64, K), 55)).to(DEV)   # tiled kernel
    C = torch.empty((64, N), device=DEV)
    with pytest.raises(tg.TileGemmError) as e:
        tg.tile_gemm(A, W, C, b_trans=True,
                     residual=torch.zeros((64, N), device=DEV))
    assert e.value.status == tg.TG_E_UNSUPPORTED


def test_noalloc_residual_equals_tile_gemm():
    M, N, K = 1, 5120, 5120
    x = synth.to_bf16(synth.normal((M, K), 56)).to(DEV)
    W = synth.to_bf16(synth.normal((N, K), 57, std=0.02)).to(DEV)
    r = synth.to_bf16(synth.normal((M, N), 58)).to(DEV)
    y0 = torch.empty((M, N), dtype=torch.bfloat16, device=DEV)
    y1 = torch.empty_like(y0)
    tg.tile_gemm(x, W, y0, b_trans=True, residual=r)
    tg.tile_gemm_noalloc(x, W, y1, b_trans=True, residual=r)
    torch.cuda.synchronize()
    assert torch.equal(y0, y1)
