"""tile_gemm_noalloc, the allocation-free variant of tile_gemm, against
tile_gemm itself and the oracle (needs an MI355X).  Two calls in a row, the
second smaller, share the library's per-device scratch; each must equal
tile_gemm's result with a workspace of its own bit for bit (same
configuration, deterministic kernels) and meet the binary32 bar against the
oracle."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import exact64, note, reference, rel_err

pytestmark = pytest.mark.gpu

tg = pytest.importorskip("paper_2606_15991_amd")
DEV = "cuda:0"


def _both(A, B, M, N, **kw):
    C_ref = torch.full((M, N), float("nan"), device=DEV)
    C_na = torch.full((M, N), float("nan"), device=DEV)
    wc = torch.zeros((M, N), dtype=torch.int32, device=DEV)
    tg.tile_gemm(A, B, C_ref, **kw)
    tg.tile_gemm_noalloc(A, B, C_na, write_count=wc, **kw)
    torch.cuda.synchronize()
    return C_ref, C_na, wc


@pytest.mark.parametrize("config", [True, False])
def test_noalloc_decode_split_two_calls(config):
    """Decode products split over programs along K: the partial tiles live
    in the scratch.  config=True names the split; False takes the default
    choice (which splits (8, 1040, 25600) eight ways)."""
    for M, N, K, sk, seed in ((8, 1040, 25600, 4, 1), (2, 1040, 1000, 3, 2)):
        note("noalloc decode", M, N, K, sk, config)
        x = synth.to_bf16(synth.normal((M, K), 40 + seed)).to(DEV)
        W = synth.to_bf16(synth.normal((N, K), 50 + seed, std=0.02)).to(DEV)
        cfg = {"kind": "skinny", "bn": 16, "ksplit": 4, "splitk": sk} \
            if config else None
        plan = tg.tile_gemm_plan(x, W, torch.empty((M, N), device=DEV),
                                 b_trans=True, config=cfg,
                                 workspace_bytes=tg.TG_NOALLOC_SCRATCH_BYTES,
                                 want_map=False)[0]
        if config or (M, N, K) == (8, 1040, 25600):
            assert plan["splitk"] > 1, plan
        C_ref, C_na, wc = _both(x, W, M, N, b_trans=True, config=cfg)
        assert torch.equal(C_na, C_ref), (M, N, K)
        assert torch.all(wc == 1)
        assert rel_err(C_na.cpu(), reference(x.cpu(), W.cpu(), True)) <= 1e-5


def test_noalloc_split_precision_two_calls():
    """BF16x6 planes in the scratch (small products whose planes fit)."""
    for M, N, K, seed in ((192, 200, 256, 3), (96, 80, 64, 4)):
        note("noalloc bf16x6", M, N, K)
        A = synth.normal((M, K), 60 + seed).to(DEV)
        B = synth.normal((K, N), 70 + seed).to(DEV)
        C_ref, C_na, wc = _both(A, B, M, N, bm=64, bn=64, precision="bf16x6")
        assert torch.equal(C_na, C_ref)
        assert torch.all(wc == 1)
        assert rel_err(C_na.cpu(), reference(A.cpu(), B.cpu())) <= 2e-6


def test_noalloc_refuses_what_it_cannot_hold():
    """Requests beyond the scratch and a workspace argument are refused on
    the host, before anything is enqueued (the output keeps its values)."""
    note("noalloc refusals")
    A = torch.zeros((1024, 1024), device=DEV)
    C = torch.full((1024, 1024), 7.0, device=DEV)
    o = tg.make_opts("bf16x6")
    st = tg.lib.tile_gemm_noalloc(tg.make_in(A), tg.make_in(A),
                                  tg.make_out(C, 256, 256), o, None)
    assert st == tg.TG_E_WORKSPACE
    assert "scratch" in tg.last_error()
    ws = torch.empty(1 << 20, dtype=torch.uint8, device=DEV)
    o = tg.make_opts(workspace=ws)
    st = tg.lib.tile_gemm_noalloc(tg.make_in(A), tg.make_in(A),
                                  tg.make_out(C, 256, 256), o, None)
    assert st == tg.TG_E_ARG
    torch.cuda.synchronize()
    assert torch.all(C == 7.0)
