"""Autotuner, tuning cache, cost-model training kernels and the learned
picker (needs an MI355X).

The MLP kernels are compared with the binary64 oracle (oracle.mlp) on the
same seeded parameters and data: forward outputs and every gradient tensor
within 1e-4 relative, Adam within 1e-6.  The picker is trained on the
autotuner's own timings and scored against exhaustive search on held-out
shapes, beside the fixed default heuristic ("the method without it").
"""
import math
import os

import numpy as np
import pytest
import torch

import synth
from gpu_util import note
from oracle import mlp as omlp

pytestmark = pytest.mark.gpu

tg = pytest.importorskip("paper_2606_15991_amd")
DEV = "cuda:0"


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("n_in,hidden,depth,batch",
                         [(16, 64, 3, 1000), (5, 8, 1, 33), (16, 64, 2, 257)])
def test_mlp_kernels_match_oracle(n_in, hidden, depth, batch):
    note("mlp", n_in, hidden, depth, batch)
    p = synth.mlp_init(n_in, hidden, depth, 11)
    p = p + synth.normal(p.shape, 12, std=0.05)        # non-zero biases
    X = synth.normal((batch, n_in), 13)
    y = synth.normal((batch,), 14)
    pd, Xd, yd = p.to(DEV), X.to(DEV), y.to(DEV)
    out = tg.tile_mlp_forward(pd, Xd, n_in, hidden, depth)
    loss, g = tg.tile_mlp_loss_grad(pd, Xd, yd, n_in, hidden, depth)
    torch.cuda.synchronize()
    p64, X64, y64 = p.double().numpy(), X.double().numpy(), y.double().numpy()
    o_ref, _ = omlp.forward(p64, X64, n_in, hidden, depth)
    assert _rel(out.cpu(), o_ref) <= 1e-5
    assert abs(loss.item() - omlp.loss(p64, X64, y64, n_in, hidden, depth)) \
        <= 1e-5 * omlp.loss(p64, X64, y64, n_in, hidden, depth)
    g_ref = omlp.grad(p64, X64, y64, n_in, hidden, depth)
    gc = g.cpu().double().numpy()
    off = 0
    for o, i in omlp.shapes(n_in, hidden, depth):
        for n in (o * i, o):
            assert _rel(gc[off:off + n], g_ref[off:off + n]) <= 1e-4, off
            off += n
    # fixed-order reductions: bitwise repeatable
    _, g2 = tg.tile_mlp_loss_grad(pd, Xd, yd, n_in, hidden, depth)
    torch.cuda.synchronize()
    assert torch.equal(g2, g)


def test_adam_kernel_matches_oracle():
    note("adam")
    n = 5000
    p = synth.normal((n,), 21)
    g = synth.normal((n,), 22)
    m = synth.normal((n,), 23) * 0.1
    v = synth.normal((n,), 24).abs() * 0.01
    pd, gd, md, vd = p.to(DEV), g.to(DEV), m.to(DEV), v.to(DEV)
    tg.tile_mlp_adam(pd, gd, md, vd, 7, lr=1e-2)
    torch.cuda.synchronize()
    pr, mr, vr = omlp.adam(p.double().numpy(), g.double().numpy(),
                           m.double().numpy(), v.double().numpy(), 7, lr=1e-2)
    assert _rel(md.cpu(), mr) <= 1e-6 and _rel(vd.cpu(), vr) <= 1e-6
    assert np.max(np.abs(pd.cpu().double().numpy() - pr)) <= 1e-6


def test_autotune_times_every_candidate_and_fills_cache():
    note("autotune 512x384x320 bf16")
    tg.tile_tune_cache_clear()
    A = synth.to_bf16(synth.normal((512, 320), 31)).to(DEV)
    B = synth.to_bf16(synth.normal((384, 320), 32)).to(DEV)
    C = torch.empty((512, 384), device=DEV)
    cands = tg.tile_gemm_candidates(A, B, C, b_trans=True)
    assert len(cands) >= 4
    best, rows = tg.tile_autotune(A, B, C, b_trans=True, reps=2)
    assert len(rows) == len(cands)
    assert all(st == 0 and ms > 0 for _, ms, st in rows)
    fastest = min(rows, key=lambda r: r[1])[0]
    assert best == fastest
    assert tg.tile_tune_cache_size() == 1
    # tile_gemm with no configuration now runs the tuned one
    cfg, _, _, _ = tg.tile_gemm_plan(A, B, C, b_trans=True, want_map=False)
    assert cfg == best


def test_tune_cache_save_load_roundtrip(tmp_path):
    note("cache roundtrip")
    A = synth.to_bf16(synth.normal((256, 256), 33)).to(DEV)
    B = synth.to_bf16(synth.normal((256, 256), 34)).to(DEV)
    C = torch.empty((256, 256), device=DEV)
    tg.tile_tune_cache_clear()
    best, _ = tg.tile_autotune(A, B, C, b_trans=True, reps=1)
    path = tmp_path / "cache.txt"
    tg.tile_tune_cache_save(path)
    tg.tile_tune_cache_clear()
    assert tg.tile_tune_cache_size() == 0
    tg.tile_tune_cache_load(path)
    assert tg.tile_tune_cache_size() == 1
    cfg, _, _, _ = tg.tile_gemm_plan(A, B, C, b_trans=True, want_map=False)
    assert cfg == best


def test_learned_picker_beats_default_and_tracks_exhaustive():
    """Small version of the picker workload: 400 training shapes, 80
    held-out shapes (M, N, K log-uniform in [1, 4096], bf16 / e4m3).  The
    learned picker must stay close to the exhaustive best and beat the one
    fixed configuration it replaces; the shape heuristic is reported."""
    from paper_2606_15991_amd import picker
    note("picker train 400 / test 80")
    tg.tile_tune_cache_clear()
    pool = picker.ShapePool(max_dim=4096)
    tr = picker.collect(synth.picker_shapes(5, 400, hi=4096), pool, reps=5)
    model = picker.train(tr, steps=1500)
    hist = model["loss_history"]
    assert hist[-1][1] < 0.5 * hist[0][1]
    picker.install(model)
    # held-out timings averaged over 20 launches: the exhaustive best is a
    # minimum over 20-45 near-tied candidates on small shapes, so timing
    # noise alone would pull every ratio below 1
    te = picker.collect(synth.picker_shapes(6, 80, hi=4096), pool, reps=20)
    tg.tile_tune_cache_clear()
    ev = picker.evaluate(te, pool)
    s = picker.summarize(ev)
    note("picker summary", s)
    # within 5 % of the exhaustive search and a large gain over the one
    # fixed configuration it replaces.  Against the library's shape
    # heuristic the two sit within timing noise of each other on this
    # small set (reported, not asserted; the full 2000 / 200 run is in the
    # picker summary under profiles/)
    assert s["mlp_geomean_frac_of_best"] >= 0.95
    assert s["mlp_geomean_frac_of_best"] > \
        1.5 * s["fixed_geomean_frac_of_best"]
    # tile_gemm itself follows the installed model when nothing is cached
    old = tg.tile_picker_mode(2)
    try:
        for e in ev[:10]:
            M, N, K, dt = e["shape"]
            A, B, C = pool.views(M, N, K, dt)
            cfg, _, _, _ = tg.tile_gemm_plan(A, B, C, b_trans=True,
                                             want_map=False)
            assert picker._key(cfg) == picker._key(e["mlp_cfg"])
    finally:
        tg.tile_picker_mode(old)
        tg.tile_picker_set(None, 0, 0, 0, None, None)
