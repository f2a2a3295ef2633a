"""Learned tile-configuration picker.

Workflow (each step runs in the library):
  1. collect: for every training shape, tile_autotune times every candidate
     configuration (HIP events) and tile_picker_features describes each
     (shape, configuration) pair;
  2. train: the cost model (MLP, `depth` hidden ReLU layers of `hidden` units)
     regresses log(ms) with mean squared error, full-batch Adam, using the
     library's GPU kernels tile_mlp_loss_grad and tile_mlp_adam;
  3. install: tile_picker_set hands the trained parameters to tile_gemm, which
     then picks argmin predicted time over tile_gemm_candidates for shapes it
     has not tuned;
  4. evaluate: on held-out shapes, the score is time of the exhaustive best /
     time of the picked configuration, both measured by the autotuner.  Two
     pickers without the cost model are scored the same way: one fixed
     configuration for every shape (the first 256 x 256 tiled candidate, the
     large-problem default) and the library's shape heuristic.

Run as a module for the full workload:
  python -m paper_2606_15991_amd.picker --train 2000 --test 200
"""
import argparse
import json
import math
import os
import sys
import time

import torch

from . import (TG_PICKER_FEATURES, make_in, make_out, tile_autotune,
               tile_gemm_plan, tile_mlp_adam, tile_mlp_loss_grad,
               tile_mlp_param_count, tile_picker_features, tile_picker_mode,
               tile_picker_set, tile_tune_cache_clear)

HIDDEN, DEPTH = 64, 3


def _ceil16(x):
    return (x + 15) // 16 * 16


class ShapePool:
    """Device buffers sized for the largest shape; every problem is a view
    with leading dimensions rounded up to 16 elements."""

    def __init__(self, max_dim=16384, device="cuda", seed=0):
        g = torch.Generator(device=device)
        g.manual_seed(seed)
        n = _ceil16(max_dim) * _ceil16(max_dim)
        self.a = (torch.randn(n, generator=g, device=device) * 0.5).to(
            torch.bfloat16)
        self.b = (torch.randn(n, generator=g, device=device) * 0.5).to(
            torch.bfloat16)
        self.c = torch.empty(n, dtype=torch.float32, device=device)

    def views(self, M, N, K, dtype):
        """A (M x K), B stored N x K, C (M x N) f32."""
        lda, ldb, ldc = _ceil16(K), _ceil16(K), _ceil16(N)
        if dtype == "fp8":
            a = self.a.view(torch.uint8).view(torch.float8_e4m3fn)
            b = self.b.view(torch.uint8).view(torch.float8_e4m3fn)
        else:
            a, b = self.a, self.b
        A = a.as_strided((M, K), (lda, 1))
        B = b.as_strided((N, K), (ldb, 1))
        C = self.c.as_strided((M, N), (ldc, 1))
        return A, B, C


def _key(cfg):
    return (cfg["kind"], cfg["bm"], cfg["bn"], cfg["bk"], cfg["wm"],
            cfg["wn"], cfg["ksplit"], cfg["stages"], cfg["sched"],
            cfg["splitk"])


def collect(shapes, pool, reps=3, log=None):
    """Autotune every shape; returns one record per shape."""
    recs = []
    t0 = time.time()
    for i, (M, N, K, dt) in enumerate(shapes):
        A, B, C = pool.views(M, N, K, dt)
        best, rows = tile_autotune(A, B, C, b_trans=True, reps=reps)
        cands = []
        for cfg, ms, st in rows:
            if st != 0 or not (ms > 0):
                continue
            f = tile_picker_features(A, B, C, cfg, b_trans=True)
            cands.append({"cfg": cfg, "ms": ms, "feat": f})
        recs.append({"shape": [M, N, K, dt], "cands": cands,
                     "best_ms": min(c["ms"] for c in cands)})
        if log and (i + 1) % 100 == 0:
            log(f"collected {i + 1}/{len(shapes)} shapes "
                f"({time.time() - t0:.1f} s)")
    return recs


def dataset(recs):
    """Features and targets.  The target is log(ms) relative to the mean
    over the same shape's candidates: the picker only ranks the candidates
    of one shape, so the model spends its capacity on the differences between
    configurations rather than on the (large, easy) differences between
    shapes."""
    X, y = [], []
    for r in recs:
        logs = [math.log(c["ms"]) for c in r["cands"]]
        mu = sum(logs) / len(logs)
        for c, lg in zip(r["cands"], logs):
            X.append(c["feat"])
            y.append(lg - mu)
    return torch.tensor(X, dtype=torch.float32), torch.tensor(
        y, dtype=torch.float32)


def train(recs, steps=3000, lr=3e-3, seed=5, device="cuda", log=None):
    """Fit the cost model on the GPU.  Returns a model dict."""
    import synth
    X, y = dataset(recs)
    mean = X.mean(dim=0)
    std = X.std(dim=0)
    std = torch.where(std > 0, std, torch.ones_like(std))
    Xn = ((X - mean) / std).to(device).contiguous()
    yd = y.to(device).contiguous()
    n_in = TG_PICKER_FEATURES
    params = synth.mlp_init(n_in, HIDDEN, DEPTH, seed).to(device)
    assert params.numel() == tile_mlp_param_count(n_in, HIDDEN, DEPTH)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    grads = torch.empty_like(params)
    loss = torch.empty(1, dtype=torch.float32, device=device)
    hist = []
    ws = None
    for t in range(1, steps + 1):
        tile_mlp_loss_grad(params, Xn, yd, n_in, HIDDEN, DEPTH, grads=grads,
                           loss=loss, ws=ws)
        tile_mlp_adam(params, grads, m, v, t, lr=lr)
        if t == 1 or t % 250 == 0 or t == steps:
            hist.append((t, float(loss.item())))
            if log:
                log(f"step {t}: loss {hist[-1][1]:.4f}")
    return {"params": params.cpu(), "mean": mean, "std": std,
            "loss_history": hist, "samples": int(X.shape[0])}


def install(model):
    tile_picker_set(model["params"].tolist(), TG_PICKER_FEATURES, HIDDEN,
                    DEPTH, model["mean"].tolist(), model["std"].tolist())


def _forward_host(model, feats):
    """Model prediction through the installed library model."""
    from . import tile_picker_predict
    return [tile_picker_predict(f) for f in feats]


def _fixed(cands):
    """The one configuration used for every shape when nothing is tuned or
    learned: the first 256 x 256 tiled candidate."""
    for c in cands:
        cfg = c["cfg"]
        if cfg["kind"] == 1 and cfg["bm"] == 256 and cfg["bn"] == 256:
            return c
    return None


def evaluate(recs, pool):
    """Score of the learned picker, the fixed configuration and the shape
    heuristic against the exhaustive best, on the autotuner's own
    timings."""
    out = []
    old = tile_picker_mode(0)
    try:
        for r in recs:
            M, N, K, dt = r["shape"]
            A, B, C = pool.views(M, N, K, dt)
            by_key = {_key(c["cfg"]): c["ms"] for c in r["cands"]}
            preds = _forward_host(None, [c["feat"] for c in r["cands"]])
            pick = r["cands"][min(range(len(preds)), key=preds.__getitem__)]
            tile_picker_mode(0)          # fixed heuristic only
            dcfg, _, _, _ = tile_gemm_plan(A, B, C, b_trans=True,
                                           want_map=False)
            d_ms = by_key.get(_key(dcfg))
            fx = _fixed(r["cands"])
            out.append({"shape": r["shape"], "best_ms": r["best_ms"],
                        "mlp_ms": pick["ms"], "default_ms": d_ms,
                        "fixed_ms": fx["ms"] if fx else None,
                        "mlp_cfg": pick["cfg"], "default_cfg": dcfg,
                        "cands": [{"cfg": c["cfg"], "ms": c["ms"],
                                   "pred": pr}
                                  for c, pr in zip(r["cands"], preds)]})
    finally:
        tile_picker_mode(old)
    return out


def summarize(ev):
    def geo(vals):
        vals = [v for v in vals if v and v > 0]
        return math.exp(sum(math.log(v) for v in vals) / len(vals))
    mlp = [e["best_ms"] / e["mlp_ms"] for e in ev]
    dft = [e["best_ms"] / e["default_ms"] for e in ev if e["default_ms"]]
    fix = [e["best_ms"] / e["fixed_ms"] for e in ev if e["fixed_ms"]]
    return {"shapes": len(ev),
            "mlp_geomean_frac_of_best": geo(mlp),
            "mlp_worst_frac": min(mlp),
            "mlp_exact_best": sum(1 for x in mlp if x >= 0.999) / len(mlp),
            "fixed_geomean_frac_of_best": geo(fix) if fix else None,
            "fixed_worst_frac": min(fix) if fix else None,
            "default_geomean_frac_of_best": geo(dft),
            "default_worst_frac": min(dft) if dft else None}


def main(argv=None):
    import synth
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=2000)
    ap.add_argument("--test", type=int, default=200)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", default=None)
    args = ap.parse_args(argv)

    def log(msg):
        print("[picker]", msg, file=sys.stderr, flush=True)

    tile_tune_cache_clear()
    pool = ShapePool()
    train_shapes = synth.picker_shapes(5, args.train)
    test_shapes = synth.picker_shapes(6, args.test) + [
        (16384, 16384, 16384, "fp8")]
    log(f"autotuning {len(train_shapes)} training shapes")
    t0 = time.time()
    tr = collect(train_shapes, pool, args.reps, log)
    t_collect = time.time() - t0
    log("training the cost model on the GPU")
    t0 = time.time()
    model = train(tr, steps=args.steps, log=log)
    t_train = time.time() - t0
    install(model)
    log(f"autotuning {len(test_shapes)} held-out shapes")
    te = collect(test_shapes, pool, args.reps, log)
    ev = evaluate(te, pool)
    s = summarize(ev)
    big = [e for e in ev if e["shape"] == [16384, 16384, 16384, "fp8"]][0]
    s["fp8_16384"] = {"best_ms": big["best_ms"], "mlp_ms": big["mlp_ms"],
                      "default_ms": big["default_ms"],
                      "mlp_cfg": big["mlp_cfg"],
                      "best_tflops": 2 * 16384 ** 3 / big["best_ms"] / 1e9}
    s.update({"train_shapes": len(train_shapes), "train_samples":
              model["samples"], "loss_history": model["loss_history"],
              "collect_s": t_collect, "train_s": t_train})
    line = json.dumps(s)
    print(line, flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump({"summary": s, "eval": ev}, f, indent=1)


if __name__ == "__main__":
    sys.path.insert(0, os.path.dirname(os.path.dirname(
        os.path.abspath(__file__))))
    main()
