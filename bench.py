#!/usr/bin/env python3
"""Benchmark of the tile-partitioned GEMM hot path on one MI355X.

Headline: BF16 GEMM M = N = K = 8192 (entries N(0,1) rounded to bf16, binary32
accumulation and output, C split into 256 x 256 sub-tensors, one persistent
launch of tile programs; A row-major, B column-major, i.e. B held as its
N x K transpose).  One step = one tile_gemm launch over the resident
inputs.  Prints ONE JSON line with TFLOP/s, the roofline fraction of the
dominant kernel, the error against the oracle on sampled rows, the oracle's
own CPU rate on those rows, and secondary measurements (FP8, FP32, split
precision, decode-shaped GB/s, grouped launch).
"""
import argparse
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

METRIC = ("GEMM TFLOP/s & %MFMA peak (bf16/fp8 vs fp32) at stated err; "
          "M=1 GB/s")
PEAK_TFLOPS = {"bf16": 2516.6, "fp8": 5033.2, "f32": 157.3}
PEAK_HBM_GBS = 8000.0


KERNEL_SOURCES = ["paper_2606_15991_amd/csrc/gemm_tiled.hip",
                  "paper_2606_15991_amd/csrc/tg_device.hpp",
                  "paper_2606_15991_amd/csrc/tg_internal.hpp"]
TRAFFIC_PROFILE = "profiles/gemm_tiled_bf16_8192_traffic.md"


def kernel_source_sha():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_from_profile():
    """HBM bytes per launch of the headline kernel from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE summary, when it was taken on the
    current kernel sources; None otherwise."""
    path = os.path.join(ROOT, TRAFFIC_PROFILE)
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                fields[k.strip().strip("`").strip("-").strip()] = v.strip()
    if fields.get("kernel_source_sha256") != kernel_source_sha():
        return None
    try:
        return int(float(fields["traffic_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def timed(fn, steps, warmup):
    """Average ms per call of fn over `steps` calls on the current stream,
    bracketed by device synchronisation, after `warmup` untimed calls."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(steps):
        fn()
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def exact64(t):
    import oracle
    t = t.detach().cpu().contiguous()
    if t.dtype == torch.bfloat16:
        return oracle.decode_bf16(t.view(torch.int16).numpy().view(np.uint16))
    if t.dtype == torch.float8_e4m3fn:
        return oracle.decode_e4m3fn(t.view(torch.uint8).numpy())
    return t.numpy().astype(np.float64)


def oracle_rows(A, B, rows, b_nk=False, sa=None, sb=None, target_s=10.0):
    """Oracle product of a seeded sample of rows, timed.  Starts with a few
    rows and grows the sample toward about target_s seconds of CPU work."""
    import oracle
    a, b = exact64(A), exact64(B)
    sa64 = None if sa is None else exact64(sa)
    sb64 = None if sb is None else exact64(sb)
    done, secs, R = [], 0.0, []
    n = 2
    i = 0
    while i < len(rows):
        take = rows[i:i + n]
        t0 = time.perf_counter()
        R.append(oracle.gemm(a[take], b, b_nk=b_nk,
                             sa=None if sa64 is None else sa64[take],
                             sb=sb64))
        secs += time.perf_counter() - t0
        done.extend(take)
        i += n
        if secs >= target_s:
            break
        n = min(n * 2, len(rows) - i) if i < len(rows) else n
    return np.asarray(done), np.concatenate(R, axis=0), secs


def clock_sample():
    """Current shader (SCLK) and memory (MCLK) clocks in MHz from the
    driver's sysfs DPM tables (the level marked '*'), or None where the
    files are not readable."""
    import glob
    out = {}
    for name, key in (("pp_dpm_sclk", "sclk_mhz"), ("pp_dpm_mclk",
                                                    "mclk_mhz")):
        for f in sorted(glob.glob(f"/sys/class/drm/card*/device/{name}")):
            try:
                with open(f) as fh:
                    for line in fh:
                        if "*" in line:
                            mhz = "".join(ch for ch in line.split(":")[-1]
                                          if ch.isdigit())
                            if mhz:
                                out[key] = int(mhz)
            except OSError:
                continue
            if key in out:
                break
    return out or None


def bench_bf16_main(args, tg):
    M = N = K = 8192
    log("bf16 8192^3: generating inputs")
    A = synth.to_bf16(synth.normal((M, K), 2))
    Bt = synth.to_bf16(synth.normal((N, K), 202))   # B^T, row-major
    Ad, Bd = A.cuda(), Bt.cuda()
    C = torch.empty((M, N), device="cuda")
    # launch configuration: the library's default, or the one given with
    # --config (profiling of other schedules on the same workload)
    cfg = json.loads(args.config) if args.config else None

    def step():
        tg.tile_gemm(Ad, Bd, C, 256, 256, b_trans=True, config=cfg)

    # clock settling: back-to-back launches for --settle-ms of wall time
    # before the warm-up (after start-up the power manager first lowers the
    # clock; launch durations settle after about 50 launches)
    settle = 0
    t0 = time.perf_counter()
    while (time.perf_counter() - t0) * 1e3 < args.settle_ms:
        for _ in range(10):
            step()
        settle += 10
        torch.cuda.synchronize()
    log(f"bf16 8192^3: {settle} settling launches, timing")
    ms = timed(step, args.steps, args.warmup)
    flops = 2.0 * M * N * K
    tflops = flops / (ms * 1e-3) / 1e12
    # the safe / unsafe twins of Sec. 5.1: the checked launch (ownership
    # rules run on the host) against the unchecked one, interleaved
    # A B B A ... in the same warm state; device time of each launch from
    # events, host time of each call from the wall clock
    s = torch.cuda.current_stream()
    dev_ms = {True: [], False: []}
    host_us = {True: [], False: []}
    pairs = 20
    for i in range(pairs):
        for checked in ((True, False) if i % 2 == 0 else (False, True)):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(s)
            h0 = time.perf_counter()
            tg.tile_gemm(Ad, Bd, C, 256, 256, b_trans=True, checked=checked,
                         config=cfg)
            host_us[checked].append((time.perf_counter() - h0) * 1e6)
            e1.record(s)
            e1.synchronize()
            dev_ms[checked].append(e0.elapsed_time(e1))
    twins = {"pairs": pairs, "order": "ABBA interleaved",
             "checked_ms_median": float(np.median(dev_ms[True])),
             "unchecked_ms_median": float(np.median(dev_ms[False])),
             "checked_over_unchecked": float(np.median(dev_ms[True]) /
                                             np.median(dev_ms[False])),
             "checked_host_us_median": float(np.median(host_us[True])),
             "unchecked_host_us_median": float(np.median(host_us[False]))}
    # per-launch durations (events between back-to-back launches) for the
    # spread of the same workload, with the clocks sampled while they run
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(31)]
    ev[0].record(s)
    for i in range(30):
        step()
        ev[i + 1].record(s)
    clocks = [clock_sample() for _ in range(5)]
    torch.cuda.synchronize()
    per = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(30)])
    spread = {"launches": 30, "p25_ms": float(np.percentile(per, 25)),
              "median_ms": float(np.median(per)),
              "p75_ms": float(np.percentile(per, 75))}
    clocks = [c for c in clocks if c]
    clock = {"source": "sysfs pp_dpm_sclk / pp_dpm_mclk, sampled during "
                       "the 30 launches", "samples": clocks} if clocks else \
        {"source": "unavailable (no readable DPM table)", "samples": []}
    step()
    torch.cuda.synchronize()
    Cc = C.cpu().numpy()
    res = {"M": M, "N": N, "K": K, "ms": ms, "tflops": tflops,
           "twins": twins, "spread": spread, "clock": clock,
           "settle_launches": settle, "A": A, "Bt": Bt, "C": Cc}
    return res


def bench_bf16_kn(args, tg):
    """Same product with B row-major (stored K x N)."""
    n = 8192
    A = synth.to_bf16(synth.normal((n, n), 2)).cuda()
    B = synth.to_bf16(synth.normal((n, n), 202)).cuda()
    C = torch.empty((n, n), device="cuda")
    ms = timed(lambda: tg.tile_gemm(A, B, C, 256, 256), 50, 100)
    return {"ms": ms, "tflops": 2.0 * n ** 3 / (ms * 1e-3) / 1e12}


def copy_calibration(nbytes=1 << 30, reps=5):
    """A plain device copy of known size, for scaling the FETCH_SIZE and
    WRITE_SIZE counters of a profiled run to bytes."""
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "reps": reps}), flush=True)


def library_reference(tg, n=8192, reps=10):
    """The vendor library's bf16 GEMM (torch.matmul, i.e. hipBLASLt) on the
    headline shape and layout, timed beside the library's default launch
    of the same product: context for the roofline fraction, and a command
    to profile both kernels in one run."""
    g = torch.Generator(device="cpu").manual_seed(2)
    A = torch.randn((n, n), generator=g).to(torch.bfloat16).cuda()
    B = torch.randn((n, n), generator=g).to(torch.bfloat16).cuda()
    C = torch.empty((n, n), device="cuda")
    Bt = B.t()
    out = {}
    for name, fn in (("library", lambda: torch.matmul(A, Bt)),
                     ("tile_gemm", lambda: tg.tile_gemm(
                         A, B, C, 256, 256, b_trans=True, checked=False))):
        ms = timed(fn, reps, reps)
        out[name] = {"ms": ms, "tflops": 2.0 * n ** 3 / (ms * 1e-3) / 1e12}
    print(json.dumps(out), flush=True)


def cpu_baseline_and_err(res, target_s):
    import oracle
    rng = np.random.default_rng(2)
    rows = rng.permutation(res["M"])[:4096]
    done, R, secs = oracle_rows(res["A"], res["Bt"], rows, b_nk=True,
                                target_s=target_s)
    got = res["C"][done].astype(np.float64)
    err = oracle.rel_fro(got, R)
    flops = 2.0 * len(done) * res["N"] * res["K"]
    cpu = {"value": flops / secs / 1e12, "unit": "TFLOP/s",
           "cores": oracle.num_threads(), "kind": "oracle",
           "sample": f"{len(done)} seeded rows of the 8192^3 bf16 product "
                     f"({secs:.1f} s)"}
    return err, cpu, len(done)


def bench_fp8(args, tg, n=8192):
    log(f"fp8 {n}^3")
    qa, sa = synth.quant_e4m3_rows(synth.normal((n, n), 5))
    qb, sb = synth.quant_e4m3_rows(synth.normal((n, n), 505))
    Ad, Bd, sad, sbd = qa.cuda(), qb.cuda(), sa.cuda(), sb.cuda()
    C = torch.empty((n, n), device="cuda")
    ms = timed(lambda: tg.tile_gemm(Ad, Bd, C, 256, 256, b_trans=True,
                                    scale_a=sad, scale_b=sbd), 50, 100)
    return {"M": n, "N": n, "K": n, "ms": ms,
            "tflops": 2.0 * n ** 3 / (ms * 1e-3) / 1e12,
            "frac_fp8_peak": 2.0 * n ** 3 / (ms * 1e-3) / 1e12 /
            PEAK_TFLOPS["fp8"]}


def bench_f32_and_split(args, tg, n=8192, sample_rows=8):
    """Plain f32 and BF16x3 / BF16x6 at n^3 (f32 N(0,1) operands).  Keeps a
    seeded sample of output rows of each for the oracle's error check in
    the CPU leg."""
    log(f"f32 / split {n}^3")
    A32 = synth.normal((n, n), 2)
    B32 = synth.normal((n, n), 202)
    A, B = A32.cuda(), B32.cuda()
    C = torch.empty((n, n), device="cuda")
    rows = np.sort(np.random.default_rng(5).permutation(n)[:sample_rows])
    rows_t = torch.from_numpy(rows).cuda()
    out, kept = {}, {}
    ms = timed(lambda: tg.tile_gemm(A, B, C, 128, 128), 3, 1)
    out["f32_ms"] = ms
    out["f32_tflops"] = 2.0 * n ** 3 / (ms * 1e-3) / 1e12
    kept["f32"] = C[rows_t].cpu().numpy()
    for prec in ("bf16x3", "bf16x6"):
        ws = torch.empty(tg.tile_gemm_workspace_size(A, B, C,
                                                     precision=prec),
                         dtype=torch.uint8, device="cuda")
        ms = timed(lambda: tg.tile_gemm(A, B, C, 256, 256, precision=prec,
                                        workspace=ws), 3, 1)
        out[prec + "_ms"] = ms
        out[prec + "_eff_tflops"] = 2.0 * n ** 3 / (ms * 1e-3) / 1e12
        kept[prec] = C[rows_t].cpu().numpy()
        del ws
    out["_sample"] = {"A": A32, "B": B32, "rows": rows, "C": kept}
    return out


def cpu_leg_split_errors(sample):
    """Relative Frobenius error of the f32, BF16x3 and BF16x6 results on
    their sampled rows against the oracle's binary64 product of the f32
    inputs (part of the CPU leg: the oracle runs here only)."""
    import oracle
    rows = sample["rows"]
    a = sample["A"].numpy().astype(np.float64)[rows]
    b = sample["B"].numpy().astype(np.float64)
    R = oracle.gemm(a, b)
    errs = {k + "_err_rel_fro": oracle.rel_fro(v.astype(np.float64), R)
            for k, v in sample["C"].items()}
    errs["split_err_rows"] = int(len(rows))
    return errs


def graph_ms(calls, reps=20, warmup=3):
    """Average ms per call of a list of launches, captured once in a HIP
    graph and replayed (the launches are microseconds long, shorter than the
    host's own per-call cost, so eager timing would measure the host)."""
    s = torch.cuda.Stream()
    for c in calls:          # eager pass: first-use set-up outside capture
        c(None)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            for c in calls:
                c(s)
    torch.cuda.synchronize()
    return timed(g.replay, reps, warmup) / len(calls)


def release_cached():
    """Return the device memory the earlier sections cached, so that a
    streaming section's buffers are laid out as in a process of their own
    (the decode sections run 1.5 us slower per 52 MB call without it)."""
    import gc
    gc.collect()
    torch.cuda.empty_cache()


def bench_decode(args, tg):
    """Decode shapes: cold = the launches of one graph stream >= 1 GB of
    distinct weight copies (more than the 256 MB Infinity Cache holds), warm
    = the same weights every launch."""
    out = []
    release_cached()
    # one workspace for the K split over programs, reused by every launch
    ws = torch.empty(64 << 20, dtype=torch.uint8, device="cuda")
    for wdt in ("bf16", "fp8"):
        for (N, K) in synth.DECODE_SHAPES:
            for M in (1, 8):
                x = synth.to_bf16(synth.normal((M, K), 3)).cuda()
                w = synth.normal((N, K), 303, std=0.02)
                if wdt == "bf16":
                    W, s = synth.to_bf16(w), None
                else:
                    W, s = synth.quant_e4m3_rows(w)
                W = W.cuda()
                s = None if s is None else s.cuda()
                wbytes = W.numel() * W.element_size()
                copies = max(2, int(np.ceil(1.0e9 / wbytes)))
                Ws = [W] + [W.clone() for _ in range(copies - 1)]
                y = torch.empty((M, N), dtype=torch.bfloat16, device="cuda")

                def call(Wi):
                    return lambda st: tg.tile_gemm(x, Wi, y, b_trans=True,
                                                   scale_b=s, checked=False,
                                                   workspace=ws, stream=st)
                ms = graph_ms([call(Wi) for Wi in Ws], reps=10)
                ms_warm = graph_ms([call(W)] * 20, reps=10)
                ms_eager = timed(lambda: tg.tile_gemm(x, W, y, b_trans=True,
                                                      scale_b=s,
                                                      workspace=ws), 40, 5)
                cfg = tg.tile_gemm_plan(x, W, y, b_trans=True,
                                        want_map=False,
                                        workspace_bytes=ws.numel())[0]
                nbytes = wbytes + (N * 4 if s is not None else 0) + \
                    2 * M * K + 2 * M * N
                out.append({"w": wdt, "M": M, "N": N, "K": K,
                            "us": ms * 1e3, "gbs": nbytes / (ms * 1e-3) / 1e9,
                            "gbs_warm": nbytes / (ms_warm * 1e-3) / 1e9,
                            "us_eager_call": ms_eager * 1e3,
                            "config": {k: cfg[k] for k in
                                       ("bn", "ksplit", "splitk")}})
                log("decode", out[-1])
                del Ws, W
    return out


def bench_grouped(args, tg):
    shapes = synth.grouped_shapes(4, 64)
    log("grouped: 64 problems")
    As = [synth.to_bf16(synth.normal((m, k), 1000 + i)).cuda()
          for i, (m, n, k) in enumerate(shapes)]
    Bs = [synth.to_bf16(synth.normal((k, n), 2000 + i)).cuda()
          for i, (m, n, k) in enumerate(shapes)]
    Cs = [torch.empty((m, n), device="cuda") for m, n, k in shapes]
    # tile configuration from the autotuner (every tiled configuration of
    # the launch timed; the workspace is left prepared with the fastest)
    launch, best, _ = tg.tile_autotune_grouped(As, Bs, Cs, reps=3)
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    tg.tile_gemm_grouped(launch)
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            tg.tile_gemm_grouped(launch, stream=s)
    torch.cuda.synchronize()
    ms = timed(g.replay, 20, 3)
    flops = sum(2.0 * m * n * k for m, n, k in shapes)
    bound = sum(max(2.0 * m * n * k / (PEAK_TFLOPS["bf16"] * 1e12),
                    (2 * (m * k + k * n) + 4 * m * n) / (PEAK_HBM_GBS * 1e9))
                for m, n, k in shapes)
    return {"problems": 64, "ms": ms, "tflops": flops / (ms * 1e-3) / 1e12,
            "frac_of_roofline_sum": bound / (ms * 1e-3), "config": best}


def bench_add(args, tg, n=16384):
    """Element-wise z = x + y over 2^28 bf16 elements (n x n): two reads and
    one write of 2 bytes per element against the 8 TB/s HBM peak.  Each
    launch is timed on its own with HIP events (median, p25, p75 over 30);
    1.6 GB per launch is far more than the 256 MB Infinity Cache holds."""
    x = synth.to_bf16(synth.normal((n, n), 61)).cuda()
    y = synth.to_bf16(synth.normal((n, n), 62)).cuda()
    z = torch.empty_like(x)
    for _ in range(10):
        tg.tile_add(x, y, z, checked=False)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    ms = []
    for _ in range(30):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(s)
        tg.tile_add(x, y, z, checked=False)
        e1.record(s)
        e1.synchronize()
        ms.append(e0.elapsed_time(e1))
    p25, med, p75 = np.percentile(ms, [25, 50, 75])
    nbytes = 3 * 2 * n * n
    gbs = nbytes / (med * 1e-3) / 1e9
    out = {"elements": n * n, "dtype": "bf16", "bytes_per_launch": nbytes,
           "ms_median": med, "ms_p25": p25, "ms_p75": p75,
           "gbs_median": gbs, "gbs_p25_p75": [nbytes / (p75 * 1e-3) / 1e9,
                                             nbytes / (p25 * 1e-3) / 1e9],
           "frac_of_hbm_peak": gbs / PEAK_HBM_GBS,
           "partition": list(tg.tile_add.last_partition)}
    log("elementwise add", out)
    return out


def bench_decode_layer(args, tg, d=5120, layers=16):
    """The decode layer rms_norm -> matvec (d x d bf16 weights stored N x K)
    -> residual add at M = 1, over `layers` layers with weights of their own
    (16 x 52 MB, more than the Infinity Cache holds), launched eagerly and
    as one captured graph, and with the normalisation fused into the
    matvec (two kernels per layer); time per layer and weight-stream GB/s."""
    release_cached()
    xs = synth.to_bf16(synth.normal((1, d), 71)).cuda()
    nw = (1.0 + synth.normal((d,), 72, std=0.1)).to(torch.bfloat16).cuda()
    Ws = [synth.to_bf16(synth.normal((d, d), 100 + i, std=0.02)).cuda()
          for i in range(layers)]
    bufs = [torch.empty((1, d), dtype=torch.bfloat16, device="cuda")
            for _ in range(3 * layers)]
    # workspaces of the K split over programs (the unfused matvec and the
    # fused one), allocated once outside the timed graphs
    ws = torch.empty(tg.tile_gemm_workspace_size(bufs[0], Ws[0], bufs[1],
                                                 b_trans=True) + 256,
                     dtype=torch.uint8, device="cuda")
    wsf = torch.empty(tg.tile_rms_norm_matvec_workspace_size(xs, Ws[0],
                                                             bufs[1]) + 256,
                      dtype=torch.uint8, device="cuda")

    def run(stream=None):
        h = xs
        for i in range(layers):
            norm, q, res = bufs[3 * i:3 * i + 3]
            tg.tile_rms_norm(h, nw, norm, 1e-6, checked=False, stream=stream)
            tg.tile_gemm(norm, Ws[i], q, b_trans=True, checked=False,
                         workspace=ws, stream=stream)
            tg.tile_add(h, q, res, checked=False, stream=stream)
            h = res
    def run_fused(stream=None):
        h = xs
        for i in range(layers):
            norm, q, res = bufs[3 * i:3 * i + 3]
            tg.tile_rms_norm_matvec(h, nw, Ws[i], q, 1e-6, checked=False,
                                    workspace=wsf, stream=stream)
            tg.tile_add(h, q, res, checked=False, stream=stream)
            h = res
    # the residual add folded into the product's store (the program that
    # owns an element of the layer output adds the layer input to it)
    def run_res(stream=None):
        h = xs
        for i in range(layers):
            norm, q, res = bufs[3 * i:3 * i + 3]
            tg.tile_rms_norm(h, nw, norm, 1e-6, checked=False, stream=stream)
            tg.tile_gemm(norm, Ws[i], res, b_trans=True, checked=False,
                         workspace=ws, residual=h, stream=stream)
            h = res

    def run_fused_res(stream=None):
        h = xs
        for i in range(layers):
            norm, q, res = bufs[3 * i:3 * i + 3]
            tg.tile_rms_norm_matvec(h, nw, Ws[i], res, 1e-6, checked=False,
                                    workspace=wsf, residual=h, stream=stream)
            h = res
    ms_eager = timed(run, 20, 5)
    ms_graph = graph_ms([lambda st: run(stream=st)], reps=20)
    ms_fused = graph_ms([lambda st: run_fused(stream=st)], reps=20)
    ms_res = graph_ms([lambda st: run_res(stream=st)], reps=20)
    ms_fused_res = graph_ms([lambda st: run_fused_res(stream=st)], reps=20)
    wbytes = 2.0 * d * d
    out = {"d": d, "layers": layers,
           "us_per_layer_eager": ms_eager * 1e3 / layers,
           "us_per_layer_graph": ms_graph * 1e3 / layers,
           "weight_gbs_graph": wbytes * layers / (ms_graph * 1e-3) / 1e9,
           "us_per_layer_graph_fused_norm": ms_fused * 1e3 / layers,
           "us_per_layer_graph_residual_folded": ms_res * 1e3 / layers,
           "us_per_layer_graph_fused_norm_residual_folded":
               ms_fused_res * 1e3 / layers}
    log("decode layer", out)
    return out


def bench_exec_modes(args, tg, n_elems=2048, chain=(1, 10, 100, 1000),
                     reps=20):
    """Host launch cost per operation of a chain of N element-wise products
    y_i = y_(i-1) * g over one 2048-element bf16 tile, in three modes:
    sync (launch, then wait for the stream, per operation), chained (N
    launches, one wait) and graph (the N launches captured once, one replay
    and one wait).  Launches go through the C ABI with descriptors built
    once (checked launches: the ownership rules run on the host per call).
    Per-operation microseconds: minimum and 75th percentile over `reps`."""
    import ctypes
    import time
    g = synth.to_bf16(1.0 + synth.normal((1, n_elems), 81, std=1e-3)).cuda()
    bufs = [synth.to_bf16(synth.normal((1, n_elems), 82)).cuda(),
            torch.empty((1, n_elems), dtype=torch.bfloat16, device="cuda")]
    din = [tg.make_in(b) for b in bufs]
    dout = [tg.make_out(b) for b in bufs]
    dg = tg.make_in(g)
    opts = tg.make_opts()

    def launch(i, stream):
        st = tg.lib.tile_mul(din[i & 1], dg, dout[(i + 1) & 1], opts, stream)
        if st:
            raise tg.TileGemmError(st, tg.last_error())

    out = []
    cur = torch.cuda.current_stream()
    for n in chain:
        res = {"N": n}
        for mode in ("sync", "chained", "graph"):
            if mode == "graph":
                gr = torch.cuda.CUDAGraph()
                s = torch.cuda.Stream()
                with torch.cuda.stream(s):
                    for i in range(n):
                        launch(i, s.cuda_stream)
                torch.cuda.synchronize()
                with torch.cuda.stream(s):
                    with torch.cuda.graph(gr, stream=s):
                        for i in range(n):
                            launch(i, s.cuda_stream)
                torch.cuda.synchronize()
            times = []
            for r in range(reps + 2):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                if mode == "sync":
                    for i in range(n):
                        launch(i, cur.cuda_stream)
                        cur.synchronize()
                elif mode == "chained":
                    for i in range(n):
                        launch(i, cur.cuda_stream)
                    cur.synchronize()
                else:
                    gr.replay()
                    torch.cuda.current_stream().synchronize()
                    torch.cuda.synchronize()
                t = (time.perf_counter() - t0) * 1e6 / n
                if r >= 2:
                    times.append(t)
            res[mode] = {"us_per_op_min": float(np.min(times)),
                         "us_per_op_p75": float(np.percentile(times, 75))}
        out.append(res)
        log("exec modes", res)
    return {"python_ctypes": out, "cpp_driver": exec_modes_cpp(reps)}


def exec_modes_cpp(reps=20):
    """The same chains launched from compiled code through the C ABI (the
    library's own per-call cost without Python's): the tg_exec_modes driver
    built beside the library, run as a child process."""
    import subprocess
    exe = os.path.join(ROOT, "paper_2606_15991_amd", "tg_exec_modes")
    if not os.path.exists(exe):
        return {"error": "tg_exec_modes is not built"}
    r = subprocess.run([exe, str(reps)], capture_output=True, text=True,
                       timeout=300)
    if r.returncode != 0:
        return {"error": r.stderr.strip()[-500:]}
    res = json.loads(r.stdout.strip().splitlines()[-1])
    log("exec modes (C++ driver)", res)
    return res


def bench_bimodal(args, tg, n=2000, stream_counts=(1, 2, 4, 8, 16, 32),
                  reps=5):
    """A queue of n GEMMs, 80 % 512^3 and 20 % 2048^3 (bf16, weights
    stored N x K, binary32 output), run (a) as single launches fanned out
    round-robin over S streams, launched eagerly from Python and captured
    in one graph, for each S in stream_counts, and (b) as one grouped
    persistent launch.  Throughput in GEMMs per millisecond (median of
    reps wall-clock runs, each bracketed by device synchronisation)."""
    sizes = synth.bimodal_sizes(96, n)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(97)
    As = [torch.randn((s, s), device="cuda", generator=gen).bfloat16()
          for s in sizes]
    Bs = [torch.randn((s, s), device="cuda", generator=gen).bfloat16()
          for s in sizes]
    Cs = [torch.empty((s, s), device="cuda") for s in sizes]
    flops = sum(2.0 * s ** 3 for s in sizes)

    def wall(fn):
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) * 1e3)
        return float(np.median(ts))

    fan = []
    for S in stream_counts:
        streams = [torch.cuda.Stream() for _ in range(S)]

        def fan_out():
            for i in range(n):
                tg.tile_gemm(As[i], Bs[i], Cs[i], b_trans=True,
                             checked=False, stream=streams[i % S])
        fan_out()
        ms_eager = wall(fan_out)
        # the same fan-out captured in one graph (fork from and join into
        # the capture stream through events)
        cap = torch.cuda.Stream()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.stream(cap):
            with torch.cuda.graph(g, stream=cap):
                ev = torch.cuda.Event()
                ev.record(cap)
                for st in streams:
                    st.wait_event(ev)
                fan_out()
                for st in streams:
                    e = torch.cuda.Event()
                    e.record(st)
                    cap.wait_event(e)
        torch.cuda.synchronize()
        g.replay()
        ms_graph = wall(g.replay)
        fan.append({"streams": S, "eager_ms": ms_eager,
                    "eager_gemm_per_ms": n / ms_eager, "graph_ms": ms_graph,
                    "graph_gemm_per_ms": n / ms_graph})
        log("bimodal fan-out", fan[-1])
        del g
    launch = tg.tile_gemm_grouped_prepare(As, Bs, Cs, b_trans=True)
    tg.tile_gemm_grouped(launch)
    ms_grouped = wall(lambda: tg.tile_gemm_grouped(launch))
    out = {"gemms": n, "big_fraction": sizes.count(2048) / n,
           "fan_out": fan,
           "grouped": {"ms": ms_grouped, "gemm_per_ms": n / ms_grouped,
                       "tflops": flops / (ms_grouped * 1e-3) / 1e12}}
    log("bimodal grouped", out["grouped"])
    del As, Bs, Cs, launch
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--quick", action="store_true",
                    help="headline workload only")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--settle-ms", type=float, default=1000.0,
                    help="wall time of back-to-back headline launches "
                         "before the warm-up (clock settling)")
    ap.add_argument("--config", default=None,
                    help="with --quick: JSON launch configuration of the "
                         "headline product (default: the library's choice)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (counter scaling)")
    ap.add_argument("--decode", action="store_true",
                    help="only the decode-shaped products (one JSON line)")
    ap.add_argument("--add", action="store_true",
                    help="only the element-wise add (one JSON line)")
    ap.add_argument("--exec-modes", action="store_true",
                    help="only the launch-mode sweep (sync / chained / "
                         "graph, N = 1..1000)")
    ap.add_argument("--bimodal", action="store_true",
                    help="only the bimodal GEMM queue (fan-out vs grouped)")
    ap.add_argument("--layer", action="store_true",
                    help="only the decode layer rms_norm -> matvec -> add")
    ap.add_argument("--library-reference", action="store_true",
                    help="only time the vendor bf16 GEMM beside the "
                         "headline launch")
    ap.add_argument("--picker", action="store_true",
                    help="also run the learned-picker evaluation "
                         "(2000 training / 200 held-out shapes)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not "
              "supported: the benchmark runs on a single GPU", file=sys.stderr)
        sys.exit(2)
    if args.config and not args.quick:
        print("--config applies to the headline launch of a --quick run",
              file=sys.stderr)
        sys.exit(2)
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    import paper_2606_15991_amd as tg
    if args.library_reference:
        library_reference(tg)
        return
    if args.decode:
        print(json.dumps({"decode": bench_decode(args, tg)}), flush=True)
        return
    if args.add:
        print(json.dumps({"elementwise_add": bench_add(args, tg)}),
              flush=True)
        return
    if args.layer:
        print(json.dumps({"decode_layer": bench_decode_layer(args, tg)}),
              flush=True)
        return
    if args.bimodal:
        print(json.dumps({"bimodal_queue": bench_bimodal(args, tg)}),
              flush=True)
        return
    if args.exec_modes:
        print(json.dumps({"exec_modes": bench_exec_modes(args, tg)}),
              flush=True)
        return

    res = bench_bf16_main(args, tg)
    extra = {"checked_vs_unchecked": res["twins"],
             "launch_spread": res["spread"],
             "settle_launches": res["settle_launches"]}
    if not args.quick:
        extra["fp8_8192"] = bench_fp8(args, tg)
        extra.update(bench_f32_and_split(args, tg))
        extra["decode"] = bench_decode(args, tg)
        extra["grouped"] = bench_grouped(args, tg)
        extra["bf16_8192_b_row_major"] = bench_bf16_kn(args, tg)
        extra["elementwise_add"] = bench_add(args, tg)
        extra["decode_layer"] = bench_decode_layer(args, tg)
        extra["exec_modes"] = bench_exec_modes(args, tg)
        extra["bimodal_queue"] = bench_bimodal(args, tg)
    if args.picker:
        from paper_2606_15991_amd import picker
        import io
        import contextlib
        buf = io.StringIO()
        with contextlib.redirect_stdout(buf):
            picker.main([])
        extra["picker"] = json.loads(buf.getvalue().strip().splitlines()[-1])
    err, cpu, nrows = cpu_baseline_and_err(res, args.cpu_seconds)
    if "_sample" in extra:
        extra.update(cpu_leg_split_errors(extra.pop("_sample")))
    tflops = res["tflops"]
    line = {
        "metric": METRIC,
        "value": round(tflops, 2),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(res["ms"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": "bf16 GEMM M=N=K=8192, N(0,1) inputs, "
                               "f32 accumulate+output, C partition 256x256, "
                               "A row-major, B column-major (stored N x K)",
                   "M": 8192, "N": 8192, "K": 8192,
                   "partition": [256, 256], "parallelism": "none",
                   **({"launch_config": json.loads(args.config)}
                      if args.config else {})},
        "roofline": {"bound": "mfma", "achieved": round(tflops, 2),
                     "peak": PEAK_TFLOPS["bf16"], "unit": "TFLOP/s",
                     "frac": round(tflops / PEAK_TFLOPS["bf16"], 4),
                     # the committed counters describe the default launch
                     "traffic": None if args.config
                     else traffic_from_profile()},
        "clock": res["clock"],
        "err_rel_fro": err,
        "err_rows": nrows,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
