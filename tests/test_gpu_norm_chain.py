"""RMS normalisation and the decode layer of Sec. 3.2's graph-scope listing
(rms_norm -> matvec -> residual add) on the GPU, against the oracle.

Tolerances:
  * rms_norm, binary32 output: relative 1e-5 per element (binary32 sum of
    squares over <= 5120 elements in a fixed tree, then about six roundings:
    about 2.5e-6 at most);
  * rms_norm, bf16 output: relative 2^-8 + 1e-5 per element (one bf16
    rounding of the binary32 value: bf16 keeps 8 significant bits, so its
    unit roundoff is 2^-8);
  * the fused normalisation + product: relative Frobenius 1e-5 (binary32
    output) against the oracle's fused definition, which holds x * nw in
    bf16 as the kernel does, 4e-3 for bf16 output and against the plain
    chain; small-integer cases bit-exact;
  * the layer (bf16 buffers): relative Frobenius 4e-3 against the oracle's
    chain, which rounds each intermediate buffer to bf16 as the layer
    stores it (bf16 unit roundoff 2^-8).
The graph replays are compared bit for bit with the eager layer (every
kernel is deterministic)."""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import exact64, note, rel_err

pytestmark = pytest.mark.gpu

tg = pytest.importorskip("paper_2606_15991_amd")
DEV = "cuda:0"


def norm_inputs(rows, d, dt, seed):
    x = synth.normal((rows, d), seed, std=2.0).to(dt)
    w = (1.0 + synth.normal((d,), seed + 1, std=0.1)).to(dt)
    return x, w


def check_norm(y, x, w, eps, dt):
    want = oracle.rms_norm(exact64(x), exact64(w), eps)
    got = exact64(y)
    tol = 1e-5 if dt == torch.float32 else 2.0 ** -8 + 1e-5
    bad = np.abs(got - want) > tol * np.abs(want) + 1e-30
    assert not bad.any(), f"{bad.sum()} elements, first {np.argwhere(bad)[:3]}"


@pytest.mark.parametrize("rows,d", [(1, 5120), (3, 1000), (16, 4096), (7, 33),
                                    (1, 1), (2, 70000)])
@pytest.mark.parametrize("dt", [torch.bfloat16, torch.float32])
def test_rms_norm_matches_oracle(rows, d, dt):
    note("rms_norm", rows, d, dt)
    x, w = norm_inputs(rows, d, dt, 7)
    y = torch.full((rows, d), 5.0, dtype=dt, device=DEV)
    tg.tile_rms_norm(x.to(DEV), w.to(DEV), y, 1e-6)
    torch.cuda.synchronize()
    check_norm(y, x, w, 1e-6, dt)


def test_rms_norm_partition_and_write_count():
    note("rms_norm partition 3 rows")
    x, w = norm_inputs(10, 300, torch.bfloat16, 9)
    y = torch.empty((10, 300), dtype=torch.bfloat16, device=DEV)
    wc = torch.zeros((10, 300), dtype=torch.int32, device=DEV)
    tg.tile_rms_norm(x.to(DEV), w.to(DEV), y, 0.5, bm=3, write_count=wc)
    torch.cuda.synchronize()
    assert tg.tile_rms_norm.last_partition == (3, 300)
    assert int(wc.min()) == 1 and int(wc.max()) == 1
    check_norm(y, x, w, 0.5, torch.bfloat16)


def test_rms_norm_rejects_bad_arguments():
    note("rms_norm argument errors")
    x = torch.ones((4, 64), dtype=torch.bfloat16, device=DEV)
    w = torch.ones((64,), dtype=torch.bfloat16, device=DEV)
    y = torch.empty_like(x)
    with pytest.raises(tg.TileGemmError):
        tg.tile_rms_norm(x, w[:32], y)
    with pytest.raises(tg.TileGemmError):
        tg.tile_rms_norm(x, w, y, eps=-1.0)
    with pytest.raises(tg.TileGemmError):
        tg.tile_rms_norm(x, w, x)                      # y is an input
    with pytest.raises(tg.TileGemmError):
        tg.tile_rms_norm(x, w.float(), y)
    dy = tg.make_out(y, 1, 32)                         # not whole rows
    assert tg.lib.tile_rms_norm(tg.make_in(x), tg.make_in(w.view(1, -1)),
                                1e-6, dy, None, None) == tg.TG_E_ARG


@pytest.mark.parametrize("M,N,K", [(1, 5120, 5120), (8, 300, 1008),
                                   (16, 64, 528), (3, 4096, 16384)])
@pytest.mark.parametrize("wdt", ["bf16", "fp8"])
@pytest.mark.parametrize("out", [torch.float32, torch.bfloat16])
def test_fused_norm_matvec_matches_oracle(M, N, K, wdt, out):
    note("fused norm matvec", M, N, K, wdt, out)
    x = synth.to_bf16(synth.normal((M, K), 31, std=2.0))
    nw = (1.0 + synth.normal((K,), 32, std=0.1)).to(torch.bfloat16)
    w = synth.normal((N, K), 33, std=0.02)
    if wdt == "bf16":
        W, sw = synth.to_bf16(w), None
    else:
        W, sw = synth.quant_e4m3_rows(w)
    y = torch.full((M, N), float("nan"), dtype=out, device=DEV)
    wc = torch.zeros((M, N), dtype=torch.int32, device=DEV)
    tg.tile_rms_norm_matvec(x.to(DEV), nw.to(DEV), W.to(DEV), y, 1e-6,
                            scale_w=None if sw is None else sw.to(DEV),
                            write_count=wc)
    torch.cuda.synchronize()
    sw64 = None if sw is None else exact64(sw)
    # the fused definition: x * nw held in bf16, row scale on the sum
    R = oracle.rms_norm_matvec(exact64(x), exact64(nw), exact64(W), 1e-6,
                               sw64)
    err = rel_err(y, R)
    note("fused err %.3g" % err)
    assert err <= (1e-5 if out == torch.float32 else 4e-3), err
    # and the plain chain without the intermediate rounding, within the
    # bf16 rounding of the weighted activations
    xn = oracle.rms_norm(exact64(x), exact64(nw), 1e-6)
    Rc = oracle.gemm(xn, exact64(W), b_nk=True, sb=sw64)
    assert rel_err(y, Rc) < 4e-3
    assert int(wc.min()) == 1 and int(wc.max()) == 1


@pytest.mark.parametrize("split", [True, False])
@pytest.mark.parametrize("M,N,K", [(1, 5120, 5120), (4, 300, 1008),
                                   (16, 64, 4096)])
@pytest.mark.parametrize("wdt", ["bf16", "fp8"])
@pytest.mark.parametrize("out", [torch.float32, torch.bfloat16])
def test_fused_norm_matvec_small_integers_bit_exact(M, N, K, wdt, out,
                                                    split):
    """Activation rows of +-2^j (j = m mod 4; eps 0, so the row scale is
    2^-j exactly), power-of-two normalisation weights and small-integer
    weights: every x * nw is a bf16 value, every partial sum an integer
    below 2^24, so the result is exact (bf16 output: one rounding of it)."""
    note("fused norm matvec exact", M, N, K, wdt, out)
    g = torch.Generator().manual_seed(34)
    sign = torch.randint(0, 2, (M, K), generator=g).float() * 2 - 1
    j = (torch.arange(M) % 4).float()[:, None]
    x = (sign * 2.0 ** j).to(torch.bfloat16)
    nw = (2.0 ** torch.randint(-1, 3, (K,), generator=g).float()).to(
        torch.bfloat16)
    Wi = synth.small_int((N, K), 35)
    W = Wi.to(torch.bfloat16) if wdt == "bf16" else Wi.to(
        torch.float8_e4m3fn)
    sw = None if wdt == "bf16" else 2.0 ** torch.randint(
        -2, 3, (N,), generator=g).float()
    y = torch.full((M, N), float("nan"), dtype=out, device=DEV)
    wc = torch.zeros((M, N), dtype=torch.int32, device=DEV)
    # split=True: the library's default given a workspace (allocated by
    # the binding), which splits K over programs for N = 300 and 64 and
    # runs one round of 20-column programs for N = 5120; split=False: no
    # workspace, one program per sub-tensor
    tg.tile_rms_norm_matvec(x.to(DEV), nw.to(DEV), W.to(DEV), y, 0.0,
                            scale_w=None if sw is None else sw.to(DEV),
                            write_count=wc,
                            workspace=None if split else False)
    torch.cuda.synchronize()
    R = oracle.rms_norm_matvec(exact64(x), exact64(nw), exact64(W), 0.0,
                               None if sw is None else exact64(sw))
    want = R if out == torch.float32 else oracle.decode_bf16(
        oracle.round_bf16(R))
    assert np.array_equal(exact64(y), want)
    assert int(wc.min()) == 1 and int(wc.max()) == 1


def test_fused_norm_matvec_rejects_bad_arguments():
    note("fused norm matvec argument errors")
    x = torch.ones((1, 64), dtype=torch.bfloat16, device=DEV)
    nw = torch.ones((64,), dtype=torch.bfloat16, device=DEV)
    W = torch.ones((32, 64), dtype=torch.bfloat16, device=DEV)
    y = torch.empty((1, 32), device=DEV)
    with pytest.raises(tg.TileGemmError):
        tg.tile_rms_norm_matvec(x, nw[:32], W, y)
    with pytest.raises(tg.TileGemmError):
        tg.tile_rms_norm_matvec(x, nw, W, y, eps=-1.0)
    with pytest.raises(tg.TileGemmError):
        tg.tile_rms_norm_matvec(torch.ones((17, 64), dtype=torch.bfloat16,
                                           device=DEV), nw, W,
                                torch.empty((17, 32), device=DEV))


class Layer:
    """One decode layer: norm = rms_norm(input), q = norm . Wq^T,
    residual = input + q, all bf16 buffers allocated up front."""

    def __init__(self, d, seed, fused=False):
        self.fused = fused
        self.x = synth.to_bf16(synth.normal((1, d), seed)).to(DEV)
        self.nw = (1.0 + synth.normal((d,), seed + 1, std=0.1)).to(
            torch.bfloat16).to(DEV)
        self.W = synth.to_bf16(synth.normal((d, d), seed + 2, std=0.02)).to(
            DEV)
        self.norm = torch.empty((1, d), dtype=torch.bfloat16, device=DEV)
        self.q = torch.empty_like(self.norm)
        self.res = torch.empty_like(self.norm)
        self.eps = 1e-6

    def run(self, stream=None):
        if self.fused:
            tg.tile_rms_norm_matvec(self.x, self.nw, self.W, self.q,
                                    self.eps, stream=stream)
        else:
            tg.tile_rms_norm(self.x, self.nw, self.norm, self.eps,
                             stream=stream)
            tg.tile_gemm(self.norm, self.W, self.q, b_trans=True,
                         stream=stream)
        tg.tile_add(self.x, self.q, self.res, stream=stream)

    def oracle(self):
        """The chain in binary64 with each stored buffer rounded to bf16."""
        xb = self.x.cpu().view(torch.int16).numpy().view(np.uint16)
        n = oracle.round_bf16(oracle.rms_norm(oracle.decode_bf16(xb),
                                              exact64(self.nw), self.eps))
        q = oracle.round_bf16(oracle.gemm(oracle.decode_bf16(n),
                                          exact64(self.W), b_nk=True))
        return oracle.decode_bf16(oracle.add_bf16(xb, q))


@pytest.mark.parametrize("fused", [False, True])
@pytest.mark.parametrize("d", [5120, 1000])
def test_decode_layer_eager_and_graph_replays(d, fused):
    note("decode layer", d, "fused" if fused else "three kernels")
    L = Layer(d, 21, fused)
    L.run()
    torch.cuda.synchronize()
    eager = L.res.clone()
    assert rel_err(eager, L.oracle()) < 4e-3
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        L.run(stream=s)
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            L.run(stream=s)
    torch.cuda.synchronize()
    for rep in range(3):
        L.res.fill_(0.0)
        L.q.fill_(0.0)
        L.norm.fill_(0.0)
        (L.W[:64].float() * 3.0).sum()                # eager work between
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(L.res.view(torch.int16), eager.view(torch.int16)), \
            f"replay {rep} differs from the eager layer"
