"""Python binding of libtilegemm.so (the C ABI declared in include/tilegemm.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of the shared library.  torch supplies device memory and streams.
The functions carry the names of the C entry points:

  tile_gemm(A, B, C, ...)            C = A . B into a partitioned output
  tile_gemm_plan(A, B, C, ...)       configuration + program -> sub-tensor map
  tile_partition_check(ins, out, ...)  ownership rules (host only)
  tile_gemm_grouped_prepare / tile_gemm_grouped   one launch, many problems
  tile_error_norm(C, R, out)         binary64 error reductions on the GPU

Following the prepare/recover protocol of the paper (Sec. 3.3), tile_gemm
returns the very tensor objects it was given.  The library is required: if
libtilegemm.so is missing the import of this package fails.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtilegemm.so")

# tg_status
TG_OK, TG_E_ARG, TG_E_DTYPE, TG_E_SHAPE, TG_E_OVERLAP, TG_E_NOCOVER, \
    TG_E_ALIAS, TG_E_WORKSPACE, TG_E_UNSUPPORTED, TG_E_HIP = range(10)
# tg_dtype
TG_F32, TG_BF16, TG_FP8_E4M3 = 0, 1, 2
# tg_precision
TG_PREC_NATIVE, TG_PREC_BF16X3, TG_PREC_BF16X6 = 0, 1, 2
# tg_kind
TG_KIND_AUTO, TG_KIND_TILED, TG_KIND_SKINNY, TG_KIND_SIMPLE = 0, 1, 2, 3
# tg_sched
TG_SCHED_ANY, TG_SCHED_LOCKSTEP, TG_SCHED_PINGPONG, TG_SCHED_CROSS, \
    TG_SCHED_STAGED, TG_SCHED_BULK, TG_SCHED_CROSS_WARM = 0, 1, 2, 3, 4, 5, 6
TG_ERROR_NORM_DOUBLES = 514

PRECISIONS = {"native": TG_PREC_NATIVE, "bf16x3": TG_PREC_BF16X3,
              "bf16x6": TG_PREC_BF16X6}
KINDS = {"auto": TG_KIND_AUTO, "tiled": TG_KIND_TILED,
         "skinny": TG_KIND_SKINNY, "simple": TG_KIND_SIMPLE}


class tg_in(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("dtype", ctypes.c_int32),
                ("trans", ctypes.c_int32), ("rows", ctypes.c_int64),
                ("cols", ctypes.c_int64), ("ld", ctypes.c_int64)]


class tg_out(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("dtype", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("rows", ctypes.c_int64),
                ("cols", ctypes.c_int64), ("ld", ctypes.c_int64),
                ("bm", ctypes.c_int32), ("bn", ctypes.c_int32)]


class tg_config(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("bm", ctypes.c_int32),
                ("bn", ctypes.c_int32), ("bk", ctypes.c_int32),
                ("wm", ctypes.c_int32), ("wn", ctypes.c_int32),
                ("ksplit", ctypes.c_int32), ("stages", ctypes.c_int32),
                ("sched", ctypes.c_int32), ("splitk", ctypes.c_int32)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class tg_opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("checked", ctypes.c_int32),
                ("scale_a", ctypes.c_void_p), ("scale_b", ctypes.c_void_p),
                ("config", ctypes.POINTER(tg_config)),
                ("workspace", ctypes.c_void_p),
                ("workspace_bytes", ctypes.c_size_t),
                ("write_count", ctypes.c_void_p),
                ("residual", ctypes.POINTER(tg_in))]


class tg_grouped_plan(ctypes.Structure):
    _fields_ = [("workspace", ctypes.c_void_p), ("n", ctypes.c_int32),
                ("total_tiles", ctypes.c_int32), ("n_prog", ctypes.c_int32),
                ("variant", ctypes.c_int32), ("tag", ctypes.c_uint64)]


class tg_tune_result(ctypes.Structure):
    _fields_ = [("cfg", tg_config), ("ms", ctypes.c_float),
                ("status", ctypes.c_int32)]


TG_PICKER_FEATURES = 24
TG_MAX_SPLITK = 16
_MAX_CANDIDATES = 128


class TileGemmError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{status_str(status)}: {message}")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with "
            "`python -c 'import __graft_entry__ as g; g.build()'`")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    i32 = ctypes.c_int32
    lib.tile_partition_check.argtypes = [P(tg_in), i32, P(tg_out), i32,
                                         ctypes.c_void_p, ctypes.c_void_p]
    lib.tile_gemm.argtypes = [P(tg_in), P(tg_in), P(tg_out), P(tg_opts),
                              ctypes.c_void_p]
    lib.tile_gemm_workspace_size.argtypes = [P(tg_in), P(tg_in), P(tg_out),
                                             P(tg_opts)]
    lib.tile_add.argtypes = [P(tg_in), P(tg_in), P(tg_out), P(tg_opts),
                             ctypes.c_void_p]
    lib.tile_mul.argtypes = [P(tg_in), P(tg_in), P(tg_out), P(tg_opts),
                             ctypes.c_void_p]
    lib.tile_rms_norm_matvec.argtypes = [P(tg_in), P(tg_in), ctypes.c_float,
                                         P(tg_in), P(tg_out), P(tg_opts),
                                         ctypes.c_void_p]
    lib.tile_rms_norm_matvec_workspace_size.argtypes = [P(tg_in), P(tg_in),
                                                        P(tg_out)]
    lib.tile_rms_norm_matvec_workspace_size.restype = ctypes.c_size_t
    lib.tile_rms_norm.argtypes = [P(tg_in), P(tg_in), ctypes.c_float,
                                  P(tg_out), P(tg_opts), ctypes.c_void_p]
    lib.tile_gemm_workspace_size.restype = ctypes.c_size_t
    lib.tile_gemm_noalloc.argtypes = [P(tg_in), P(tg_in), P(tg_out),
                                      P(tg_opts), ctypes.c_void_p]
    lib.tile_gemm_plan.argtypes = [P(tg_in), P(tg_in), P(tg_out), P(tg_opts),
                                   P(tg_config), P(i32), ctypes.c_void_p,
                                   ctypes.c_void_p]
    lib.tile_gemm_grouped_workspace_size.argtypes = [i32]
    lib.tile_gemm_grouped_workspace_size.restype = ctypes.c_size_t
    lib.tile_gemm_grouped_prepare.argtypes = [i32, P(tg_in), P(tg_in),
                                              P(tg_out), P(tg_opts),
                                              ctypes.c_void_p, ctypes.c_size_t,
                                              P(tg_grouped_plan),
                                              ctypes.c_void_p]
    lib.tile_gemm_grouped.argtypes = [P(tg_grouped_plan), ctypes.c_void_p]
    lib.tile_error_norm.argtypes = [ctypes.c_void_p, i32, ctypes.c_void_p,
                                    ctypes.c_int64, ctypes.c_void_p,
                                    ctypes.c_void_p]
    lib.tg_status_str.argtypes = [i32]
    lib.tg_status_str.restype = ctypes.c_char_p
    lib.tg_last_error.argtypes = []
    lib.tg_last_error.restype = ctypes.c_char_p
    lib.tg_device_cus.argtypes = []
    lib.tg_device_cus.restype = i32
    fp = P(ctypes.c_float)
    vp = ctypes.c_void_p
    lib.tile_gemm_candidates.argtypes = [P(tg_in), P(tg_in), P(tg_out),
                                         P(tg_opts), P(tg_config), i32]
    lib.tile_gemm_candidates.restype = i32
    lib.tile_autotune.argtypes = [P(tg_in), P(tg_in), P(tg_out), P(tg_opts),
                                  i32, P(tg_tune_result), i32, P(i32),
                                  P(tg_config), vp]
    lib.tile_autotune_grouped.argtypes = [i32, P(tg_in), P(tg_in), P(tg_out),
                                          P(tg_opts), vp, ctypes.c_size_t,
                                          i32, P(tg_tune_result), i32, P(i32),
                                          P(tg_config), P(tg_grouped_plan),
                                          vp]
    lib.tile_autotune_grouped.restype = i32
    lib.tile_tune_cache_clear.argtypes = []
    lib.tile_tune_cache_size.argtypes = []
    lib.tile_tune_cache_size.restype = i32
    lib.tile_tune_cache_save.argtypes = [ctypes.c_char_p]
    lib.tile_tune_cache_load.argtypes = [ctypes.c_char_p]
    lib.tile_picker_features.argtypes = [P(tg_in), P(tg_in), P(tg_out),
                                         P(tg_config), fp]
    lib.tile_picker_set.argtypes = [fp, i32, i32, i32, fp, fp]
    lib.tile_picker_predict.argtypes = [fp, fp]
    lib.tile_picker_mode.argtypes = [i32]
    lib.tile_picker_mode.restype = i32
    lib.tile_mlp_param_count.argtypes = [i32, i32, i32]
    lib.tile_mlp_param_count.restype = ctypes.c_size_t
    lib.tile_mlp_workspace_bytes.argtypes = [i32, i32, i32, i32]
    lib.tile_mlp_workspace_bytes.restype = ctypes.c_size_t
    lib.tile_mlp_forward.argtypes = [vp, i32, i32, i32, vp, i32, vp, vp,
                                     ctypes.c_size_t, vp]
    lib.tile_mlp_loss_grad.argtypes = [vp, i32, i32, i32, vp, vp, i32, vp,
                                       vp, vp, ctypes.c_size_t, vp]
    lib.tile_mlp_adam.argtypes = [vp, vp, vp, vp, ctypes.c_int64,
                                  ctypes.c_double, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_double, i32, vp]
    for f in ("tile_autotune", "tile_tune_cache_clear", "tile_tune_cache_save",
              "tile_tune_cache_load", "tile_picker_features",
              "tile_picker_set", "tile_picker_predict", "tile_mlp_forward",
              "tile_mlp_loss_grad", "tile_mlp_adam"):
        getattr(lib, f).restype = i32
    for f in ("tile_partition_check", "tile_gemm", "tile_gemm_noalloc",
              "tile_gemm_plan",
              "tile_gemm_grouped_prepare", "tile_gemm_grouped",
              "tile_add", "tile_mul", "tile_rms_norm", "tile_rms_norm_matvec",
              "tile_error_norm"):
        getattr(lib, f).restype = i32
    return lib


lib = _load()


def status_str(st) -> str:
    return lib.tg_status_str(int(st)).decode()


def last_error() -> str:
    return lib.tg_last_error().decode()


def _raise(st):
    if st != TG_OK:
        raise TileGemmError(st, last_error())


_DT = {torch.float32: TG_F32, torch.bfloat16: TG_BF16,
       torch.float8_e4m3fn: TG_FP8_E4M3}


def dtype_code(t: torch.dtype) -> int:
    try:
        return _DT[t]
    except KeyError:
        raise TileGemmError(TG_E_DTYPE, f"unsupported dtype {t}") from None


def _ld(t: torch.Tensor) -> int:
    if t.dim() != 2:
        raise TileGemmError(TG_E_SHAPE, "operands are 2-D matrices")
    if t.shape[1] > 1 and t.stride(1) != 1:
        raise TileGemmError(TG_E_SHAPE, "rows must be contiguous")
    if t.shape[0] > 1 or t.stride(0) >= t.shape[1]:
        return int(t.stride(0))
    return int(max(t.shape[1], 1))


def make_in(t: torch.Tensor, trans: bool = False) -> tg_in:
    """Immutable-input descriptor of a 2-D row-major tensor (stored shape)."""
    return tg_in(t.data_ptr(), dtype_code(t.dtype), int(trans),
                 int(t.shape[0]), int(t.shape[1]), _ld(t))


def make_out(t: torch.Tensor, bm: int = 0, bn: int = 0) -> tg_out:
    """Mutable-output descriptor with its partition bm x bn."""
    return tg_out(t.data_ptr(), dtype_code(t.dtype), 0, int(t.shape[0]),
                  int(t.shape[1]), _ld(t), int(bm), int(bn))


def make_config(cfg) -> tg_config:
    if cfg is None:
        return None
    if isinstance(cfg, tg_config):
        return cfg
    c = tg_config()
    for k, v in cfg.items():
        if k == "kind" and isinstance(v, str):
            v = KINDS[v]
        setattr(c, k, int(v))
    return c


def _stream(stream):
    if stream is None:
        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
        return None
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


def _ptr(t):
    return None if t is None else t.data_ptr()


def make_opts(precision="native", scale_a=None, scale_b=None, config=None,
              workspace=None, write_count=None, checked=True, residual=None):
    o = tg_opts()
    o.precision = PRECISIONS[precision] if isinstance(precision, str) \
        else int(precision)
    o.checked = int(bool(checked))
    o.scale_a = _ptr(scale_a)
    o.scale_b = _ptr(scale_b)
    c = make_config(config)
    o._cfg = c  # keep alive
    o.config = ctypes.pointer(c) if c is not None else None
    if workspace is not None:
        o.workspace = workspace.data_ptr()
        o.workspace_bytes = workspace.numel() * workspace.element_size()
    o.write_count = _ptr(write_count)
    if residual is not None:
        r = make_in(residual)
        o._res = r  # keep alive
        o.residual = ctypes.pointer(r)
    return o


def tile_gemm(A, B, C, bm=0, bn=0, *, b_trans=False, precision="native",
              scale_a=None, scale_b=None, config=None, workspace=None,
              write_count=None, checked=True, residual=None, stream=None):
    """C = diag(scale_a) A B diag(scale_b) (+ residual, decode products only)
    into C's bm x bn partition.

    B is K x N, or the stored N x K matrix when b_trans.  BF16x3/x6 and
    decode products split along K over several programs need a workspace
    (allocated here from torch when not given).  Returns (A, B, C) -- the
    same tensor objects."""
    da, db = make_in(A), make_in(B, b_trans)
    dc = make_out(C, bm, bn)
    o = make_opts(precision, scale_a, scale_b, config, workspace, write_count,
                  checked, residual)
    if workspace is None:
        need = lib.tile_gemm_workspace_size(da, db, dc, o)
        if need:
            workspace = torch.empty(need, dtype=torch.uint8, device=C.device)
            o.workspace = workspace.data_ptr()
            o.workspace_bytes = need
    _raise(lib.tile_gemm(da, db, dc, o, _stream(stream)))
    tile_gemm.last_partition = (dc.bm, dc.bn)
    return A, B, C


TG_NOALLOC_SCRATCH_BYTES = 8 << 20


def tile_gemm_noalloc(A, B, C, bm=0, bn=0, *, b_trans=False,
                      precision="native", scale_a=None, scale_b=None,
                      config=None, write_count=None, checked=True,
                      residual=None, stream=None):
    """tile_gemm without any device allocation: where tile_gemm takes a
    workspace the library's own per-device scratch is used (calls that
    overlap on one device race on it).  Returns (A, B, C)."""
    da, db = make_in(A), make_in(B, b_trans)
    dc = make_out(C, bm, bn)
    o = make_opts(precision, scale_a, scale_b, config, None, write_count,
                  checked, residual)
    _raise(lib.tile_gemm_noalloc(da, db, dc, o, _stream(stream)))
    tile_gemm_noalloc.last_partition = (dc.bm, dc.bn)
    return A, B, C


def tile_add(x, y, z, bm=0, bn=0, *, checked=True, write_count=None,
             stream=None):
    """z = x + y element by element into z's bm x bn partition (bf16 or
    fp32, one shape and dtype for all three).  Returns z."""
    dz = make_out(z, bm, bn)
    o = make_opts(write_count=write_count, checked=checked)
    _raise(lib.tile_add(make_in(x), make_in(y), dz, o, _stream(stream)))
    tile_add.last_partition = (dz.bm, dz.bn)
    return z


def tile_mul(x, y, z, bm=0, bn=0, *, checked=True, write_count=None,
             stream=None):
    """z = x * y element by element into z's bm x bn partition (bf16 or
    fp32).  Returns z."""
    dz = make_out(z, bm, bn)
    o = make_opts(write_count=write_count, checked=checked)
    _raise(lib.tile_mul(make_in(x), make_in(y), dz, o, _stream(stream)))
    tile_mul.last_partition = (dz.bm, dz.bn)
    return z


def tile_rms_norm(x, w, y, eps=1e-6, bm=0, *, checked=True,
                  write_count=None, stream=None):
    """y = x * w / sqrt(mean(x^2) + eps) per row (x, y rows x d; w of d
    elements, 1-D or 1 x d), into y's bm x d partition.  Returns y."""
    if w.dim() == 1:
        w = w.view(1, -1)
    dy = make_out(y, bm, y.shape[1] if bm else 0)
    o = make_opts(write_count=write_count, checked=checked)
    _raise(lib.tile_rms_norm(make_in(x), make_in(w), float(eps), dy, o,
                             _stream(stream)))
    tile_rms_norm.last_partition = (dy.bm, dy.bn)
    return y


def tile_rms_norm_matvec_workspace_size(x, W, y) -> int:
    return int(lib.tile_rms_norm_matvec_workspace_size(
        make_in(x), make_in(W, True), make_out(y)))


def tile_rms_norm_matvec(x, nw, W, y, eps=1e-6, *, scale_w=None,
                         checked=True, write_count=None, workspace=None,
                         residual=None, stream=None):
    """y = rms_norm(x; nw, eps) . W^T (+ residual) with the normalisation
    fused into the decode product (x: M x K bf16, M <= 16; nw: K bf16; W
    stored N x K).
    The workspace of a K split over programs is allocated here from torch
    when not given (workspace=False: no split).  Returns y."""
    if nw.dim() == 1:
        nw = nw.view(1, -1)
    dy = make_out(y)
    if workspace is None:
        need = tile_rms_norm_matvec_workspace_size(x, W, y)
        workspace = torch.empty(need, dtype=torch.uint8, device=y.device) \
            if need else None
    elif workspace is False:
        workspace = None
    o = make_opts(scale_b=scale_w, write_count=write_count, checked=checked,
                  workspace=workspace, residual=residual)
    _raise(lib.tile_rms_norm_matvec(make_in(x), make_in(nw), float(eps),
                                    make_in(W, True), dy, o, _stream(stream)))
    tile_rms_norm_matvec.last_partition = (dy.bm, dy.bn)
    return y


def tile_gemm_workspace_size(A, B, C, bm=0, bn=0, *, b_trans=False,
                             precision="native", config=None) -> int:
    return int(lib.tile_gemm_workspace_size(
        make_in(A), make_in(B, b_trans), make_out(C, bm, bn),
        make_opts(precision, config=config)))


def tile_gemm_plan(A, B, C, bm=0, bn=0, *, b_trans=False, precision="native",
                   config=None, want_map=True, workspace_bytes=None):
    """(config dict, n_prog, prog_offsets list, prog_tiles list) of the
    launch tile_gemm makes for a caller supplying workspace_bytes of
    workspace (default: as much as tile_gemm_workspace_size asks, which is
    what this binding's tile_gemm allocates)."""
    da, db = make_in(A), make_in(B, b_trans)
    dc = make_out(C, bm, bn)
    o = make_opts(precision, config=config)
    o.workspace_bytes = int(lib.tile_gemm_workspace_size(da, db, dc, o)) \
        if workspace_bytes is None else int(workspace_bytes)
    cfg = tg_config()
    n = ctypes.c_int32(0)
    _raise(lib.tile_gemm_plan(da, db, dc, o, cfg, ctypes.byref(n), None,
                              None))
    if not want_map:
        return cfg.as_dict(), n.value, None, None
    tm = -(-int(C.shape[0]) // cfg.bm) if C.shape[0] else 0
    tn = -(-int(C.shape[1]) // cfg.bn) if C.shape[1] else 0
    offs = (ctypes.c_int32 * (n.value + 1))()
    ids = (ctypes.c_int32 * max(tm * tn, 1))()
    _raise(lib.tile_gemm_plan(da, db, dc, o, cfg, ctypes.byref(n), offs,
                              ids))
    return cfg.as_dict(), n.value, list(offs), list(ids)[:tm * tn]


def tile_partition_check(ins, out, prog_offsets=None, prog_tiles=None) -> int:
    """Status of the ownership rules for descriptors `ins` (list of tg_in)
    and `out` (tg_out with its partition).  Host only; returns the status."""
    arr = (tg_in * max(len(ins), 1))(*ins)
    if prog_offsets is None:
        return int(lib.tile_partition_check(arr, len(ins), out, 0, None,
                                            None))
    po = (ctypes.c_int32 * len(prog_offsets))(*prog_offsets)
    pt = (ctypes.c_int32 * max(len(prog_tiles), 1))(*prog_tiles)
    return int(lib.tile_partition_check(arr, len(ins), out,
                                        len(prog_offsets) - 1, po, pt))


def tile_gemm_grouped_workspace_size(n: int) -> int:
    return int(lib.tile_gemm_grouped_workspace_size(int(n)))


class GroupedLaunch:
    """A prepared grouped launch: the host plan, the device workspace holding
    its problem table, and the tensors it borrows (kept alive while the
    launch exists)."""

    def __init__(self, As, Bs, Cs, workspace, plan, partitions,
                 write_count=None):
        self.As, self.Bs, self.Cs = As, Bs, Cs
        self.workspace = workspace
        self.plan = plan
        self.partitions = partitions
        self.write_count = write_count


def _grouped_descs(As, Bs, Cs, b_trans):
    n = len(As)
    ia = (tg_in * n)(*[make_in(a) for a in As])
    ib = (tg_in * n)(*[make_in(b, b_trans) for b in Bs])
    oc = (tg_out * n)(*[make_out(c) for c in Cs])
    return n, ia, ib, oc


def tile_gemm_grouped_prepare(As, Bs, Cs, *, b_trans=False, config=None,
                              workspace=None, write_count=None,
                              stream=None) -> GroupedLaunch:
    """Validate the problems and write their table; write_count (device
    int32, sum of M_i * N_i counters, problem after problem) counts
    stores."""
    n, ia, ib, oc = _grouped_descs(As, Bs, Cs, b_trans)
    need = tile_gemm_grouped_workspace_size(n)
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=Cs[0].device)
    o = make_opts(config=config, write_count=write_count)
    plan = tg_grouped_plan()
    _raise(lib.tile_gemm_grouped_prepare(
        n, ia, ib, oc, o, workspace.data_ptr(),
        workspace.numel() * workspace.element_size(), ctypes.byref(plan),
        _stream(stream)))
    return GroupedLaunch(As, Bs, Cs, workspace, plan,
                         [(oc[i].bm, oc[i].bn) for i in range(n)],
                         write_count)


def tile_autotune_grouped(As, Bs, Cs, *, b_trans=False, reps=3,
                          workspace=None, write_count=None, stream=None):
    """Time every tiled configuration of one grouped launch; returns
    (GroupedLaunch prepared with the fastest, best config dict,
    [(cfg, ms, status)])."""
    n, ia, ib, oc = _grouped_descs(As, Bs, Cs, b_trans)
    need = tile_gemm_grouped_workspace_size(n)
    if workspace is None:
        workspace = torch.empty(need, dtype=torch.uint8, device=Cs[0].device)
    res = (tg_tune_result * _MAX_CANDIDATES)()
    nres = ctypes.c_int32(0)
    best = tg_config()
    plan = tg_grouped_plan()
    _raise(lib.tile_autotune_grouped(
        n, ia, ib, oc, make_opts(write_count=write_count),
        workspace.data_ptr(), workspace.numel() * workspace.element_size(),
        int(reps), res, _MAX_CANDIDATES, ctypes.byref(nres),
        ctypes.byref(best), ctypes.byref(plan), _stream(stream)))
    rows = [(res[i].cfg.as_dict(), float(res[i].ms), int(res[i].status))
            for i in range(nres.value)]
    launch = GroupedLaunch(As, Bs, Cs, workspace, plan,
                           [(oc[i].bm, oc[i].bn) for i in range(n)],
                           write_count)
    return launch, best.as_dict(), rows


def tile_gemm_grouped(launch: GroupedLaunch, stream=None):
    _raise(lib.tile_gemm_grouped(ctypes.byref(launch.plan), _stream(stream)))
    return launch.Cs


def tile_error_norm(C, R, out=None, stream=None):
    """(sum (C-R)^2, sum R^2) in binary64 on the GPU; returns the device
    buffer of TG_ERROR_NORM_DOUBLES doubles (first two entries)."""
    if out is None:
        out = torch.empty(TG_ERROR_NORM_DOUBLES, dtype=torch.float64,
                          device=C.device)
    assert R.dtype == torch.float64 and R.numel() == C.numel()
    _raise(lib.tile_error_norm(C.data_ptr(), dtype_code(C.dtype),
                               R.data_ptr(), C.numel(), out.data_ptr(),
                               _stream(stream)))
    return out


def device_cus() -> int:
    return int(lib.tg_device_cus())


# ------------------------------------------------------------ configuration

def tile_gemm_candidates(A, B, C, bm=0, bn=0, *, b_trans=False,
                         precision="native"):
    """Configurations tile_gemm accepts for these arguments (dicts)."""
    buf = (tg_config * _MAX_CANDIDATES)()
    n = lib.tile_gemm_candidates(make_in(A), make_in(B, b_trans),
                                 make_out(C, bm, bn), make_opts(precision),
                                 buf, _MAX_CANDIDATES)
    if n < 0:
        raise TileGemmError(TG_E_ARG, last_error())
    return [buf[i].as_dict() for i in range(min(n, _MAX_CANDIDATES))]


def tile_autotune(A, B, C, bm=0, bn=0, *, b_trans=False, precision="native",
                  scale_a=None, scale_b=None, workspace=None, reps=3,
                  stream=None):
    """Time every candidate; returns (best config dict, [(cfg, ms, status)]).
    The winner is recorded in the library's tuning cache.  Without a given
    workspace one as large as the hungriest candidate needs is allocated
    here from torch."""
    res = (tg_tune_result * _MAX_CANDIDATES)()
    nres = ctypes.c_int32(0)
    best = tg_config()
    o = make_opts(precision, scale_a, scale_b, None, workspace)
    if workspace is None:
        need = max([tile_gemm_workspace_size(
            A, B, C, bm, bn, b_trans=b_trans, precision=precision,
            config=c) for c in tile_gemm_candidates(
                A, B, C, bm, bn, b_trans=b_trans, precision=precision)] +
            [0])
        if need:
            workspace = torch.empty(need, dtype=torch.uint8, device=C.device)
            o.workspace = workspace.data_ptr()
            o.workspace_bytes = need
    st = lib.tile_autotune(make_in(A), make_in(B, b_trans),
                           make_out(C, bm, bn), o, int(reps), res,
                           _MAX_CANDIDATES, ctypes.byref(nres),
                           ctypes.byref(best), _stream(stream))
    _raise(st)
    rows = [(res[i].cfg.as_dict(), float(res[i].ms), int(res[i].status))
            for i in range(nres.value)]
    return best.as_dict(), rows


def tile_tune_cache_clear():
    _raise(lib.tile_tune_cache_clear())


def tile_tune_cache_size() -> int:
    return int(lib.tile_tune_cache_size())


def tile_tune_cache_save(path):
    _raise(lib.tile_tune_cache_save(str(path).encode()))


def tile_tune_cache_load(path):
    _raise(lib.tile_tune_cache_load(str(path).encode()))


def tile_picker_features(A, B, C, config, bm=0, bn=0, *, b_trans=False):
    f = (ctypes.c_float * TG_PICKER_FEATURES)()
    c = make_config(config)
    _raise(lib.tile_picker_features(make_in(A), make_in(B, b_trans),
                                    make_out(C, bm, bn), c, f))
    return list(f)


def _fbuf(vals):
    return (ctypes.c_float * len(vals))(*[float(v) for v in vals])


def tile_picker_set(params, n_in, hidden, depth, mean, std):
    """Install a cost model (host copy); params=None removes it."""
    if params is None:
        _raise(lib.tile_picker_set(None, 0, 0, 0, None, None))
        return
    p = [float(x) for x in params]
    _raise(lib.tile_picker_set(_fbuf(p), n_in, hidden, depth, _fbuf(mean),
                               _fbuf(std)))


def tile_picker_predict(feat) -> float:
    out = ctypes.c_float(0)
    _raise(lib.tile_picker_predict(_fbuf(feat), ctypes.byref(out)))
    return float(out.value)


def tile_picker_mode(mode=-1) -> int:
    return int(lib.tile_picker_mode(int(mode)))


def tile_mlp_param_count(n_in, hidden, depth) -> int:
    return int(lib.tile_mlp_param_count(n_in, hidden, depth))


def tile_mlp_workspace_bytes(n_in, hidden, depth, batch) -> int:
    return int(lib.tile_mlp_workspace_bytes(n_in, hidden, depth, batch))


def _mlp_ws(n_in, hidden, depth, batch, device, ws):
    need = tile_mlp_workspace_bytes(n_in, hidden, depth, batch)
    if ws is None or ws.numel() * ws.element_size() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=device)
    return ws, need


def tile_mlp_forward(params, X, n_in, hidden, depth, out=None, ws=None,
                     stream=None):
    batch = X.shape[0]
    if out is None:
        out = torch.empty(batch, dtype=torch.float32, device=X.device)
    ws, need = _mlp_ws(n_in, hidden, depth, batch, X.device, ws)
    _raise(lib.tile_mlp_forward(params.data_ptr(), n_in, hidden, depth,
                                X.data_ptr(), batch, out.data_ptr(),
                                ws.data_ptr(), ws.numel(), _stream(stream)))
    return out


def tile_mlp_loss_grad(params, X, y, n_in, hidden, depth, grads=None,
                       loss=None, ws=None, stream=None):
    batch = X.shape[0]
    if grads is None:
        grads = torch.empty_like(params)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=X.device)
    ws, need = _mlp_ws(n_in, hidden, depth, batch, X.device, ws)
    _raise(lib.tile_mlp_loss_grad(params.data_ptr(), n_in, hidden, depth,
                                  X.data_ptr(), y.data_ptr(), batch,
                                  grads.data_ptr(), loss.data_ptr(),
                                  ws.data_ptr(), ws.numel(), _stream(stream)))
    return loss, grads


def tile_mlp_adam(params, grads, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999,
                  eps=1e-8, stream=None):
    _raise(lib.tile_mlp_adam(params.data_ptr(), grads.data_ptr(),
                             m.data_ptr(), v.data_ptr(), params.numel(),
                             lr, beta1, beta2, eps, int(t), _stream(stream)))
    return params
