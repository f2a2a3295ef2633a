"""Helpers shared by the GPU parity tests: decode the exact operand values
with the oracle and build oracle references from the seeded CPU inputs."""
import sys

import numpy as np
import torch

import oracle


def note(*args):
    """Name the case before a GPU step (flushed, so a crash still shows it)."""
    print("[case]", *args, flush=True)
    sys.stdout.flush()


def exact64(t: torch.Tensor) -> np.ndarray:
    """The binary64 values a CPU tensor stores, decoded by the oracle."""
    t = t.detach().cpu().contiguous()
    if t.dtype == torch.float32:
        return t.numpy().astype(np.float64)
    if t.dtype == torch.bfloat16:
        return oracle.decode_bf16(t.view(torch.int16).numpy().view(np.uint16))
    if t.dtype == torch.float8_e4m3fn:
        return oracle.decode_e4m3fn(t.view(torch.uint8).numpy())
    raise TypeError(t.dtype)


def reference(A, B, b_trans=False, sa=None, sb=None) -> np.ndarray:
    """Oracle product of the values the kernel consumes."""
    return oracle.gemm(exact64(A), exact64(B), b_nk=b_trans,
                       sa=None if sa is None else exact64(sa),
                       sb=None if sb is None else exact64(sb))


def reference_entries(A, B, ii, jj, b_trans=False, sa=None, sb=None):
    return oracle.gemm_entries(exact64(A), exact64(B), ii, jj, b_nk=b_trans,
                               sa=None if sa is None else exact64(sa),
                               sb=None if sb is None else exact64(sb))


def rel_err(C, R) -> float:
    return oracle.rel_fro(exact64(C).ravel(), np.asarray(R).ravel())


def higham_ok(C, A, B, b_trans=False, K=None, u=2.0 ** -24, out_u=None):
    """Every element within the fp32-accumulation bound
    |C - AB| <= gamma_K |A||B| (+ one output rounding)."""
    a, b = np.abs(exact64(A)), np.abs(exact64(B))
    absab = oracle.gemm(a, b, b_nk=b_trans)
    R = oracle.gemm(exact64(A), exact64(B), b_nk=b_trans)
    K = a.shape[1] if K is None else K
    g = K * u / (1 - K * u)
    c = exact64(C)
    out_u = u if out_u is None else out_u
    bound = g * absab + out_u * np.abs(R) + 1e-300
    return bool(np.all(np.abs(c - R) <= bound)), float(
        np.max(np.abs(c - R) / bound))
