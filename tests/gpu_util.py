"""Helpers shared by the GPU tests: build plans through the C ABI binding and
compare against the FP64 oracle."""
from __future__ import annotations

import numpy as np
import torch

import oracle
from oracle import loops_ref as L

TOL = {torch.float64: 1e-12, torch.float32: 1e-5, torch.float16: 5e-3, torch.bfloat16: 5e-3}
SPLITS = ("auto", "csr", "bcsr", "boundary")


def dev():
    return torch.device("cuda:0")


def to_dev(x, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(dev())


def quantized_dense(B, dtype):
    """B rounded to `dtype` (torch's conversion), returned as FP64 numpy."""
    return torch.as_tensor(B).to(dtype).to(torch.float64).numpy()


def rounded_slabs(G, row_blocks, dtype=torch.float16):
    """dC as the FP16/BF16 SDDMM's matrix-core form reads it: each listed
    16-row block scaled by the power of two 2^(e-15) that puts its largest
    magnitude in [2^14, 2^15) (e held at -111 or above, so a slab below
    2^-112 is scaled by 2^126 only), rounded to `dtype` (nearest even) and
    scaled back; other rows unchanged."""
    out = np.array(G, dtype=np.float64, copy=True)
    for rb in np.asarray(row_blocks):
        sl = slice(16 * int(rb), min(16 * int(rb) + 16, out.shape[0]))
        mx = float(np.max(np.abs(out[sl]))) if out[sl].size else 0.0
        if mx == 0.0 or not np.isfinite(mx):
            continue
        e = max(int(np.frexp(np.float32(mx))[1]), -111)
        s = np.ldexp(1.0, e - 15)
        q = torch.as_tensor(out[sl] / s).to(torch.float32).to(dtype).to(torch.float64).numpy()
        out[sl] = q * s
    return out


def effective_vals(a_m, row_ptr, vals, dtype):
    """Values of A as the plan stores them, in FP64: FP64 exact, FP32
    rounded, FP16/BF16 quantised per 16-row block (oracle's quantize_ref)."""
    if dtype == torch.float64:
        return np.asarray(vals, dtype=np.float64)
    if dtype == torch.float32:
        return np.asarray(vals, dtype=np.float64).astype(np.float32).astype(np.float64)
    fmt = "f16" if dtype == torch.float16 else "bf16"
    _, _, deq = L.quantize_ref(a_m, row_ptr, vals, 16, fmt)
    return deq


def oracle_forward(a, B):
    return oracle.spmm(a.m, a.k, a.row_ptr, a.col_idx, a.vals, B)


def make_plan(hs, a, dtype, split="auto", backward=False, vals_dtype=torch.float64, **kw):
    return hs.Plan(a.row_ptr, a.col_idx, to_dev(a.vals, vals_dtype), (a.m, a.k), compute=dtype,
                   split=split, backward=backward, **kw)


def scaled_row_errors(X, ref, absref):
    """Per-row error of X against ref, each row measured against the row of
    |A| |B| (absref, the scale any rounding error of that row is bounded
    by): ||X_i - ref_i|| / ||absref_i|| (rows whose absref is zero must
    match exactly and count 0 if they do, inf otherwise).  Unlike a norm over
    the whole matrix, one wrong row cannot hide among many right ones."""
    X = np.asarray(X, dtype=np.float64).reshape(len(ref), -1)
    ref = np.asarray(ref, dtype=np.float64).reshape(len(ref), -1)
    absref = np.asarray(absref, dtype=np.float64).reshape(len(ref), -1)
    num = np.linalg.norm(X - ref, axis=1)
    den = np.linalg.norm(absref, axis=1)
    out = np.where(den > 0, num / np.where(den > 0, den, 1.0), np.where(num == 0, 0.0, np.inf))
    return out


def abs_forward(a, B):
    """|A| |B| by the oracle: the per-row error scale of C = A B."""
    return oracle.spmm(a.m, a.k, a.row_ptr, a.col_idx, np.abs(a.vals), np.abs(B))


def abs_transposed(a, G):
    """|A|^T |G| by the oracle: the per-row error scale of dB = A^T G."""
    return oracle.spmm_t(a.m, a.k, a.row_ptr, a.col_idx, np.abs(a.vals), np.abs(G))


def abs_sddmm(a, G, B):
    """<|G_row(e)|, |B_col(e)|> by the oracle: the error scale of each dA[e]."""
    return oracle.sddmm(a.m, a.k, a.row_ptr, a.col_idx, np.abs(G), np.abs(B))


# Per-row bars of scaled_row_errors.  Rounding each input of a product to the
# compute type moves it by at most 2u |a||b| (u = 2^-53 FP64, 2^-24 FP32,
# 2^-11 FP16, 2^-8 BF16), and an FP32 (FP64) sum of L terms adds at most
# L u_acc sum |a||b|; rows here have at most a few thousand terms.  The bars
# sit a few times above those bounds.
ROW_TOL = {torch.float64: 1e-12, torch.float32: 1e-5, torch.float16: 2e-3, torch.bfloat16: 1e-2}
