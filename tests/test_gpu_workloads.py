"""Parity at the workloads' full sizes, in the launch configuration the
benchmark times (AUTO split unless stated), against the FP64 oracle.

Power law 2^20 x 2^20 (FP16/BF16 vs FP32; forward on sampled rows at both
widths, the whole forward + backward step element by element at n = 64),
GCN graph 232,965 nodes (FP32 forward + backward), and members of the
structure sweep at their full row counts (FP64/FP32/FP16).
"""
import numpy as np
import pytest
import torch

import gen
import oracle
from tests.gpu_util import (ROW_TOL, TOL, abs_forward, abs_sddmm, abs_transposed, effective_vals, make_plan,
                            quantized_dense, scaled_row_errors, to_dev)

pytestmark = pytest.mark.gpu

hs = pytest.importorskip("paper_2511_08158_amd")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def powerlaw():
    return gen.config3(n=256)


def _sample_rows(a, rows):
    """Sub-CSR of the given rows (for the oracle to evaluate one by one)."""
    lens = np.diff(a.row_ptr)[rows]
    rp = np.concatenate([[0], np.cumsum(lens)])
    sl = [slice(a.row_ptr[r], a.row_ptr[r + 1]) for r in rows]
    col = np.concatenate([a.col_idx[s] for s in sl])
    val = np.concatenate([a.vals[s] for s in sl])
    return rp, col, val


@pytest.mark.parametrize("dtype", [torch.float16, torch.bfloat16, torch.float32])
@pytest.mark.parametrize("n", [64, 256])
def test_powerlaw_full_size(powerlaw, dtype, n):
    a, b = powerlaw
    b = b[:, :n]
    print(f"powerlaw dtype={dtype} n={n}", flush=True)
    plan = make_plan(hs, a, dtype, "auto")
    info = plan.info()
    assert info["long_rows"] > 0          # the 20,000-entry rows are split
    C = plan.run(to_dev(b, dtype))
    torch.cuda.synchronize()
    # sampled rows: the longest ones, rows of every part, and random rows
    g = np.random.default_rng(0)
    lens = np.diff(a.row_ptr)
    rows = np.unique(np.concatenate([np.argsort(lens)[-8:], g.choice(a.m, 3000, replace=False)]))
    rp, col, val = _sample_rows(a, rows)
    Cs = C[torch.as_tensor(rows, device=C.device)].double().cpu().numpy()
    ref = oracle.spmm(rows.size, a.k, rp, col, val, b)
    assert oracle.rel_err(Cs, ref) <= TOL[dtype]
    if dtype != torch.float32:
        # kernel error on the stored operands (same rows, same quantisation)
        Aq = effective_vals(a.m, a.row_ptr, a.vals, dtype)
        _, _, valq = _sample_rows(gen.Csr(a.m, a.k, a.row_ptr, a.col_idx, Aq), rows)
        refk = oracle.spmm(rows.size, a.k, rp, col, valq, quantized_dense(b, dtype))
        assert oracle.rel_err(Cs, refk) <= 1e-5


@pytest.mark.parametrize("dtype", [torch.float16, torch.bfloat16])
def test_powerlaw_bcsr_only_mfma_at_scale(powerlaw, dtype):
    """Every row block through the FP16/BF16 MFMA kernel at 2^20 rows."""
    a, b = powerlaw
    b = b[:, :64]
    plan = make_plan(hs, a, dtype, "bcsr")
    C = plan.run(to_dev(b, dtype))
    torch.cuda.synchronize()
    rows = np.random.default_rng(1).choice(a.m, 2000, replace=False)
    rows.sort()
    rp, col, val = _sample_rows(a, rows)
    Cs = C[torch.as_tensor(rows, device=C.device)].double().cpu().numpy()
    assert oracle.rel_err(Cs, oracle.spmm(rows.size, a.k, rp, col, val, b)) <= TOL[dtype]


def test_gcn_full_forward_backward():
    a, x = gen.config4()
    print(f"gcn nnz={a.nnz}", flush=True)
    G = gen.dense(0, gen.GRAD, a.m, x.shape[1])
    plan = make_plan(hs, a, torch.float32, "auto", backward=True)
    X = to_dev(x, torch.float32)
    C = plan.run(X)
    dX, dA = plan.backward(X, to_dev(G, torch.float32))
    torch.cuda.synchronize()
    assert oracle.rel_err(C.double().cpu().numpy(), oracle.spmm(a.m, a.k, a.row_ptr, a.col_idx, a.vals, x)) <= 1e-5
    assert oracle.rel_err(dX.double().cpu().numpy(),
                          oracle.spmm_t(a.m, a.k, a.row_ptr, a.col_idx, a.vals, G)) <= 1e-5
    assert oracle.rel_err(dA.double().cpu().numpy(),
                          oracle.sddmm(a.m, a.k, a.row_ptr, a.col_idx, G, x)) <= 1e-5


@pytest.mark.parametrize("i", [1, 2, 5, 6, 7, 9, 10, 14])
def test_sweep_members(i):
    """Small members of the structure sweep (uniform / banded / block
    diagonal / power law) in FP64, FP32 and FP16, AUTO vs CSR-only."""
    spec = gen.config5_spec(i)
    a = gen.config5(i)
    print(f"sweep {i} {spec}", flush=True)
    n = gen.SWEEP_N[i % 5]
    b = gen.dense(i, gen.DENSE, a.k, n, "uniform")
    ref = oracle.spmm(a.m, a.k, a.row_ptr, a.col_idx, a.vals, b)
    for dtype in (torch.float64, torch.float32, torch.float16):
        for split in ("auto", "csr"):
            plan = make_plan(hs, a, dtype, split)
            C = plan.run(to_dev(b, dtype))
            torch.cuda.synchronize()
            assert oracle.rel_err(C.double().cpu().numpy(), ref) <= TOL[dtype], (dtype, split)


@pytest.mark.parametrize("dtype", [torch.float16, torch.bfloat16, torch.float32])
def test_powerlaw_backward_full_size(powerlaw, dtype):
    """The power-law workload's whole step at 2^20 rows, n = 64: C, dB =
    A^T dC (through the transposed plan, whose hub columns become rows of up
    to thousands of entries) and dA = SDDMM(dC, B), every element against the
    FP64 oracle on the unrounded inputs, by Frobenius norm and row by row."""
    a, b = powerlaw
    n = 64
    b = np.ascontiguousarray(b[:, :n])
    G = gen.dense(0, gen.GRAD, a.m, n)
    print(f"powerlaw backward dtype={dtype}", flush=True)
    plan = make_plan(hs, a, dtype, "auto", backward=True, n_hint=n)
    Bd = to_dev(b, dtype)
    C = plan.run(Bd)
    dB, dA = plan.backward(Bd, to_dev(G, torch.float32))
    torch.cuda.synchronize()
    C, dB, dA = (t.double().cpu().numpy() for t in (C, dB, dA))
    checks = (
        ("C", C, oracle.spmm(a.m, a.k, a.row_ptr, a.col_idx, a.vals, b), abs_forward(a, b)),
        ("dB", dB, oracle.spmm_t(a.m, a.k, a.row_ptr, a.col_idx, a.vals, G), abs_transposed(a, G)),
        ("dA", dA, oracle.sddmm(a.m, a.k, a.row_ptr, a.col_idx, G, b), abs_sddmm(a, G, b)),
    )
    for name, x, ref, absref in checks:
        assert oracle.rel_err(x, ref) <= TOL[dtype], name
        worst = float(scaled_row_errors(x, ref, absref).max())
        print(f"  {name}: rel {oracle.rel_err(x, ref):.2e}, worst row {worst:.2e}", flush=True)
        assert worst <= ROW_TOL[dtype], name
