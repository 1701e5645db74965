"""The one-pass backward: dB = A^T dC and dA = SDDMM(dC, B) computed together
on the BCSR-part of A^T, each tile's gathered row of dC serving its dB
product and its entries' dA dot products (Sec. 3.3 product and its gradient).

It must be taken exactly when the plan and operands qualify (FP32 / FP64,
A^T all BCSR-part, n up to 256 FP32 / 128 FP64, 16-byte rows), give dB
bitwise equal to the separate product (the same MFMA walk), and give dA
against the oracle within the precision's bars, per entry (each entry
scaled by <|dC_row|, |B_col|>), over ragged shapes, empty row blocks, row
blocks of A^T with thousands of tiles, unsorted duplicated input and every
qualifying width class."""
import numpy as np
import pytest
import torch

import gen
import oracle
from tests.gpu_util import ROW_TOL, TOL, abs_sddmm, abs_transposed, make_plan, scaled_row_errors, to_dev

pytestmark = pytest.mark.gpu

hs = pytest.importorskip("paper_2511_08158_amd")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _messy(seed, m=150, k=130, extra=120):
    """Rows grouped, columns shuffled inside rows, duplicated entries."""
    g = np.random.default_rng(seed)
    a = gen.random_csr(seed, m, k, 0.1)
    r = np.concatenate([a.rows(), g.integers(0, m, extra)])
    c = np.concatenate([a.col_idx, g.integers(0, k, extra)])
    v = g.standard_normal(r.size)
    order = np.lexsort((g.random(r.size), r))
    r, c, v = r[order], c[order], v[order]
    rp = np.zeros(m + 1, np.int64)
    np.add.at(rp, r + 1, 1)
    return gen.Csr(m, k, np.cumsum(rp).astype(np.int32), c.astype(np.int32), v)


def _matrix(kind):
    if kind == "stencil":
        a, _ = gen.config2(grid=12)                    # 576 rows, 5 % random entries
        return a
    if kind == "ragged":
        return gen.random_csr(3, 301, 275, 0.04)     # ragged last row blocks of A and A^T
    if kind == "empty_blocks":
        a = gen.random_csr(4, 333, 250, 0.05)
        keep = (a.col_idx // 16) % 3 != 1             # every third row block of A^T empty
        return gen.csr_from_coo(a.m, a.k, a.rows()[keep], a.col_idx[keep], a.vals[keep])
    if kind == "long_blocks":
        # row blocks of A^T with about 2000 tiles: many chunks of 64 tiles
        # and a partial last round of 16
        return gen.random_csr(5, 1990, 41, 0.3)
    if kind == "messy":
        return _messy(6)
    raise ValueError(kind)


# every width class of the two workgroup shapes (two waves up to 128 FP32 /
# 64 FP64 columns, four waves up to 256 / 128), partial last column chunks
WIDTHS = {torch.float32: [4, 8, 36, 64, 68, 100, 128, 132, 200, 256],
          torch.float64: [2, 6, 32, 34, 64, 66, 100, 128]}


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("kind", ["stencil", "ragged", "empty_blocks", "long_blocks", "messy"])
def test_fused_backward(dtype, kind, monkeypatch):
    a = _matrix(kind)
    plan = make_plan(hs, a, dtype, "bcsr", backward=True)
    for n in WIDTHS[dtype]:
        print(f"fused backward dtype={dtype} kind={kind} n={n}", flush=True)
        g = np.random.default_rng(n)
        B = g.standard_normal((a.k, n))
        G = g.standard_normal((a.m, n))
        Bd, Gd = to_dev(B, dtype), to_dev(G, dtype)
        monkeypatch.setenv("HSPMM_BWD_FUSED", "1")
        assert plan.backward_fused(Bd, Gd)
        dB_f, dA_f = plan.backward(Bd, Gd)
        monkeypatch.setenv("HSPMM_BWD_FUSED", "0")
        assert not plan.backward_fused(Bd, Gd)
        dB_s, dA_s = plan.backward(Bd, Gd)
        torch.cuda.synchronize()
        monkeypatch.delenv("HSPMM_BWD_FUSED")
        assert torch.equal(dB_f, dB_s)
        ref_dB = oracle.spmm_t(a.m, a.k, a.row_ptr, a.col_idx, a.vals, G)
        assert oracle.rel_err(dB_f.double().cpu().numpy(), ref_dB) <= TOL[dtype]
        assert scaled_row_errors(dB_f.double().cpu().numpy(), ref_dB, abs_transposed(a, G)).max() <= ROW_TOL[dtype]
        ref_dA = oracle.sddmm(a.m, a.k, a.row_ptr, a.col_idx, G, B)
        scale_dA = abs_sddmm(a, G, B)
        for dA in (dA_f, dA_s):
            x = dA.double().cpu().numpy()
            assert oracle.rel_err(x, ref_dA) <= TOL[dtype]
            err = np.abs(x - ref_dA) / np.where(scale_dA > 0, scale_dA, 1.0)
            assert err.max() <= ROW_TOL[dtype]


def test_fused_integer_inputs_bitwise():
    """Integer A, B, dC with small sums: every partial sum is exact in FP32,
    so dB and dA equal the oracle bit for bit whatever the summation order."""
    a = gen.random_csr(7, 260, 230, 0.06, dist="int")
    g = np.random.default_rng(7)
    n = 64
    B = g.integers(-3, 4, (a.k, n)).astype(float)
    G = g.integers(-3, 4, (a.m, n)).astype(float)
    plan = make_plan(hs, a, torch.float32, "bcsr", backward=True)
    Bd, Gd = to_dev(B, torch.float32), to_dev(G, torch.float32)
    assert plan.backward_fused(Bd, Gd)
    dB, dA = plan.backward(Bd, Gd)
    torch.cuda.synchronize()
    assert np.array_equal(dB.double().cpu().numpy(), oracle.spmm_t(a.m, a.k, a.row_ptr, a.col_idx, a.vals, G))
    assert np.array_equal(dA.double().cpu().numpy(), oracle.sddmm(a.m, a.k, a.row_ptr, a.col_idx, G, B))


def test_fused_only_when_it_qualifies():
    """Cases outside the one-pass path say so and still give the right
    gradients through the separate products."""
    a = gen.random_csr(8, 200, 180, 0.05)
    g = np.random.default_rng(8)
    # wider than one panel, a CSR-part in A^T, and a low-precision plan
    cases = [(torch.float32, "bcsr", 260), (torch.float64, "bcsr", 130), (torch.float32, "csr", 64),
             (torch.float16, "bcsr", 64)]
    for dtype, split, n in cases:
        print(f"fused qualification dtype={dtype} split={split} n={n}", flush=True)
        plan = make_plan(hs, a, dtype, split, backward=True)
        od = torch.float64 if dtype == torch.float64 else torch.float32
        B = g.standard_normal((a.k, n))
        G = g.standard_normal((a.m, n))
        Bd, Gd = to_dev(B, dtype), to_dev(G, od)
        assert not plan.backward_fused(Bd, Gd)
        dB, dA = plan.backward(Bd, Gd)
        torch.cuda.synchronize()
        tol = TOL[dtype]
        assert oracle.rel_err(dB.double().cpu().numpy(),
                              oracle.spmm_t(a.m, a.k, a.row_ptr, a.col_idx, a.vals, G)) <= max(tol, 1e-5)
    # a misaligned dC (offset by one element) is not taken either
    plan = make_plan(hs, a, torch.float32, "bcsr", backward=True)
    Bd = to_dev(g.standard_normal((a.k, 64)), torch.float32)
    Gbig = to_dev(g.standard_normal((a.m * 64 + 1,)), torch.float32)
    Gd = Gbig[1:].view(a.m, 64)
    assert not plan.backward_fused(Bd, Gd)


def test_fused_one_gradient_requests_use_separate_products():
    """Asking for one gradient runs that product alone, with the same
    results as the fused call."""
    a = _matrix("stencil")
    n = 128
    g = np.random.default_rng(9)
    Bd = to_dev(g.standard_normal((a.k, n)), torch.float32)
    Gd = to_dev(g.standard_normal((a.m, n)), torch.float32)
    plan = make_plan(hs, a, torch.float32, "bcsr", backward=True)
    assert plan.backward_fused(Bd, Gd)
    dB, dA = plan.backward(Bd, Gd)
    dB1, _ = plan.backward(Bd, Gd, need_dB=True, need_dA=False)
    _, dA1 = plan.backward(Bd, Gd, need_dB=False, need_dA=True)
    torch.cuda.synchronize()
    assert torch.equal(dB, dB1)
    ref = oracle.sddmm(a.m, a.k, a.row_ptr, a.col_idx, Gd.double().cpu().numpy(), Bd.double().cpu().numpy())
    assert oracle.rel_err(dA.double().cpu().numpy(), ref) <= 1e-5
    assert oracle.rel_err(dA1.double().cpu().numpy(), ref) <= 1e-5
