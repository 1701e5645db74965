"""The one-pass backward: dB = A^T dC and dA = SDDMM(dC, B) computed together
on the BCSR-part of A^T, each tile's gathered row of dC serving its dB
product and its entries' dA dot products (Sec. 3.3 product and its gradient).

It must be taken exactly when the plan and operands qualify (n up to 256
FP32 / 128 FP64 with 16-byte rows; a BCSR-part in A^T only for FP32 /
FP64 plans), give dB bitwise equal to the separate product (the same walk
of each part), and give dA against the oracle within FP32's (FP64's)
bars, per entry (each entry scaled by <|dC_row|, |B_col|>; for FP16 / BF16
plans the dot products run in FP32 on the rounded B), over ragged shapes,
empty row blocks, row blocks of A^T with thousands of tiles, long rows of
A^T cut into segments, unsorted duplicated input, each split and every
width class."""
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


def _hub(seed=10, m=700, k=300):
    """Columns 0 and 1 used by most rows: long rows of A^T, cut into
    segments whose partial rows are summed afterwards."""
    g = np.random.default_rng(seed)
    a = gen.random_csr(seed, m, k, 0.02)
    r = np.concatenate([a.rows(), np.arange(m), np.arange(0, m, 2)])
    c = np.concatenate([a.col_idx, np.zeros(m, np.int32), np.ones((m + 1) // 2, np.int32)])
    key = np.unique(r.astype(np.int64) * k + c)
    return gen.csr_from_coo(m, k, key // k, key % k, g.standard_normal(key.size))


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
    if kind == "hub":
        return _hub()
    raise ValueError(kind)


# every width class of the two workgroup shapes of the BCSR-part (two waves
# up to 128 FP32 / 64 FP64 columns, four waves up to 256 / 128) and of the
# CSR-part's lane groups (4 to 64 lanes), partial last column chunks
WIDTHS = {torch.float32: [4, 8, 36, 64, 68, 100, 128, 132, 200, 256],
          torch.float64: [2, 6, 32, 34, 64, 66, 100, 128],
          torch.float16: [4, 64, 128, 132, 200, 256],
          torch.bfloat16: [36, 128, 256]}
OUT = {torch.float64: torch.float64}

CASES = ([(dt, k, sp) for dt in (torch.float32, torch.float64)
          for k in ("stencil", "ragged", "empty_blocks", "long_blocks", "messy", "hub") for sp in ("bcsr", "csr", "auto")]
         + [(dt, k, "csr") for dt in (torch.float16, torch.bfloat16) for k in ("stencil", "messy", "hub")])


@pytest.mark.parametrize("dtype,kind,split", CASES)
def test_fused_backward(dtype, kind, split, monkeypatch):
    a = _matrix(kind)
    plan = make_plan(hs, a, dtype, split, backward=True)
    od = OUT.get(dtype, torch.float32)
    for n in WIDTHS[dtype]:
        print(f"fused backward dtype={dtype} kind={kind} split={split} n={n}", flush=True)
        g = np.random.default_rng(n)
        B = g.standard_normal((a.k, n))
        G = g.standard_normal((a.m, n))
        Bd, Gd = to_dev(B, dtype), to_dev(G, od)
        monkeypatch.setenv("HSPMM_BWD_FUSED", "1")
        fused = plan.backward_fused(Bd, Gd)
        # a CSR-part in A^T is fused from 256-byte rows of B
        wide = n * Bd.element_size() >= 256
        if split == "bcsr" or wide:
            assert fused
        if split == "csr" and not wide:
            assert not fused
        dB_f, dA_f = plan.backward(Bd, Gd)
        monkeypatch.setenv("HSPMM_BWD_FUSED", "0")
        assert not plan.backward_fused(Bd, Gd)
        dB_s, dA_s = plan.backward(Bd, Gd)
        torch.cuda.synchronize()
        monkeypatch.delenv("HSPMM_BWD_FUSED")
        # the same dB walk in both forms
        assert torch.equal(dB_f, dB_s)
        ref_dB = oracle.spmm_t(a.m, a.k, a.row_ptr, a.col_idx, a.vals, G)
        assert oracle.rel_err(dB_f.double().cpu().numpy(), ref_dB) <= TOL[dtype]
        assert scaled_row_errors(dB_f.double().cpu().numpy(), ref_dB, abs_transposed(a, G)).max() <= ROW_TOL[dtype]
        # dA against the oracle on the plan's B (FP16 / BF16: B as rounded)
        Bq = Bd.double().cpu().numpy()
        ref_dA = oracle.sddmm(a.m, a.k, a.row_ptr, a.col_idx, G, Bq)
        scale_dA = abs_sddmm(a, G, Bq)
        x = dA_f.double().cpu().numpy()
        assert oracle.rel_err(x, ref_dA) <= min(TOL[dtype], 1e-5)
        err = np.abs(x - ref_dA) / np.where(scale_dA > 0, scale_dA, 1.0)
        assert err.max() <= min(ROW_TOL[dtype], 1e-5)
        assert oracle.rel_err(dA_s.double().cpu().numpy(), oracle.sddmm(a.m, a.k, a.row_ptr, a.col_idx, G, B)) <= TOL[dtype]


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
    # wider than the widest form, a CSR-part in A^T with rows of B under
    # 256 bytes, and a low-precision plan with a BCSR-part in A^T (its MFMA
    # form holds B in the compute type)
    cases = [(torch.float32, "bcsr", 260), (torch.float64, "bcsr", 130), (torch.float32, "csr", 260),
             (torch.float32, "csr", 32), (torch.float16, "csr", 64), (torch.float16, "bcsr", 128),
             (torch.bfloat16, "bcsr", 128)]
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
