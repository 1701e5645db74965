"""GPU parity of the hybrid SpMM against the FP64 oracle, through the C ABI.

Bars: FP64 relative Frobenius error <= 1e-12, FP32 <= 1e-5, FP16/BF16
(FP32 accumulation) <= 5e-3 against the oracle on the original FP64 inputs;
bit-exact where every partial sum is exact (integer-valued inputs) and for
every integer array of the built format (Alg. 1 replayed on the CPU).
"""
import numpy as np
import pytest
import torch

import gen
import oracle
from oracle import loops_ref as L
from tests.gpu_util import (SPLITS, TOL, dev, effective_vals, make_plan, oracle_forward,
                            quantized_dense, to_dev)

pytestmark = pytest.mark.gpu

hs = pytest.importorskip("paper_2511_08158_amd")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _run(plan, B, dtype):
    C = plan.run(to_dev(B, dtype))
    torch.cuda.synchronize()
    return C.double().cpu().numpy()


# ---------------------------------------------------------------------------
# config 1: 4096 x 4096, 10 per row, FP64, N = 32
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("split", SPLITS)
def test_config1_fp64_all_splits(split):
    a, b = gen.config1()
    print(f"config1 fp64 split={split}", flush=True)
    plan = make_plan(hs, a, torch.float64, split)
    C = _run(plan, b, torch.float64)
    ref = oracle_forward(a, b)
    assert oracle.rel_err(C, ref) <= 1e-12


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.float16, torch.bfloat16])
@pytest.mark.parametrize("split", SPLITS)
def test_integer_valued_bitwise(dtype, split):
    """Every partial sum exact => the result equals the oracle bit for bit,
    whatever the split, tile order or reduction tree."""
    print(f"integer dtype={dtype} split={split}", flush=True)
    a = gen.random_csr(11, 203, 177, 0.08, dist="int")
    g = np.random.default_rng(3)
    B = g.integers(-4, 5, (a.k, 48)).astype(np.float64)
    plan = make_plan(hs, a, dtype, split)
    C = _run(plan, B, dtype)
    assert np.array_equal(C, oracle_forward(a, B))


def test_identity_and_permutation_bitwise():
    m = 333
    g = np.random.default_rng(1)
    B = g.standard_normal((m, 40))
    p = g.permutation(m)
    for cols in (np.arange(m), p):
        a = gen.csr_from_coo(m, m, np.arange(m), cols, np.ones(m))
        for split in SPLITS:
            plan = make_plan(hs, a, torch.float64, split)
            assert np.array_equal(_run(plan, B, torch.float64), B[cols])


# ---------------------------------------------------------------------------
# ragged shapes, several tiles, every dtype and split
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.float16, torch.bfloat16])
@pytest.mark.parametrize("n", [1, 3, 16, 36, 64, 130, 256, 520])
def test_ragged_all_splits(dtype, n):
    print(f"ragged dtype={dtype} n={n}", flush=True)
    a = gen.random_csr(5, 357, 291, 0.05)
    B = np.random.default_rng(n).standard_normal((a.k, n))
    Bq = quantized_dense(B, dtype)
    Aq = effective_vals(a.m, a.row_ptr, a.vals, dtype)
    ref_e2e = oracle_forward(a, B)
    ref_k = oracle.spmm(a.m, a.k, a.row_ptr, a.col_idx, Aq, Bq)
    for split in SPLITS:
        plan = make_plan(hs, a, dtype, split)
        C = _run(plan, B, dtype)
        assert oracle.rel_err(C, ref_e2e) <= TOL[dtype], split
        # kernel error against the oracle on the stored (quantised) operands
        kt = 1e-12 if dtype == torch.float64 else 2e-6
        assert oracle.rel_err(C, ref_k) <= kt, split


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.float16])
def test_split_launch_equals_fused(dtype, monkeypatch):
    """HSPMM_HYBRID_LAUNCH=2 launches the two parts as two kernels instead of
    one fused launch: the same per-row work, so C, dB and dA are bitwise
    equal to the fused launch's."""
    a = gen.random_csr(9, 420, 390, 0.04)
    g = np.random.default_rng(6)
    rows = np.repeat(np.arange(a.m), np.diff(a.row_ptr))
    keep = (rows < 200) | (rows >= 260)
    # rows 200..259 hold a dense 60 x 40 block: BCSR row blocks; the rest CSR
    extra_r = np.repeat(np.arange(200, 260), 40)
    extra_c = np.tile(np.arange(100, 140), 60)
    a = gen.csr_from_coo(a.m, a.k, np.concatenate([rows[keep], extra_r]),
                         np.concatenate([a.col_idx[keep], extra_c]),
                         np.concatenate([a.vals[keep], g.standard_normal(extra_r.size)]))
    plan = make_plan(hs, a, dtype, "boundary", backward=True, r_boundary=208)
    info = plan.info()
    assert info["rows_csr"] == 208 and info["rb_bcsr"] == (a.m - 208 + 15) // 16
    B = g.standard_normal((a.k, 48))
    G = g.standard_normal((a.m, 48))
    od = torch.float64 if dtype == torch.float64 else torch.float32
    out = {}
    for mode in ("1", "2"):
        monkeypatch.setenv("HSPMM_HYBRID_LAUNCH", mode)
        C = plan.run(to_dev(B, dtype))
        dB, dA = plan.backward(to_dev(B, dtype), to_dev(G, od))
        torch.cuda.synchronize()
        out[mode] = [t.double().cpu().numpy() for t in (C, dB, dA)]
    monkeypatch.delenv("HSPMM_HYBRID_LAUNCH", raising=False)
    for x, y in zip(out["1"], out["2"]):
        assert np.array_equal(x, y)
    assert oracle.rel_err(out["1"][0], oracle_forward(a, B)) <= TOL[dtype]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.float16, torch.bfloat16])
@pytest.mark.parametrize("pad", [3, 8])
def test_leading_dimensions(dtype, pad):
    """B and C as column slices of wider matrices (ld = n + pad): pad 8
    keeps 16-byte rows (the vector kernels, bitwise equal to contiguous
    operands), pad 3 breaks them (the one-column-per-lane kernels, checked
    against the oracle); the backward reads B with the same leading
    dimension."""
    a = gen.random_csr(23, 300, 260, 0.05)
    n = 40
    g = np.random.default_rng(pad)
    B = g.standard_normal((a.k, n))
    G = g.standard_normal((a.m, n))
    od = torch.float64 if dtype == torch.float64 else torch.float32
    for split in ("auto", "csr", "bcsr"):
        plan = make_plan(hs, a, dtype, split, backward=True)
        Bc = to_dev(B, dtype)
        Bw = torch.zeros((a.k, n + pad), dtype=dtype, device=Bc.device)
        Bw[:, :n] = Bc
        Cw = torch.full((a.m, n + pad), 7.0, dtype=od, device=Bc.device)
        C1 = plan.run(Bc)
        C2 = plan.run(Bw[:, :n], out=Cw[:, :n])
        dB1, dA1 = plan.backward(Bc, to_dev(G, od))
        dB2, dA2 = plan.backward(Bw[:, :n], to_dev(G, od))
        torch.cuda.synchronize()
        assert torch.all(Cw[:, n:] == 7.0), split          # nothing written past n
        c1, c2 = C1.double().cpu().numpy(), C2.double().cpu().numpy()
        if pad == 8:
            assert np.array_equal(c1, c2), split
            assert torch.equal(dB1, dB2) and torch.equal(dA1, dA2), split
        assert oracle.rel_err(c2, oracle_forward(a, B)) <= TOL[dtype], split
        assert oracle.rel_err(dA2.double().cpu().numpy(), oracle.sddmm(a.m, a.k, a.row_ptr, a.col_idx, G, B)) <= TOL[dtype], split


def test_empty_and_degenerate():
    # empty rows, an empty matrix, nnz = 0, a single column
    a = gen.csr_from_coo(40, 30, np.array([3, 3, 17]), np.array([0, 29, 5]), np.array([1.0, 2.0, 3.0]))
    B = np.random.default_rng(0).standard_normal((30, 8))
    for split in SPLITS:
        plan = make_plan(hs, a, torch.float32, split)
        assert oracle.rel_err(_run(plan, B, torch.float32), oracle_forward(a, B)) <= 1e-6
    z = gen.csr_from_coo(20, 10, np.zeros(0, int), np.zeros(0, int))
    plan = make_plan(hs, z, torch.float32, "auto")
    assert np.array_equal(_run(plan, np.ones((10, 4)), torch.float32), np.zeros((20, 4)))
    one = gen.csr_from_coo(5, 1, np.arange(5), np.zeros(5, int), np.arange(5.0))
    plan = make_plan(hs, one, torch.float64, "bcsr")
    assert np.array_equal(_run(plan, np.full((1, 3), 2.0), torch.float64), np.arange(5.0)[:, None] * 2.0 * np.ones((1, 3)))


def test_long_rows_are_split_deterministically():
    """Rows far longer than a wave's share are cut into segments and summed
    in a fixed order: parity and bitwise-repeatable results."""
    g = np.random.default_rng(4)
    m, k = 64, 20000
    lens = np.full(m, 5)
    lens[[3, 40]] = [9000, 17000]
    rows = np.repeat(np.arange(m), lens)
    cols = np.concatenate([np.sort(g.choice(k, l, replace=False)) for l in lens])
    a = gen.csr_from_coo(m, k, rows, cols, g.standard_normal(rows.size))
    B = g.standard_normal((k, 64))
    plan = make_plan(hs, a, torch.float32, "csr")
    assert plan.info()["long_rows"] == 2
    C1 = _run(plan, B, torch.float32)
    C2 = _run(plan, B, torch.float32)
    assert np.array_equal(C1, C2)
    assert oracle.rel_err(C1, oracle_forward(a, B)) <= 1e-5


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.float16])
@pytest.mark.parametrize("n", [5, 64, 300])
@pytest.mark.parametrize("longest", [1500, 17000])
def test_long_row_reduce_forms(dtype, n, longest):
    """Partial rows of split rows are summed by one workgroup per (row,
    column chunk): rows of 4 and 47 (small workgroup) or 532 segments (large
    workgroup), n odd (one column per lane), 64 (one chunk) and 300 (two or
    three chunks of 16-byte loads); parity and bitwise-repeatable results."""
    print(f"long-row reduce dtype={dtype} n={n} longest={longest}", flush=True)
    g = np.random.default_rng(11)
    m, k = 96, 20000
    lens = np.full(m, 3)
    lens[[0, 17, 95]] = [100, 1500, longest]
    rows = np.repeat(np.arange(m), lens)
    cols = np.concatenate([np.sort(g.choice(k, l, replace=False)) for l in lens])
    a = gen.csr_from_coo(m, k, rows, cols, g.standard_normal(rows.size))
    B = g.standard_normal((k, n))
    plan = make_plan(hs, a, dtype, "csr")
    assert plan.info()["long_rows"] == 3
    C1 = _run(plan, B, dtype)
    C2 = _run(plan, B, dtype)
    assert np.array_equal(C1, C2)
    assert oracle.rel_err(C1, oracle_forward(a, B)) <= TOL[dtype]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_wide_row_blocks_forward(dtype):
    """FP32/FP64 BCSR-parts run one wave per row block when every row block
    has at most 2048 tiles and the four-wave split otherwise: a plan with one
    row block of ~10,000 tiles (integer values, bitwise against the oracle)
    and the same matrix without it (the one-wave form) give the oracle's
    result, and so do both forms on a real-valued copy within tolerance."""
    print(f"wide row blocks dtype={dtype}", flush=True)
    g = np.random.default_rng(23)
    m, k, n = 50, 12000, 40
    dens = np.full(m, 0.004)
    dens[16:32] = 0.1                      # row block 1: ~9,800 distinct columns
    rows, cols = [], []
    for i in range(m):
        c = np.flatnonzero(g.random(k) < dens[i])
        rows.append(np.full(c.size, i)); cols.append(c)
    rows = np.concatenate(rows); cols = np.concatenate(cols)
    vals = g.integers(-3, 4, rows.size).astype(float)
    a = gen.csr_from_coo(m, k, rows, cols, vals)
    B = g.integers(-3, 4, (k, n)).astype(float)
    wide = make_plan(hs, a, dtype, "bcsr")
    assert wide.info()["nblk"] > 2048
    assert np.array_equal(_run(wide, B, dtype), oracle_forward(a, B))
    keep = (rows < 16) | (rows >= 32)
    a2 = gen.csr_from_coo(m, k, rows[keep], cols[keep], vals[keep])
    narrow = make_plan(hs, a2, dtype, "bcsr")
    assert np.array_equal(_run(narrow, B, dtype), oracle_forward(a2, B))
    ar = gen.csr_from_coo(m, k, rows, cols, g.standard_normal(rows.size))
    Br = g.standard_normal((k, n))
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    assert oracle.rel_err(_run(make_plan(hs, ar, dtype, "bcsr"), Br, dtype), oracle_forward(ar, Br)) <= tol


# ---------------------------------------------------------------------------
# the built format equals Alg. 1 replayed on the CPU
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("split", SPLITS)
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.float16])
def test_format_equals_alg1_replay(split, dtype):
    a = gen.random_csr(8, 150, 120, 0.1)
    a.vals[::7] = 0.0  # explicit zeros are stored entries
    plan = make_plan(hs, a, dtype, split)
    cls = plan.export("rb_class").astype(bool)
    ref = L.convert_assign_ref(a.m, a.row_ptr, a.col_idx, a.vals, cls, 16)
    for f in ("csr_rows", "csr_ptr", "csr_col", "bcsr_rb", "blk_ptr", "blk_col"):
        assert np.array_equal(plan.export(f), ref[f]), f
    nnz, nblk = L.rowblock_stats_ref(a.m, a.row_ptr, a.col_idx, 16)
    assert np.array_equal(plan.export("rb_nnz"), nnz)
    if split != "csr":
        assert np.array_equal(plan.export("rb_nblk"), nblk)
    if split == "boundary":
        r = plan.info()["r_boundary"]
        assert np.array_equal(cls, np.arange(cls.size) * 16 >= r)
    if dtype == torch.float64:
        assert np.array_equal(plan.export("csr_val"), ref["csr_val"])
        assert np.array_equal(plan.export("blk_val").reshape(-1, 16), ref["blk_val"])
    elif dtype == torch.float32:
        assert np.array_equal(plan.export("csr_val"), ref["csr_val"].astype(np.float32))
    else:
        # FP16 codes: the decision is an integer, taken in FP64 on both sides
        codes, s, _ = L.quantize_ref(a.m, a.row_ptr, a.vals, 16, "f16")
        assert np.array_equal(plan.export("rb_scale"), s)
        rows = np.repeat(np.arange(a.m), np.diff(a.row_ptr))
        mask_csr = ~cls[rows // 16]
        got = plan.export("csr_val").view(np.uint16)
        assert np.array_equal(got, codes[mask_csr])


@pytest.mark.parametrize("fmt,dtype", [("f16", torch.float16), ("bf16", torch.bfloat16)])
def test_quantisation_codes_bit_exact(fmt, dtype):
    """Values spanning many binades (incl. FP16 subnormals after scaling)
    get the same codes and scales as the CPU reference."""
    g = np.random.default_rng(9)
    a = gen.random_csr(9, 96, 80, 0.2)
    a.vals = g.standard_normal(a.nnz) * 2.0 ** g.integers(-30, 10, a.nnz)
    codes, s, _ = L.quantize_ref(a.m, a.row_ptr, a.vals, 16, fmt)
    plan = make_plan(hs, a, dtype, "csr")
    assert np.array_equal(plan.export("rb_scale"), s)
    assert np.array_equal(plan.export("csr_val").view(np.uint16), codes)
    plan = make_plan(hs, a, dtype, "bcsr")
    ref = L.convert_assign_ref(a.m, a.row_ptr, a.col_idx, codes.astype(np.float64),
                               np.ones((a.m + 15) // 16, bool), 16)
    assert np.array_equal(plan.export("blk_val").view(np.uint16).reshape(-1, 16).astype(np.float64),
                          ref["blk_val"])


# ---------------------------------------------------------------------------
# unsorted rows and duplicates
# ---------------------------------------------------------------------------
def _messy(seed, m=70, k=55, extra=60):
    g = np.random.default_rng(seed)
    a = gen.random_csr(seed, m, k, 0.12)
    r = np.concatenate([a.rows(), g.integers(0, m, extra)])
    c = np.concatenate([a.col_idx, g.integers(0, k, extra)])
    v = g.standard_normal(r.size)
    order = np.lexsort((g.random(r.size), r))  # rows grouped, columns shuffled
    r, c, v = r[order], c[order], v[order]
    rp = np.zeros(m + 1, np.int64)
    np.add.at(rp, r + 1, 1)
    return np.cumsum(rp).astype(np.int32), c.astype(np.int32), v, m, k


@pytest.mark.parametrize("split", SPLITS)
def test_unsorted_and_duplicates(split):
    rp, c, v, m, k = _messy(2)
    B = np.random.default_rng(0).standard_normal((k, 24))
    plan = hs.Plan(rp, c, to_dev(v), (m, k), compute=torch.float64, split=split, backward=True)
    info = plan.info()
    assert info["canonical_input"] == 0 and info["nnz"] < info["nnz_input"]
    C = _run(plan, B, torch.float64)
    assert oracle.rel_err(C, oracle.spmm(m, k, rp, c, v, B)) <= 1e-12
    G = np.random.default_rng(1).standard_normal((m, 24))
    dB, dA = plan.backward(to_dev(B), to_dev(G))
    torch.cuda.synchronize()
    assert oracle.rel_err(dB.cpu().numpy(), oracle.spmm_t(m, k, rp, c, v, G)) <= 1e-12
    assert oracle.rel_err(dA.cpu().numpy(), oracle.sddmm(m, k, rp, c, G, B)) <= 1e-12
    # canonical CSR equals the CPU canonical form
    ptr, col, val, _ = L.canonicalize_ref(m, k, rp, c, v)
    if split == "csr":
        assert np.array_equal(plan.export("csr_ptr"), ptr)
        assert np.array_equal(plan.export("csr_col"), col)


# ---------------------------------------------------------------------------
# determinism and value updates
# ---------------------------------------------------------------------------
def test_rerun_bitwise_identical_and_update_values():
    a, b = gen.config2(grid=32)
    plan = make_plan(hs, a, torch.float32, "auto", backward=True)
    C1 = _run(plan, b, torch.float32)
    C2 = _run(plan, b, torch.float32)
    assert np.array_equal(C1, C2)
    v2 = np.random.default_rng(5).standard_normal(a.nnz)
    plan.update_values(to_dev(v2))
    a2 = gen.Csr(a.m, a.k, a.row_ptr, a.col_idx, v2)
    assert oracle.rel_err(_run(plan, b, torch.float32), oracle_forward(a2, b)) <= 1e-5


@pytest.mark.parametrize("dtype", [torch.float64, torch.float16, torch.bfloat16])
@pytest.mark.parametrize("split", ["auto", "csr", "bcsr"])
def test_update_values_rescales(dtype, split):
    """New values of another magnitude through update_values: the per-row-
    block scales of FP16/BF16 are recomputed (values 1e4 times larger would
    overflow FP16 under the old scales) and C, dB and dA follow the new
    values."""
    a = gen.random_csr(14, 200, 180, 0.08)
    g = np.random.default_rng(12)
    B = g.standard_normal((a.k, 32))
    G = g.standard_normal((a.m, 32))
    plan = make_plan(hs, a, dtype, split, backward=True)
    v2 = g.standard_normal(a.nnz) * 1e4
    plan.update_values(to_dev(v2))
    a2 = gen.Csr(a.m, a.k, a.row_ptr, a.col_idx, v2)
    od = torch.float64 if dtype == torch.float64 else torch.float32
    C = _run(plan, B, dtype)
    dB, dA = plan.backward(to_dev(B, dtype), to_dev(G, od))
    torch.cuda.synchronize()
    assert np.isfinite(C).all()
    assert oracle.rel_err(C, oracle_forward(a2, B)) <= TOL[dtype]
    assert oracle.rel_err(dB.double().cpu().numpy(),
                          oracle.spmm_t(a.m, a.k, a.row_ptr, a.col_idx, v2, G)) <= TOL[dtype]
    # dA does not depend on the values
    assert oracle.rel_err(dA.double().cpu().numpy(), oracle.sddmm(a.m, a.k, a.row_ptr, a.col_idx, G, B)) <= TOL[dtype]


# ---------------------------------------------------------------------------
# config 2 (block stencil, FP32, N = 128) at full size
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("split", SPLITS)
def test_config2_fp32_full(split):
    print(f"config2 fp32 split={split}", flush=True)
    a, b = gen.config2()
    plan = make_plan(hs, a, torch.float32, split, backward=True)
    info = plan.info()
    if split == "bcsr":
        assert info["rb_bcsr"] == (a.m + 15) // 16
    C = _run(plan, b, torch.float32)
    assert oracle.rel_err(C, oracle_forward(a, b)) <= 1e-5
    G = gen.dense(0, gen.GRAD, a.m, b.shape[1])
    dB, dA = plan.backward(to_dev(b, torch.float32), to_dev(G, torch.float32))
    torch.cuda.synchronize()
    assert oracle.rel_err(dB.double().cpu().numpy(),
                          oracle.spmm_t(a.m, a.k, a.row_ptr, a.col_idx, a.vals, G)) <= 1e-5
    assert oracle.rel_err(dA.double().cpu().numpy(),
                          oracle.sddmm(a.m, a.k, a.row_ptr, a.col_idx, G, b)) <= 1e-5


# ---------------------------------------------------------------------------
# two plans on two streams at once (each plan on one stream at a time)
# ---------------------------------------------------------------------------
def test_two_plans_on_two_streams_bitwise():
    print("two plans, two streams", flush=True)
    a1, b1 = gen.config2(grid=32)                        # stencil, AUTO puts it in the BCSR-part
    a2 = gen.random_csr(5, 3000, 2500, 0.01)             # scattered, CSR-part
    b2 = gen.dense(5, gen.DENSE, a2.k, 48)
    g1 = gen.dense(1, gen.GRAD, a1.m, b1.shape[1])
    g2 = gen.dense(2, gen.GRAD, a2.m, b2.shape[1])
    p1 = make_plan(hs, a1, torch.float32, "auto", backward=True)
    p2 = make_plan(hs, a2, torch.float32, "auto", backward=True)
    B1, B2, G1, G2 = (to_dev(x, torch.float32) for x in (b1, b2, g1, g2))

    def both(p, B, G):
        C = p.run(B)
        dB, dA = p.backward(B, G)
        return C, dB, dA

    ref1, ref2 = both(p1, B1, G1), both(p2, B2, G2)
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    s1.wait_stream(torch.cuda.current_stream())
    s2.wait_stream(torch.cuda.current_stream())
    got1, got2 = [], []
    for _ in range(3):
        with torch.cuda.stream(s1):
            got1.append(both(p1, B1, G1))
        with torch.cuda.stream(s2):
            got2.append(both(p2, B2, G2))
    torch.cuda.synchronize()
    for ref, got in ((ref1, got1), (ref2, got2)):
        for outs in got:
            for r, g in zip(ref, outs):
                assert torch.equal(r, g)
    assert oracle.rel_err(ref1[0].double().cpu().numpy(), oracle_forward(a1, b1)) <= TOL[torch.float32]
    assert oracle.rel_err(ref2[0].double().cpu().numpy(), oracle_forward(a2, b2)) <= TOL[torch.float32]
