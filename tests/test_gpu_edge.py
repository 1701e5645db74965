"""Edge cases on the GPU: empty row blocks in the FP16/BF16 matrix-core
forms, the Eq. 1 boundary the library solves against the oracle's Eq. 1, the
FP16/BF16 SDDMM on a dC slab far below FP16's range, the autograd function
with several forward calls on one plan, the binding's operand checks, row
pointers across long stretches of empty rows, and the backward of a matrix
without entries and at n = 0."""
import gc

import numpy as np
import pytest
import torch

import gen
import oracle
from oracle import loops_ref as L
from tests.gpu_util import TOL, effective_vals, make_plan, quantized_dense, rounded_slabs, to_dev

pytestmark = pytest.mark.gpu

hs = pytest.importorskip("paper_2511_08158_amd")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _with_empty_row_blocks(seed, m=40, k=70):
    """Rows 0..15 hold entries, rows 16..39 none: row block 1 is empty and
    row block 2 (rows 32..39, the ragged last one) is empty too."""
    g = np.random.default_rng(seed)
    rows = np.repeat(np.arange(16), 9)
    cols = np.concatenate([np.sort(g.choice(k, 9, replace=False)) for _ in range(16)])
    return gen.csr_from_coo(m, k, rows, cols, g.standard_normal(rows.size))


@pytest.mark.parametrize("dtype", [torch.float16, torch.bfloat16, torch.float32, torch.float64])
@pytest.mark.parametrize("split,rb", [("bcsr", -1), ("boundary", 0), ("boundary", 16)])
@pytest.mark.parametrize("n", [8, 64, 136])
def test_trailing_empty_row_block(dtype, split, rb, n):
    """Forced splits put empty row blocks in the BCSR-part; when the last
    BCSR row block is empty its tile range starts at the end of the value
    array.  C, dB and dA still equal the oracle, and the empty rows are 0."""
    print(f"empty trailing row block dtype={dtype} split={split} r={rb} n={n}", flush=True)
    a = _with_empty_row_blocks(3)
    kw = {"r_boundary": rb} if split == "boundary" else {}
    plan = make_plan(hs, a, dtype, split, backward=True, **kw)
    info = plan.info()
    assert info["rb_bcsr"] == (3 if rb <= 0 else 2)
    g = np.random.default_rng(n)
    B = g.standard_normal((a.k, n))
    G = g.standard_normal((a.m, n))
    od = torch.float64 if dtype == torch.float64 else torch.float32
    C = plan.run(to_dev(B, dtype))
    dB, dA = plan.backward(to_dev(B, dtype), to_dev(G, od))
    torch.cuda.synchronize()
    C = C.double().cpu().numpy()
    assert np.all(C[16:] == 0.0)
    assert oracle.rel_err(C, oracle.spmm(a.m, a.k, a.row_ptr, a.col_idx, a.vals, B)) <= TOL[dtype]
    assert oracle.rel_err(dB.double().cpu().numpy(),
                          oracle.spmm_t(a.m, a.k, a.row_ptr, a.col_idx, a.vals, G)) <= TOL[dtype]
    assert oracle.rel_err(dA.double().cpu().numpy(),
                          oracle.sddmm(a.m, a.k, a.row_ptr, a.col_idx, G, B)) <= TOL[dtype]


@pytest.mark.parametrize("n_hint", [16, 128])
def test_eq1_boundary_matches_oracle(n_hint):
    """BOUNDARY with r_boundary < 0 solves Eq. 1 with each part's aggregate
    throughput TP = m / (predicted time of the whole matrix in that part):
    the boundary equals the oracle's Eq. 1 on the same predicted times, lies
    strictly inside the matrix for this input, and the row-block classes
    follow it."""
    a = gen.random_csr(41, 400, 300, 0.05)
    plan = make_plan(hs, a, torch.float32, "boundary", r_boundary=-1, n_hint=n_hint)
    info = plan.info()
    tc, tb = info["pred_us_csr_all"], info["pred_us_bcsr_all"]
    assert tc > 0 and tb > 0
    want = L.eq1_boundary(a.m, a.m / tc, 1.0, a.m / tb, 1.0, 16)
    assert info["r_boundary"] == want
    assert 0 < want < a.m
    cls = plan.export("rb_class").astype(bool)
    assert np.array_equal(cls, np.arange(cls.size) * 16 >= want)
    assert info["rows_csr"] == want


@pytest.mark.parametrize("dtype", [torch.float16, torch.bfloat16])
def test_sddmm_tiny_dC_slab(dtype):
    """A 16-row slab of dC near 1e-36 (below 2^-112): the FP16/BF16 matrix-
    core SDDMM scales it by 2^126 at most, so its dA stays finite and, row
    block by row block, within the tolerance of the oracle; the other slabs
    are unaffected."""
    a = gen.random_csr(17, 64, 90, 0.12)
    g = np.random.default_rng(5)
    n = 64
    B = g.standard_normal((a.k, n))
    G = g.standard_normal((a.m, n))
    G[16:32] *= 1e-36
    plan = make_plan(hs, a, dtype, "bcsr", backward=True)
    _, dA = plan.backward(to_dev(B, dtype), to_dev(G, torch.float32), need_dB=False)
    torch.cuda.synchronize()
    dA = dA.double().cpu().numpy()
    assert np.isfinite(dA).all()
    ref = oracle.sddmm(a.m, a.k, a.row_ptr, a.col_idx, G, B)
    rows = np.repeat(np.arange(a.m), np.diff(a.row_ptr))
    for q in range(4):
        sel = rows // 16 == q
        assert oracle.rel_err(dA[sel], ref[sel]) <= TOL[dtype], q
    # against the inputs as the kernel reads them (B rounded, dC slabs
    # scaled and rounded)
    Gq = rounded_slabs(G.astype(np.float32).astype(np.float64), plan.export("bcsr_rb"), dtype)
    refk = oracle.sddmm(a.m, a.k, a.row_ptr, a.col_idx, Gq, quantized_dense(B, dtype))
    sel = rows // 16 == 1
    assert oracle.rel_err(dA[sel], refk[sel]) <= 1e-5


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.float16])
def test_autograd_two_forward_calls_one_backward(dtype):
    """Two forward calls on one plan with different learnable values, then
    one backward: each call's gradients are those of its own values (the
    plan is re-packed from the values saved by the call being
    differentiated)."""
    a = gen.random_csr(7, 180, 150, 0.06)
    g = np.random.default_rng(9)
    n = 24
    v1 = g.standard_normal(a.nnz)
    v2 = g.standard_normal(a.nnz) * 3.0
    B1, B2 = g.standard_normal((a.k, n)), g.standard_normal((a.k, n))
    G1, G2 = g.standard_normal((a.m, n)), g.standard_normal((a.m, n))
    plan = make_plan(hs, a, dtype, "auto", backward=True)
    od = torch.float64 if dtype == torch.float64 else torch.float32
    t1 = to_dev(v1, torch.float64).requires_grad_(True)
    t2 = to_dev(v2, torch.float64).requires_grad_(True)
    X1 = to_dev(B1, dtype).requires_grad_(True)
    X2 = to_dev(B2, dtype).requires_grad_(True)
    C1 = hs.spmm(plan, t1, X1)
    C2 = hs.spmm(plan, t2, X2)
    loss = (C1 * to_dev(G1, od)).sum() + (C2 * to_dev(G2, od)).sum()
    loss.backward()
    torch.cuda.synchronize()
    # dB is returned in B's dtype (FP16 for the FP16 plan: rounded once more)
    tol_db = {torch.float64: 1e-12, torch.float32: 1e-5, torch.float16: 5e-3}[dtype]
    for v, X, G, Bn, t in ((v1, X1, G1, B1, t1), (v2, X2, G2, B2, t2)):
        Aq = effective_vals(a.m, a.row_ptr, v, dtype)
        ref_db = oracle.spmm_t(a.m, a.k, a.row_ptr, a.col_idx, Aq, G)
        assert oracle.rel_err(X.grad.double().cpu().numpy(), ref_db) <= tol_db
        ref_da = oracle.sddmm(a.m, a.k, a.row_ptr, a.col_idx, G, Bn)
        assert oracle.rel_err(t.grad.double().cpu().numpy(), ref_da) <= TOL[dtype]


def test_autograd_new_values_tensor_at_a_reused_address():
    """A static (not learnable) value tensor replaced by a new one: the new
    tensor is packed even when the caching allocator hands it the freed
    tensor's address at version 0."""
    a = gen.random_csr(8, 120, 100, 0.08)
    g = np.random.default_rng(2)
    B = g.standard_normal((a.k, 16))
    plan = make_plan(hs, a, torch.float32, "auto")
    X = to_dev(B, torch.float32)
    for trial in range(4):
        v = g.standard_normal(a.nnz)
        t = to_dev(v, torch.float64)
        C = hs.spmm(plan, t, X)
        torch.cuda.synchronize()
        ref = oracle.spmm(a.m, a.k, a.row_ptr, a.col_idx, v, B)
        assert oracle.rel_err(C.double().cpu().numpy(), ref) <= 1e-5, trial
        del t, C
        gc.collect()


def test_binding_rejects_bad_operands():
    """run(out=...) and backward(dC) reject operands of the wrong device,
    dtype, shape or layout before anything reaches the C ABI; the plan keeps
    working afterwards."""
    a = gen.random_csr(4, 60, 50, 0.1)
    plan = make_plan(hs, a, torch.float32, "auto", backward=True)
    B = to_dev(np.ones((a.k, 8)), torch.float32)
    d = B.device
    bad_out = [torch.empty((a.m, 8)),                                   # host memory
               torch.empty((a.m, 8), dtype=torch.float64, device=d),    # dtype
               torch.empty((a.m, 7), device=d),                         # columns
               torch.empty((a.m + 1, 8), device=d),                     # rows
               torch.empty((8, a.m), device=d).t()]                     # column-major
    for o in bad_out:
        with pytest.raises(hs.HspmmError):
            plan.run(B, out=o)
    G = torch.ones((a.m, 8), device=d)
    for dC in (G.cpu(), G.double(), G[:, :7], G[:-1], torch.ones((8, a.m), device=d).t()):
        with pytest.raises(hs.HspmmError):
            plan.backward(B, dC)
    C = plan.run(B)
    torch.cuda.synchronize()
    ref = oracle.spmm(a.m, a.k, a.row_ptr, a.col_idx, a.vals, np.ones((a.k, 8)))
    assert oracle.rel_err(C.double().cpu().numpy(), ref) <= 1e-5


def test_timing_events_bracket_the_kernels():
    """hybrid_spmm_set_timing_events: the products record the given events
    from their kernels' own timestamps -- positive durations that add up to
    no more than the step bracketed by ordinary events -- the results are
    unchanged, and clearing the events leaves later products untimed."""
    a, b = gen.config2(grid=32)
    g = gen.dense(0, gen.GRAD, a.m, b.shape[1])
    plan = make_plan(hs, a, torch.float32, "auto", backward=True)
    B = to_dev(b, torch.float32)
    dC = to_dev(g, torch.float32)
    ref = plan.run(B)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(8)]
    for e in ev:
        e.record()
    torch.cuda.synchronize()
    ev[6].record()
    hs.set_timing_events(ev[0], ev[1])
    C = plan.run(B)
    hs.set_timing_events(ev[2], ev[3])
    dB, _ = plan.backward(B, dC, need_dA=False)
    hs.set_timing_events(ev[4], ev[5])
    _, dA = plan.backward(B, dC, need_dB=False)
    hs.set_timing_events()
    ev[7].record()
    C2 = plan.run(B)
    torch.cuda.synchronize()
    ks = [ev[2 * i].elapsed_time(ev[2 * i + 1]) for i in range(3)]
    assert all(t > 0 for t in ks), ks
    assert sum(ks) <= ev[6].elapsed_time(ev[7]) + 1e-3
    assert torch.equal(C, ref) and torch.equal(C2, ref)
    assert oracle.rel_err(dB.double().cpu().numpy(),
                          oracle.spmm_t(a.m, a.k, a.row_ptr, a.col_idx, a.vals, g)) <= 1e-5
    assert oracle.rel_err(dA.double().cpu().numpy(), oracle.sddmm(a.m, a.k, a.row_ptr, a.col_idx, g, b)) <= 1e-5


@pytest.mark.parametrize("dtype", [torch.float32, torch.float16])
def test_eq1_boundary_from_measured_throughputs(dtype):
    """BOUNDARY with r_boundary = HSPMM_R_MEASURED: the plan times the
    forward of the whole matrix in the CSR-part and in the BCSR-part and
    solves Eq. 1 with TP = m / time; the boundary equals the oracle's Eq. 1
    on the times the plan reports, the row blocks follow it, and the product
    is the oracle's."""
    from paper_2511_08158_amd import _lib
    a, b = gen.config2(grid=32)
    plan = make_plan(hs, a, dtype, "boundary", backward=True, r_boundary=_lib.R_MEASURED, n_hint=64)
    info = plan.info()
    tc, tb = info["meas_us_csr_all"], info["meas_us_bcsr_all"]
    print(f"measured whole-matrix forward: CSR-part {tc:.1f} us, BCSR-part {tb:.1f} us, "
          f"r_boundary {info['r_boundary']} of {a.m}", flush=True)
    assert tc > 0 and tb > 0
    want = L.eq1_boundary(a.m, a.m / tc, 1.0, a.m / tb, 1.0, 16)
    assert info["r_boundary"] == want
    cls = plan.export("rb_class").astype(bool)
    assert np.array_equal(cls, np.arange(cls.size) * 16 >= want)
    C = plan.run(to_dev(b, dtype))
    torch.cuda.synchronize()
    assert oracle.rel_err(C.double().cpu().numpy(),
                          oracle.spmm(a.m, a.k, a.row_ptr, a.col_idx, a.vals, b)) <= TOL[dtype]


@pytest.mark.parametrize("split", ["auto", "csr", "bcsr"])
def test_long_stretches_of_empty_rows(split):
    """Entries in the first and last rows only, in 12 of 60,000 columns:
    A's row pointer and A^T's have tens of thousands of empty rows in a
    row, at the start, in the middle and at the end of the key lists.
    Forward, dB and dA against the oracle."""
    print(f"empty stretches split={split}", flush=True)
    g = np.random.default_rng(31)
    m, k, n = 5000, 60000, 64
    cols = np.array([0, 1, 2, 3, 17, 18, 30000, 30001, 59990, 59995, 59998, 59999])
    r = np.concatenate([np.zeros(cols.size, np.int64), np.full(cols.size, m - 1)])
    c = np.concatenate([cols, cols])
    a = gen.csr_from_coo(m, k, r, c, g.standard_normal(r.size))
    plan = make_plan(hs, a, torch.float32, split, backward=True)
    B = g.standard_normal((k, n))
    G = g.standard_normal((m, n))
    Bd, Gd = to_dev(B, torch.float32), to_dev(G, torch.float32)
    C = plan.run(Bd)
    dB, dA = plan.backward(Bd, Gd)
    torch.cuda.synchronize()
    assert oracle.rel_err(C.double().cpu().numpy(), oracle.spmm(a.m, a.k, a.row_ptr, a.col_idx, a.vals, B)) <= TOL[torch.float32]
    assert oracle.rel_err(dB.double().cpu().numpy(),
                          oracle.spmm_t(a.m, a.k, a.row_ptr, a.col_idx, a.vals, G)) <= TOL[torch.float32]
    assert oracle.rel_err(dA.double().cpu().numpy(), oracle.sddmm(a.m, a.k, a.row_ptr, a.col_idx, G, B)) <= TOL[torch.float32]
    # the rows of C and dB without entries are exactly zero
    Ch, dBh = C.cpu().numpy(), dB.cpu().numpy()
    assert not Ch[1:m - 1].any()
    keep = np.ones(k, bool)
    keep[cols] = False
    assert not dBh[keep].any()


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_backward_degenerate_shapes(dtype):
    """A matrix without entries: C and dB are all zeros (written, not left
    as they were), dA is empty.  n = 0: C and dB are empty and every dA
    entry is the empty dot product, 0."""
    print(f"degenerate backward dtype={dtype}", flush=True)
    od = torch.float64 if dtype == torch.float64 else torch.float32
    z = gen.csr_from_coo(40, 30, np.zeros(0, int), np.zeros(0, int))
    plan = make_plan(hs, z, dtype, "auto", backward=True)
    g = np.random.default_rng(5)
    Bd = to_dev(g.standard_normal((30, 8)), dtype)
    Gd = to_dev(g.standard_normal((40, 8)), od)
    C = torch.full((40, 8), 7.0, dtype=od, device=Bd.device)
    plan.run(Bd, out=C)
    dB, dA = plan.backward(Bd, Gd)
    torch.cuda.synchronize()
    assert not C.cpu().numpy().any()
    assert dB.shape == (30, 8) and not dB.cpu().numpy().any()
    assert dA.numel() == 0
    a = gen.random_csr(6, 70, 50, 0.1)
    plan = make_plan(hs, a, dtype, "auto", backward=True)
    B0 = torch.zeros((50, 0), dtype=dtype, device=Bd.device)
    G0 = torch.zeros((70, 0), dtype=od, device=Bd.device)
    C0 = plan.run(B0)
    dB0, dA0 = plan.backward(B0, G0)
    torch.cuda.synchronize()
    assert C0.shape == (70, 0) and dB0.shape == (50, 0)
    assert dA0.shape == (a.nnz,) and not dA0.cpu().numpy().any()
