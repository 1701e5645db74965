"""Backward of the hybrid SpMM on the GPU: dB = A^T dC through the device-built
transposed plan and dA = SDDMM(dC, B) on A's pattern, against the FP64
oracle, central finite differences and torch.autograd.gradcheck."""
import numpy as np
import pytest
import torch

import gen
import oracle
from tests.gpu_util import SPLITS, TOL, effective_vals, make_plan, quantized_dense, rounded_slabs, to_dev

pytestmark = pytest.mark.gpu

hs = pytest.importorskip("paper_2511_08158_amd")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.float16, torch.bfloat16])
@pytest.mark.parametrize("split", SPLITS)
def test_backward_vs_oracle(dtype, split):
    """dB and dA against the oracle; for FP16/BF16 the gradient is that of the
    computed product (stored, quantised A; B as given), in FP32."""
    print(f"backward dtype={dtype} split={split}", flush=True)
    a = gen.random_csr(21, 301, 257, 0.06)
    n = 72
    g = np.random.default_rng(2)
    B = g.standard_normal((a.k, n))
    G = g.standard_normal((a.m, n))
    plan = make_plan(hs, a, dtype, split, backward=True)
    od = torch.float64 if dtype == torch.float64 else torch.float32
    dB, dA = plan.backward(to_dev(B, dtype), to_dev(G, od))
    torch.cuda.synchronize()
    Aq = effective_vals(a.m, a.row_ptr, a.vals, dtype)
    Bq = quantized_dense(B, dtype)
    Gq = G.astype(np.float32).astype(np.float64) if od == torch.float32 else G
    ref_db = oracle.spmm_t(a.m, a.k, a.row_ptr, a.col_idx, Aq, Gq)
    # FP16/BF16: the BCSR-part's SDDMM multiplies dC rounded to the compute
    # type (each 16-row slab after its power-of-two scale) on matrix cores
    half = dtype in (torch.float16, torch.bfloat16)
    Gd = rounded_slabs(Gq, plan.export("bcsr_rb"), dtype) if half else Gq
    ref_da = oracle.sddmm(a.m, a.k, a.row_ptr, a.col_idx, Gd, Bq)
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    assert oracle.rel_err(dB.double().cpu().numpy(), ref_db) <= tol
    assert oracle.rel_err(dA.double().cpu().numpy(), ref_da) <= tol
    # end-to-end against the unquantised problem
    assert oracle.rel_err(dB.double().cpu().numpy(),
                          oracle.spmm_t(a.m, a.k, a.row_ptr, a.col_idx, a.vals, G)) <= TOL[dtype]
    assert oracle.rel_err(dA.double().cpu().numpy(),
                          oracle.sddmm(a.m, a.k, a.row_ptr, a.col_idx, G, B)) <= TOL[dtype]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.float16, torch.bfloat16])
@pytest.mark.parametrize("n", [5, 40, 200, 300, 1024])
@pytest.mark.parametrize("split", ["bcsr", "csr"])
def test_sddmm_forms_by_width(dtype, n, split):
    """Every form of the SDDMM against the oracle on the inputs as the
    kernels read them: one column per lane (n = 5), the dC slab held in LDS
    (n = 40), the FP16/BF16 matrix-core form up to n = 256, dC read from global
    memory per step (n = 200, 300 and 1024 for the FP32-MFMA forms) and CSR
    lane groups that loop over several column panels (n = 300, 1024)."""
    print(f"sddmm forms dtype={dtype} n={n} split={split}", flush=True)
    a = gen.random_csr(31, 150, 170, 0.09)
    g = np.random.default_rng(8)
    B = g.standard_normal((a.k, n))
    G = g.standard_normal((a.m, n))
    plan = make_plan(hs, a, dtype, split, backward=True)
    od = torch.float64 if dtype == torch.float64 else torch.float32
    dB, dA = plan.backward(to_dev(B, dtype), to_dev(G, od))
    torch.cuda.synchronize()
    Bq = quantized_dense(B, dtype)
    Gq = G.astype(np.float32).astype(np.float64) if od == torch.float32 else G
    if dtype in (torch.float16, torch.bfloat16) and split == "bcsr" and n % 8 == 0 and n <= 256:
        Gq = rounded_slabs(Gq, plan.export("bcsr_rb"), dtype)
    ref = oracle.sddmm(a.m, a.k, a.row_ptr, a.col_idx, Gq, Bq)
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    assert oracle.rel_err(dA.double().cpu().numpy(), ref) <= tol
    assert oracle.rel_err(dA.double().cpu().numpy(), oracle.sddmm(a.m, a.k, a.row_ptr, a.col_idx, G, B)) <= TOL[dtype]


@pytest.mark.parametrize("split", SPLITS)
def test_backward_integer_bitwise(split):
    a = gen.random_csr(3, 190, 170, 0.07, dist="int")
    g = np.random.default_rng(0)
    B = g.integers(-3, 4, (a.k, 40)).astype(float)
    G = g.integers(-3, 4, (a.m, 40)).astype(float)
    plan = make_plan(hs, a, torch.float32, split, backward=True)
    dB, dA = plan.backward(to_dev(B, torch.float32), to_dev(G, torch.float32))
    torch.cuda.synchronize()
    assert np.array_equal(dB.double().cpu().numpy(), oracle.spmm_t(a.m, a.k, a.row_ptr, a.col_idx, a.vals, G))
    assert np.array_equal(dA.double().cpu().numpy(), oracle.sddmm(a.m, a.k, a.row_ptr, a.col_idx, G, B))


@pytest.mark.parametrize("split", SPLITS)
def test_concurrent_backward_equals_sequential(split, monkeypatch):
    """With HSPMM_BWD_CONCURRENT=1 the SDDMM runs on the plan's side stream
    beside dB; both gradients are bitwise those of the sequential backward,
    on two calls in a row (the side stream and its events are reused)."""
    print(f"concurrent backward split={split}", flush=True)
    a = gen.random_csr(5, 700, 650, 0.03)
    g = np.random.default_rng(8)
    B = to_dev(g.standard_normal((a.k, 48)), torch.float32)
    G = to_dev(g.standard_normal((a.m, 48)), torch.float32)
    plan = make_plan(hs, a, torch.float32, split, backward=True)
    monkeypatch.delenv("HSPMM_BWD_CONCURRENT", raising=False)
    ref = [t.cpu().numpy() for t in plan.backward(B, G)]
    monkeypatch.setenv("HSPMM_BWD_CONCURRENT", "1")
    for _ in range(2):
        got = [t.cpu().numpy() for t in plan.backward(B, G)]
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
    assert oracle.rel_err(ref[1], oracle.sddmm(a.m, a.k, a.row_ptr, a.col_idx,
                                               G.double().cpu().numpy(), B.double().cpu().numpy())) <= 1e-5


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.float16, torch.bfloat16])
def test_sddmm_wide_row_blocks(dtype):
    """Row blocks with thousands of tiles (many rounds of 64 tiles per wave),
    a ragged last row block, empty rows and unsorted duplicated input: the
    BCSR-part's destinations (ranks from the tile occupancy masks) against
    the oracle, and dA bitwise equal between the BCSR-only and CSR-only
    plans in FP64 with integer values."""
    print(f"sddmm wide row blocks dtype={dtype}", flush=True)
    g = np.random.default_rng(17)
    m, k, n = 45, 6000, 32
    dens = np.where(np.arange(m) % 7 == 3, 0.0, g.uniform(0.02, 0.4, m))
    rows, cols = [], []
    for i in range(m):
        c = np.flatnonzero(g.random(k) < dens[i])
        rows.append(np.full(c.size, i)); cols.append(c)
    rows = np.concatenate(rows); cols = np.concatenate(cols)
    dup = g.choice(rows.size, 50, replace=False)
    rows = np.concatenate([rows, rows[dup]]); cols = np.concatenate([cols, cols[dup]])
    perm = g.permutation(rows.size)
    rows, cols = rows[perm], cols[perm]
    order = np.argsort(rows, kind="stable")
    rows, cols = rows[order], cols[order]          # rows grouped, columns unsorted
    row_ptr = np.concatenate([[0], np.cumsum(np.bincount(rows, minlength=m))]).astype(np.int32)
    vals = g.integers(-3, 4, rows.size).astype(float)
    a = gen.Csr(m, k, row_ptr, cols.astype(np.int32), vals)
    B = g.integers(-3, 4, (k, n)).astype(float)
    G = g.integers(-3, 4, (m, n)).astype(float)
    od = torch.float64 if dtype == torch.float64 else torch.float32
    plan = make_plan(hs, a, dtype, "bcsr")
    assert plan.info()["nblk"] > 4 * 64 * 4
    _, dA = plan.backward(to_dev(B, dtype), to_dev(G, od), need_dB=False, need_dA=True)
    torch.cuda.synchronize()
    ref = oracle.sddmm(a.m, a.k, a.row_ptr, a.col_idx, G, B)
    assert np.array_equal(dA.double().cpu().numpy(), ref)
    if dtype == torch.float64:
        plan_c = make_plan(hs, a, dtype, "csr")
        _, dA_c = plan_c.backward(to_dev(B, dtype), to_dev(G, od), need_dB=False, need_dA=True)
        assert np.array_equal(dA_c.cpu().numpy(), dA.cpu().numpy())


def test_transposed_format_equals_cpu_transpose():
    from oracle import loops_ref as L
    a = gen.random_csr(4, 120, 90, 0.1)
    plan = make_plan(hs, a, torch.float32, "csr", backward=True)
    ptr, col, val, perm = L.transpose_ref(a.m, a.k, a.row_ptr, a.col_idx, a.vals)
    assert np.array_equal(plan.export("csr_ptr", which=1), ptr)
    assert np.array_equal(plan.export("csr_col", which=1), col)
    assert np.array_equal(plan.export("csr_val", which=1), val.astype(np.float32))


def test_backward_without_transposed_plan_is_an_error():
    a = gen.random_csr(1, 40, 40, 0.1)
    plan = make_plan(hs, a, torch.float32, "auto", backward=False)
    B = to_dev(np.ones((40, 4)), torch.float32)
    with pytest.raises(hs.HspmmError) as e:
        plan.backward(B, to_dev(np.ones((40, 4)), torch.float32), need_dB=True, need_dA=False)
    assert e.value.code == -4
    # dA alone needs no transposed plan
    _, dA = plan.backward(B, to_dev(np.ones((40, 4)), torch.float32), need_dB=False, need_dA=True)
    torch.cuda.synchronize()
    assert dA.shape[0] == a.nnz


def test_gradcheck_tiny_fp64():
    a = gen.random_csr(7, 18, 14, 0.3)
    dev = torch.device("cuda:0")
    vals = torch.tensor(a.vals, device=dev, requires_grad=True)
    B = torch.tensor(np.random.default_rng(1).standard_normal((a.k, 5)), device=dev, requires_grad=True)
    for split in SPLITS:
        plan = hs.Plan(a.row_ptr, a.col_idx, vals.detach(), (a.m, a.k), compute=torch.float64, split=split,
                       backward=True)
        assert torch.autograd.gradcheck(lambda v, b: hs.spmm(plan, v, b), (vals, B), eps=1e-6, atol=1e-9)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float16, torch.bfloat16])
def test_autograd_low_precision(dtype):
    """spmm's autograd function in FP32/FP16/BF16 with learnable values:
    every forward re-packs the values (quantised per row block for
    FP16/BF16); the gradients of vals and B match the products the library
    computes directly, and both match the oracle within the precision's
    tolerance."""
    a = gen.random_csr(8, 150, 140, 0.07)
    dev = torch.device("cuda:0")
    g = np.random.default_rng(9)
    vals = torch.tensor(a.vals, device=dev, dtype=torch.float32, requires_grad=True)
    Bn = g.standard_normal((a.k, 24))
    Gn = g.standard_normal((a.m, 24))
    B = to_dev(Bn, dtype).requires_grad_(True)
    plan = hs.Plan(a.row_ptr, a.col_idx, vals.detach(), (a.m, a.k), compute=dtype, split="auto", backward=True)
    for step in range(2):
        C = hs.spmm(plan, vals, B)
        C.backward(to_dev(Gn, torch.float32))
        torch.cuda.synchronize()
        dB_ref, dA_ref = plan.backward(B.detach(), to_dev(Gn, torch.float32))
        torch.cuda.synchronize()
        assert torch.equal(B.grad.float(), dB_ref.to(B.dtype).float())
        assert torch.equal(vals.grad, dA_ref.to(vals.dtype))
        assert oracle.rel_err(vals.grad.double().cpu().numpy(),
                              oracle.sddmm(a.m, a.k, a.row_ptr, a.col_idx, Gn, Bn)) <= TOL[dtype]
        with torch.no_grad():
            vals.mul_(2.0)   # a new version of the values: the next forward re-packs them
        vals.grad = None
        B.grad = None
    assert oracle.rel_err(C.detach().double().cpu().numpy(),
                          oracle.spmm(a.m, a.k, a.row_ptr, a.col_idx, a.vals * 2.0, Bn)) <= TOL[dtype]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("split", SPLITS)
@pytest.mark.parametrize("n", [64, 128])
def test_gcn_subgraph_parity(dtype, split, n):
    """The FD subgraph (dense-ish BFS ball, one 497-entry row) through every
    split: forward and both gradients against the oracle."""
    full, _ = gen.config4()
    sub = gen.config4_fd_subgraph(full, 512)
    g = np.random.default_rng(11)
    X = g.standard_normal((sub.k, n))
    G = g.standard_normal((sub.m, n))
    plan = make_plan(hs, sub, dtype, split, backward=True)
    od = torch.float64 if dtype == torch.float64 else torch.float32
    C = plan.run(to_dev(X, dtype))
    dX, dA = plan.backward(to_dev(X, dtype), to_dev(G, od))
    torch.cuda.synchronize()
    e = (oracle.rel_err(C.double().cpu().numpy(), oracle.spmm(sub.m, sub.k, sub.row_ptr, sub.col_idx, sub.vals, X)),
         oracle.rel_err(dX.double().cpu().numpy(), oracle.spmm_t(sub.m, sub.k, sub.row_ptr, sub.col_idx, sub.vals, G)),
         oracle.rel_err(dA.double().cpu().numpy(), oracle.sddmm(sub.m, sub.k, sub.row_ptr, sub.col_idx, G, X)))
    print(f"subgraph {dtype} {split} n={n}: C {e[0]:.2e} dX {e[1]:.2e} dA {e[2]:.2e} info {plan.info()}", flush=True)
    assert max(e) <= TOL[dtype]


def test_finite_differences_gcn_subgraph():
    """Central differences (eps 1e-3, FP64) on the 512-node BFS subgraph of
    the GCN graph.  L = <A(vals) X, G> is linear in X and in vals, so the
    differences are exact up to rounding."""
    full, _ = gen.config4()
    sub = gen.config4_fd_subgraph(full, 512)
    dev = torch.device("cuda:0")
    g = np.random.default_rng(11)
    X = g.standard_normal((sub.k, 128))
    G = g.standard_normal((sub.m, 128))
    plan = hs.Plan(sub.row_ptr, sub.col_idx, to_dev(sub.vals), (sub.m, sub.k), compute=torch.float64,
                   split="auto", backward=True)
    Xd, Gd = to_dev(X), to_dev(G)
    dX, dA = plan.backward(Xd, Gd)

    def loss(vals=None, Xv=None):
        # every evaluation sets the values it needs (A itself unless perturbed)
        plan.update_values(to_dev(sub.vals if vals is None else vals))
        C = plan.run(Xd if Xv is None else Xv)
        return float((C * Gd).sum())

    eps = 1e-3
    tol = 1e-8
    # 8 random directions over all coordinates
    for d in range(8):
        D = torch.tensor(g.standard_normal(X.shape), device=dev)
        fd = (loss(Xv=Xd + eps * D) - loss(Xv=Xd - eps * D)) / (2 * eps)
        an = float((dX * D).sum())
        assert abs(fd - an) <= tol * max(1.0, abs(an))
        dv = g.standard_normal(sub.nnz)
        fd = (loss(vals=sub.vals + eps * dv) - loss(vals=sub.vals - eps * dv)) / (2 * eps)
        an = float(np.dot(dA.cpu().numpy(), dv))
        assert abs(fd - an) <= tol * max(1.0, abs(an))
    plan.update_values(to_dev(sub.vals))
    # 64 seeded single entries each
    for e in g.choice(sub.nnz, 64, replace=False):
        dv = np.zeros(sub.nnz)
        dv[e] = 1.0
        fd = (loss(vals=sub.vals + eps * dv) - loss(vals=sub.vals - eps * dv)) / (2 * eps)
        assert abs(fd - float(dA[e])) <= tol * max(1.0, abs(fd))
    plan.update_values(to_dev(sub.vals))
    for idx in g.choice(X.size, 64, replace=False):
        i, j = divmod(int(idx), X.shape[1])
        D = torch.zeros_like(Xd)
        D[i, j] = 1.0
        fd = (loss(Xv=Xd + eps * D) - loss(Xv=Xd - eps * D)) / (2 * eps)
        assert abs(fd - float(dX[i, j])) <= tol * max(1.0, abs(fd))
    # and the gradient agrees with the oracle
    ref_dx = oracle.spmm_t(sub.m, sub.k, sub.row_ptr, sub.col_idx, sub.vals, G)
    assert oracle.rel_err(dX.cpu().numpy(), ref_dx) <= 1e-12


def test_autograd_training_step_gcn_layer():
    """spmm inside a tiny two-layer graph network: gradients of a dense
    weight through the SpMM match the same network evaluated with the
    oracle's products on the CPU."""
    a = gen.random_csr(13, 257, 257, 0.03)
    dev = torch.device("cuda:0")
    g = np.random.default_rng(3)
    X = torch.tensor(g.standard_normal((257, 16)), device=dev)
    W = torch.tensor(g.standard_normal((16, 8)), device=dev, requires_grad=True)
    plan = hs.Plan(a.row_ptr, a.col_idx, to_dev(a.vals), (a.m, a.k), compute=torch.float64, backward=True)
    vals = to_dev(a.vals)
    H = torch.relu(hs.spmm(plan, vals, X @ W))
    loss = (H ** 2).sum()
    loss.backward()
    # CPU reference with dense matrices
    Ad = torch.tensor(a.to_scipy().toarray())
    Wc = W.detach().cpu().clone().requires_grad_(True)
    Hc = torch.relu(Ad @ (X.cpu() @ Wc))
    (Hc ** 2).sum().backward()
    assert torch.allclose(W.grad.cpu(), Wc.grad, rtol=1e-11, atol=1e-11)
