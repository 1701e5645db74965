"""Groups of BCSR row blocks that share columns (the LDS-staged group
kernels of the FP32 / FP64 forward and of dB = A^T dC; off by default,
HSPMM_GROUPS=1 forces them on, -1 lets the plan decide).

The grouping itself is a performance choice: any partition of the row
blocks gives the same product.  What is pinned exactly is the stage each
group loads and where each tile reads its B row: the staged columns of a
group are every column its tiles use, in ascending order (or none, for a
row block with more columns than the stage holds), and a tile reads stage
row `index of its column` when staged and column `-(bsrc + 1)`
otherwise.  The products are checked against the
oracle and, bit for bit, against the ungrouped kernels (the same MFMA
steps in the same order; only where the B operand comes from differs)."""
import numpy as np
import pytest
import torch

import gen
import oracle
from tests.gpu_util import ROW_TOL, TOL, abs_forward, make_plan, scaled_row_errors, to_dev

pytestmark = pytest.mark.gpu

hs = pytest.importorskip("paper_2511_08158_amd")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def check_group_format(plan, which=0):
    """The exported groups against their definition, from the canonical
    tile lists of the plan (integers, exact)."""
    rb = plan.export("bcsr_rb", which)
    bptr = plan.export("blk_ptr", which)
    bcol = plan.export("blk_col", which)
    gptr = plan.export("grp_ptr", which)
    grb = plan.export("grp_rb", which)
    uptr = plan.export("grp_uptr", which)
    ucol = plan.export("grp_ucol", which)
    bsrc = plan.export("blk_bsrc", which)
    assert np.array_equal(np.sort(grb), rb)                     # every row block once
    assert gptr[0] == 0 and gptr[-1] == rb.size and np.all(np.diff(gptr) > 0)
    assert uptr[0] == 0 and uptr[-1] == ucol.size and uptr.size == gptr.size
    slot_of = {int(r): s for s, r in enumerate(rb)}
    seen = np.zeros(bcol.size, bool)
    for g in range(gptr.size - 1):
        slots = [slot_of[int(r)] for r in grb[gptr[g]:gptr[g + 1]]]
        cols = np.concatenate([bcol[bptr[s]:bptr[s + 1]] for s in slots])
        got = ucol[uptr[g]:uptr[g + 1]]
        if got.size or len(slots) > 1:
            assert np.array_equal(got, np.unique(cols)), g
        local = {int(c): i for i, c in enumerate(got)}
        for s in slots:
            for t in range(bptr[s], bptr[s + 1]):
                c = int(bcol[t])
                assert bsrc[t] == (local[c] if c in local else -(c + 1)), (g, s, t)
                seen[t] = True
    assert seen.all()


@pytest.mark.parametrize("which", [0, 1])
def test_stencil_groups_format(which, monkeypatch):
    a, _ = gen.config2(grid=32)
    monkeypatch.setenv("HSPMM_GROUPS", "-1")
    plan = make_plan(hs, a, torch.float32, "auto", backward=True)
    monkeypatch.delenv("HSPMM_GROUPS", raising=False)
    info = plan.info()
    assert info["ngroups"] > 0
    assert info["grp_staged_tiles"] >= 0.3 * info["nblk"]
    check_group_format(plan, which)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("n", [4, 36, 64, 128, 200, 256])
def test_grouped_equals_ungrouped_and_oracle(dtype, n, monkeypatch):
    """The block stencil (grid 32) with and without groups: C, dB and dA
    bitwise equal, and against the oracle within the precision's bars."""
    print(f"groups dtype={dtype} n={n}", flush=True)
    a, _ = gen.config2(grid=32)
    g = np.random.default_rng(n)
    B = g.standard_normal((a.k, n))
    G = g.standard_normal((a.m, n))
    out = {}
    for mode in ("0", "1"):
        monkeypatch.setenv("HSPMM_GROUPS", mode)
        plan = make_plan(hs, a, dtype, "auto", backward=True)
        assert (plan.info()["ngroups"] > 0) == (mode != "0")
        Bd = to_dev(B, dtype)
        C = plan.run(Bd)
        dB, dA = plan.backward(Bd, to_dev(G, dtype))
        torch.cuda.synchronize()
        out[mode] = [t.cpu() for t in (C, dB, dA)]
    monkeypatch.delenv("HSPMM_GROUPS", raising=False)
    for x, y in zip(out["0"], out["1"]):
        assert torch.equal(x, y)
    C = out["1"][0].double().numpy()
    ref = oracle.spmm(a.m, a.k, a.row_ptr, a.col_idx, a.vals, B)
    assert oracle.rel_err(C, ref) <= TOL[dtype]
    assert scaled_row_errors(C, ref, abs_forward(a, B)).max() <= ROW_TOL[dtype]
    assert oracle.rel_err(out["1"][1].double().numpy(),
                          oracle.spmm_t(a.m, a.k, a.row_ptr, a.col_idx, a.vals, G)) <= TOL[dtype]


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_forced_groups_on_irregular_matrices(dtype, seed, monkeypatch):
    """Groups forced on (HSPMM_GROUPS=1) over matrices where they pay
    little: random, banded and with empty row blocks, so that groups with
    no staged column, single-row-block groups and a ragged last row block
    all occur; the format and the product still hold."""
    g = np.random.default_rng(seed)
    if seed == 0:
        a = gen.random_csr(seed, 420, 380, 0.03)
    elif seed == 1:
        a = gen.config5(1 if dtype == torch.float32 else 5, max_rows=3000)
    else:
        a = gen.random_csr(seed, 333, 300, 0.05)
        keep = (a.rows() // 16) % 3 != 1                       # every third row block empty
        a = gen.csr_from_coo(a.m, a.k, a.rows()[keep], a.col_idx[keep], a.vals[keep])
    monkeypatch.setenv("HSPMM_GROUPS", "1")
    plan = make_plan(hs, a, dtype, "bcsr", backward=True)
    monkeypatch.delenv("HSPMM_GROUPS", raising=False)
    info = plan.info()
    if info["ngroups"] == 0:
        pytest.skip("no tile of this matrix shares a column inside a group")
    check_group_format(plan, 0)
    n = 40
    B = g.standard_normal((a.k, n))
    G = g.standard_normal((a.m, n))
    Bd = to_dev(B, dtype)
    C = plan.run(Bd)
    dB, _ = plan.backward(Bd, to_dev(G, dtype), need_dA=False)
    torch.cuda.synchronize()
    assert oracle.rel_err(C.double().cpu().numpy(), oracle.spmm(a.m, a.k, a.row_ptr, a.col_idx, a.vals, B)) <= TOL[dtype]
    assert oracle.rel_err(dB.double().cpu().numpy(),
                          oracle.spmm_t(a.m, a.k, a.row_ptr, a.col_idx, a.vals, G)) <= TOL[dtype]
