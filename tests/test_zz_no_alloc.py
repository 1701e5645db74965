"""hybrid_spmm_run_noalloc, called through the C ABI, against
hybrid_spmm_run: the same kernels, so the results must be bitwise equal, on
two calls in a row (the second with a smaller input), on a second smaller
plan, and past the static scratch's capacity it must refuse without
launching.  The plans have rows split across waves, so the static scratch is
really used."""
import ctypes

import numpy as np
import pytest
import torch

import gen
import oracle
from tests.gpu_util import TOL, make_plan, to_dev

pytestmark = pytest.mark.gpu

hs = pytest.importorskip("paper_2511_08158_amd")
from paper_2511_08158_amd import _lib  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _long_rows(seed, m, k, longest):
    g = np.random.default_rng(seed)
    lens = np.full(m, 6)
    lens[[1, m // 2, m - 1]] = [longest // 3, longest, longest // 2]
    rows = np.repeat(np.arange(m), lens)
    cols = np.concatenate([np.sort(g.choice(k, int(l), replace=False)) for l in lens])
    return gen.csr_from_coo(m, k, rows, cols, g.standard_normal(rows.size))


def _noalloc(plan, B, C):
    L = _lib.load()
    n = B.shape[1]
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return L.hybrid_spmm_run_noalloc(plan.handle, n, ctypes.c_void_p(B.data_ptr()), B.stride(0),
                                     ctypes.c_void_p(C.data_ptr()), C.stride(0), stream)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64, torch.float16])
def test_noalloc_equals_run_two_calls(dtype):
    print(f"noalloc two calls dtype={dtype}", flush=True)
    a = _long_rows(1, 80, 20000, 17000)
    small = _long_rows(2, 40, 9000, 6000)
    plan = make_plan(hs, a, dtype, "csr")
    plan_s = make_plan(hs, small, dtype, "csr")
    assert plan.info()["long_rows"] == 3 and plan_s.info()["long_rows"] == 3
    od = torch.float64 if dtype == torch.float64 else torch.float32
    g = np.random.default_rng(3)
    cases = [(plan, a, 256), (plan, a, 40), (plan_s, small, 24)]   # each after a larger one
    for p, mat, n in cases:
        B = to_dev(g.standard_normal((mat.k, n)), dtype)
        ref = p.run(B)
        C = torch.full((mat.m, n), float("nan"), dtype=od, device=B.device)
        assert _noalloc(p, B, C) == 0, _lib.load().hybrid_spmm_last_error()
        torch.cuda.synchronize()
        assert torch.equal(C, ref), (mat.m, n)
        assert oracle.rel_err(C.double().cpu().numpy(),
                              oracle.spmm(mat.m, mat.k, mat.row_ptr, mat.col_idx, mat.vals,
                                          B.double().cpu().numpy())) <= TOL[dtype]


def test_noalloc_hybrid_plan_and_refusal():
    """A plan with both parts (the fused launch) gives run's result; an n
    whose split rows would need more than the static array is refused with
    HSPMM_ERR_OOM, C is left untouched, and the entry point works again
    afterwards."""
    a, b = gen.config2(grid=32)
    long = _long_rows(4, 64, 4096, 4000)
    # rows with long entries (CSR-part, rows 0..63) above the stencil
    # (BCSR-part, the contiguous split of Alg. 1 at row 64)
    rows = np.concatenate([long.rows(), a.rows() + long.m])
    cols = np.concatenate([long.col_idx, a.col_idx])
    vals = np.concatenate([long.vals, a.vals])
    h = gen.csr_from_coo(a.m + long.m, a.k, rows, cols, vals)
    plan = make_plan(hs, h, torch.float32, "boundary", r_boundary=64)
    info = plan.info()
    assert info["rb_bcsr"] == a.m // 16 and info["rows_csr"] == 64 and info["long_rows"] == 3
    B = to_dev(b, torch.float32)
    ref = plan.run(B)
    C = torch.empty_like(ref)
    assert _noalloc(plan, B, C) == 0
    torch.cuda.synchronize()
    assert torch.equal(C, ref)
    # far too wide: every split row's partial needs n * 4 bytes
    n_big = 65_536
    Bw = torch.zeros((h.k, n_big), dtype=torch.float32, device=B.device)
    Cw = torch.full((h.m, n_big), 3.0, dtype=torch.float32, device=B.device)
    rc = _noalloc(plan, Bw, Cw)
    assert rc == -6
    assert b"static" in _lib.load().hybrid_spmm_last_error()
    torch.cuda.synchronize()
    assert bool((Cw == 3.0).all())
    del Bw, Cw
    C2 = torch.empty_like(ref)
    assert _noalloc(plan, B, C2) == 0
    torch.cuda.synchronize()
    assert torch.equal(C2, ref)
