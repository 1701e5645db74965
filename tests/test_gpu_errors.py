"""Error paths on the device: invalid CSR input is found by the plan's
checking kernels before any kernel depends on it, the workspace cap and the
argument checks return their status codes, and a failed call leaves the
library usable."""
import ctypes

import numpy as np
import pytest
import torch

import gen
import oracle
from tests.gpu_util import TOL, make_plan, oracle_forward, to_dev

pytestmark = pytest.mark.gpu

hs = pytest.importorskip("paper_2511_08158_amd")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _plan_raw(m, k, row_ptr, col_idx, vals, **kw):
    dev = torch.device("cuda:0")
    return hs.Plan(np.asarray(row_ptr), np.asarray(col_idx), torch.tensor(vals, device=dev), (m, k), **kw)


def _code(fn):
    with pytest.raises(hs.HspmmError) as e:
        fn()
    return e.value.code


def test_invalid_csr_is_rejected():
    print("invalid csr", flush=True)
    vals = np.ones(4)
    # row pointer decreasing, not starting at 0, not ending at nnz
    assert _code(lambda: _plan_raw(3, 5, [0, 3, 2, 4], [0, 1, 2, 3], vals)) == -2
    assert _code(lambda: _plan_raw(3, 5, [1, 2, 3, 4], [0, 1, 2, 3], vals)) == -2
    assert _code(lambda: _plan_raw(3, 5, [0, 1, 2, 3], [0, 1, 2, 3], vals)) == -2
    # a column outside [0, k)
    assert _code(lambda: _plan_raw(3, 5, [0, 1, 2, 4], [0, 1, 2, 5], vals)) == -2
    assert _code(lambda: _plan_raw(3, 5, [0, 1, 2, 4], [0, -1, 2, 3], vals)) == -2
    assert hs.library().hybrid_spmm_last_error() != b""


def test_workspace_cap_block_rows_and_leading_dimension():
    print("workspace cap", flush=True)
    a = gen.random_csr(2, 120, 110, 0.1)
    assert _code(lambda: make_plan(hs, a, torch.float32, "auto", max_workspace_bytes=1)) == -6
    # B_r other than the MFMA height is refused
    L = hs.library()
    from paper_2511_08158_amd import _lib
    dev = torch.device("cuda:0")
    rp = torch.as_tensor(a.row_ptr, device=dev, dtype=torch.int32)
    ci = torch.as_tensor(a.col_idx, device=dev, dtype=torch.int32)
    v = torch.as_tensor(a.vals, device=dev)
    opts = _lib.PlanOpts(ctypes.sizeof(_lib.PlanOpts), 1, 0, 32, -1, 128, 0, 0)
    out = ctypes.c_void_p()
    rc = L.hybrid_spmm_plan(ctypes.byref(out), a.m, a.k, a.nnz, ctypes.c_void_p(rp.data_ptr()),
                            ctypes.c_void_p(ci.data_ptr()), ctypes.c_void_p(v.data_ptr()), 0, ctypes.byref(opts),
                            ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == -1 and not out.value
    # ld < n
    plan = make_plan(hs, a, torch.float32, "auto")
    B = to_dev(np.ones((a.k, 8)), torch.float32)
    C = torch.empty((a.m, 8), device=dev)
    rc = L.hybrid_spmm_run(plan.handle, 8, ctypes.c_void_p(B.data_ptr()), 7, ctypes.c_void_p(C.data_ptr()), 8,
                           ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == -1
    # the plan and the library still work after the failed calls
    Bn = np.random.default_rng(0).standard_normal((a.k, 8))
    Cg = plan.run(to_dev(Bn, torch.float32))
    torch.cuda.synchronize()
    assert oracle.rel_err(Cg.double().cpu().numpy(), oracle_forward(a, Bn)) <= TOL[torch.float32]
