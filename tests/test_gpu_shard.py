"""Row-block sharding of the path, shown on one GPU: each shard's plan is
built from a contiguous range of A's row blocks (with B whole), writes its
own rows of C and dA, and the shards' partial dB = A_s^T dC_s add up to the
full dB (the sum a reduce-scatter would form across GPUs)."""
import numpy as np
import pytest
import torch

import gen
import oracle
from tests.gpu_util import TOL, to_dev

pytestmark = pytest.mark.gpu

hs = pytest.importorskip("paper_2511_08158_amd")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _rows(a, r0, r1):
    lo, hi = a.row_ptr[r0], a.row_ptr[r1]
    return gen.Csr(r1 - r0, a.k, (a.row_ptr[r0:r1 + 1] - lo).astype(np.int32), a.col_idx[lo:hi], a.vals[lo:hi])


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("shards", [2, 3])
def test_row_block_shards(dtype, shards):
    print(f"shards={shards} dtype={dtype}", flush=True)
    a, b = gen.config2(grid=32)                          # 4,096 rows, stencil + 5 % scattered entries
    g = gen.dense(0, gen.GRAD, a.m, b.shape[1])
    nrb = (a.m + 15) // 16
    cuts = [16 * (nrb * s // shards) for s in range(shards)] + [a.m]
    od = torch.float64 if dtype == torch.float64 else torch.float32
    B = to_dev(b, dtype)
    C_parts, dA_parts, dB_sum = [], [], None
    for r0, r1 in zip(cuts[:-1], cuts[1:]):
        s = _rows(a, r0, r1)
        plan = hs.Plan(s.row_ptr, s.col_idx, to_dev(s.vals), (s.m, s.k), compute=dtype, split="auto", backward=True)
        C_parts.append(plan.run(B))
        dB_s, dA_s = plan.backward(B, to_dev(g[r0:r1], od))
        dA_parts.append(dA_s)
        dB_sum = dB_s.double() if dB_sum is None else dB_sum + dB_s.double()
    torch.cuda.synchronize()
    C = torch.cat(C_parts).double().cpu().numpy()
    dA = torch.cat(dA_parts).double().cpu().numpy()
    assert oracle.rel_err(C, oracle.spmm(a.m, a.k, a.row_ptr, a.col_idx, a.vals, b)) <= TOL[dtype]
    assert oracle.rel_err(dA, oracle.sddmm(a.m, a.k, a.row_ptr, a.col_idx, g, b)) <= TOL[dtype]
    assert oracle.rel_err(dB_sum.cpu().numpy(), oracle.spmm_t(a.m, a.k, a.row_ptr, a.col_idx, a.vals, g)) <= TOL[dtype]
    # a shard's rows of C are bitwise those of the whole-matrix plan (the
    # same row blocks, the same per-row order of summation) when both plans
    # put them in the same part
    full = hs.Plan(a.row_ptr, a.col_idx, to_dev(a.vals), (a.m, a.k), compute=dtype, split="csr")
    Cf = full.run(B).double().cpu().numpy()
    C_csr = []
    for r0, r1 in zip(cuts[:-1], cuts[1:]):
        s = _rows(a, r0, r1)
        p = hs.Plan(s.row_ptr, s.col_idx, to_dev(s.vals), (s.m, s.k), compute=dtype, split="csr")
        C_csr.append(p.run(B).double().cpu().numpy())
    assert np.array_equal(np.concatenate(C_csr), Cf)
