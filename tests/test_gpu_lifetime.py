"""Plan lifetime against queued work: the products record nothing on their
streams, so destroying a plan must itself wait until every kernel that
reads the plan's memory has finished.  Products are queued on a side
stream, the plan is destroyed at once (no host wait in between), and the
outputs, owned by the caller, must still equal the oracle's."""
import numpy as np
import pytest
import torch

import gen
import oracle
from tests.gpu_util import TOL, make_plan, to_dev

pytestmark = pytest.mark.gpu

hs = pytest.importorskip("paper_2511_08158_amd")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("split", ["auto", "csr"])
def test_destroy_waits_for_queued_products(split):
    a, _ = gen.config2(grid=32)                       # 4,096 rows, both forms of the backward
    n = 128
    g = np.random.default_rng(21)
    B = g.standard_normal((a.k, n))
    G = g.standard_normal((a.m, n))
    plan = make_plan(hs, a, torch.float32, split, backward=True)
    Bd, Gd = to_dev(B, torch.float32), to_dev(G, torch.float32)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        # a queue of products long enough to be running when destroy is called
        for _ in range(30):
            C = plan.run(Bd)
            dB, dA = plan.backward(Bd, Gd)
        plan.close()
    torch.cuda.synchronize()
    assert plan._h is None
    ref_c = oracle.spmm(a.m, a.k, a.row_ptr, a.col_idx, a.vals, B)
    ref_db = oracle.spmm_t(a.m, a.k, a.row_ptr, a.col_idx, a.vals, G)
    ref_da = oracle.sddmm(a.m, a.k, a.row_ptr, a.col_idx, G, B)
    assert oracle.rel_err(C.double().cpu().numpy(), ref_c) <= TOL[torch.float32]
    assert oracle.rel_err(dB.double().cpu().numpy(), ref_db) <= TOL[torch.float32]
    assert oracle.rel_err(dA.double().cpu().numpy(), ref_da) <= TOL[torch.float32]
