"""Calibration of the workgroup partition (the GPU analogue of the thread
split of Sec. 3.5): the library's Eq. 2 fit and Eq. 3 argmax against the
oracle's least squares and brute-force enumeration on the samples it
measured, and results unchanged by the partition."""
import numpy as np
import pytest
import torch

import gen
import oracle
from oracle import loops_ref as L
from tests.gpu_util import TOL, make_plan, oracle_forward, to_dev

pytestmark = pytest.mark.gpu

hs = pytest.importorskip("paper_2511_08158_amd")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _check_fit(info):
    x = np.array(info["cand_x"], float)
    y = np.array(info["cand_y"], float)
    perf = np.array(info["cand_gflops"], float)
    coef = np.array(info["coef"])
    cols = [0]
    if np.unique(x).size >= 2 and info["x_max"] > 0:
        cols.append(1)
    if np.unique(y).size >= 2 and info["y_max"] > 0:
        cols.append(2)
    if np.unique(x).size >= 3 and info["x_max"] > 0:
        cols.append(3)
    if np.unique(y).size >= 3 and info["y_max"] > 0:
        cols.append(4)
    full = np.stack([np.ones_like(x), x, y, x * x, y * y], axis=1)
    ref = np.zeros(5)
    sol, *_ = np.linalg.lstsq(full[:, cols], perf, rcond=None)
    ref[cols] = sol
    if len(cols) == 5:
        assert np.allclose(L.fit_quadratic_ref(x, y, perf), ref, rtol=1e-9, atol=1e-9)
    scale = max(1.0, float(np.abs(perf).max()))
    pred = full @ coef
    pred_ref = full @ ref
    assert np.max(np.abs(pred - pred_ref)) <= 1e-6 * scale
    best = L.argmax_ref(coef, info["T"], x_min=1 if info["x_max"] else 0, y_min=1 if info["y_max"] else 0,
                        x_max=info["x_max"], y_max=info["y_max"])
    assert tuple(info["best"]) == best


def test_calibrate_mixed_plan():
    a, b = gen.config2(grid=64)            # 16,384 rows: half CSR-part, half BCSR-part
    plan = make_plan(hs, a, torch.float32, "boundary", r_boundary=a.m // 2)
    info = plan.info()
    assert info["rows_csr"] == a.m // 2 and info["rb_bcsr"] == a.m // 32
    B = to_dev(b, torch.float32)
    C0 = plan.run(B).cpu().numpy()
    cal = plan.calibrate(B, reps=3)
    print("calibration", cal, flush=True)
    assert len(cal["cand_x"]) > 5
    assert all(g > 0 for g in cal["cand_gflops"])
    _check_fit(cal)
    C1 = plan.run(B).cpu().numpy()
    # every row of C has one writer whatever the partition: bitwise equal
    assert np.array_equal(C0, C1)
    assert oracle.rel_err(C1, oracle_forward(a, b)) <= 1e-5


@pytest.mark.parametrize("split", ["csr", "bcsr"])
def test_calibrate_one_part(split):
    a, b = gen.config2(grid=48)
    plan = make_plan(hs, a, torch.float32, split)
    B = to_dev(b, torch.float32)
    C0 = plan.run(B).cpu().numpy()
    cal = plan.calibrate(B, reps=2)
    if split == "csr":
        assert cal["y_max"] == 0 and all(v == 0 for v in cal["cand_y"]) and cal["best"][1] == 0
    else:
        assert cal["x_max"] == 0 and all(v == 0 for v in cal["cand_x"]) and cal["best"][0] == 0
    _check_fit(cal)
    assert np.array_equal(plan.run(B).cpu().numpy(), C0)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float16, torch.bfloat16])
def test_calibrate_mixed_plan_other_dtypes(dtype):
    """The calibrated partition caps each part's workgroups, so the BCSR
    forms of every precision walk several units per workgroup: C stays
    bitwise the same, and the backward after calibration is unchanged."""
    print(f"calibration dtype={dtype}", flush=True)
    a, b = gen.config2(grid=48)
    plan = make_plan(hs, a, dtype, "boundary", backward=True, r_boundary=a.m // 2)
    B = to_dev(b, dtype)
    od = torch.float64 if dtype == torch.float64 else torch.float32
    G = to_dev(gen.dense(0, gen.GRAD, a.m, b.shape[1]), od)
    C0 = plan.run(B).cpu().numpy()
    dB0, dA0 = plan.backward(B, G)
    cal = plan.calibrate(B, reps=2)
    _check_fit(cal)
    assert np.array_equal(plan.run(B).cpu().numpy(), C0)
    dB1, dA1 = plan.backward(B, G)
    torch.cuda.synchronize()
    assert torch.equal(dB0, dB1) and torch.equal(dA0, dA1)
    # and against the FP64 oracle on the unrounded inputs
    g = gen.dense(0, gen.GRAD, a.m, b.shape[1])
    assert oracle.rel_err(C0, oracle_forward(a, b)) <= TOL[dtype]
    assert oracle.rel_err(dB1.double().cpu().numpy(),
                          oracle.spmm_t(a.m, a.k, a.row_ptr, a.col_idx, a.vals, g)) <= TOL[dtype]
    assert oracle.rel_err(dA1.double().cpu().numpy(),
                          oracle.sddmm(a.m, a.k, a.row_ptr, a.col_idx, g, b)) <= TOL[dtype]
