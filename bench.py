"""Benchmark: hybrid CSR+BCSR SpMM forward + backward on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload stencil|gcn|powerlaw]

A step is one pass of the whole path over one batch of synthetic input with
everything resident in HBM: C = A B, dB = A^T dC and dA = SDDMM(dC, B) on
A's pattern (the plan is built once, outside the timed region, as the paper
excludes format conversion from its SpMM timing).  Default workload: the
65,536 x 65,536 block stencil (128 x 128 grid, 4 DOFs, 9-point, dense 4x4
couplings, +5 % scattered entries; 2,451,523 stored entries), dense width
N = 128, FP32.

Prints one JSON line: GFLOP/s of the hybrid (AUTO split) step counting
6 nnz N flops (2 nnz N per product, Table 3's convention), the same for the
CSR-only path, the roofline entry of the dominant kernel (HIP events on
the launch stream), and the CPU baseline: the FP64 oracle timed on the host
cores, whose outputs of the same step are also the references of the
error of every GPU output (without the CPU baseline, the errors are null).
The oracle runs in that leg only.

Timing protocol of the graded figures: every timed step is cold -- a read
sweep over a 1 GiB buffer between steps, outside the events, evicts the
inputs, the plan and the outputs from L2 and the 256 MB MALL (the block
stencil's 87 MB per product would otherwise be served from the MALL).  The
sweep reads rather than writes: a 1 GiB fill leaves the caches full of dirty
lines whose write-back then lands inside the next timed step (measured on the
stencil step: 132 us after a fill, 116 us after a read sweep or after a fill
followed by a read sweep).  Each step runs from its first kernel's start to
its last kernel's end, from the kernels' own dispatch timestamps, with no
event or marker between them.  `value` and `ms_per_step` are the median over
the K timed steps; the roofline entry uses the dominant kernel's mean
duration over K more cold steps in which every product records its own
start and stop.  Warm (back-to-back) figures are reported beside them.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
from pathlib import Path

ROOT = Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s


def rel_err(x, ref):
    """Frobenius-norm relative error (absolute when the reference is zero)."""
    import numpy as np
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    d = float(np.linalg.norm(x - ref))
    r = float(np.linalg.norm(ref))
    return d / r if r > 0 else d


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="stencil", choices=["stencil", "gcn", "powerlaw"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device copy 10 times (calibrates HBM byte counters)")
    ap.add_argument("--sweep", action="store_true",
                    help="structure sweep: forward GFLOP/s of the AUTO split vs CSR-only per matrix and N")
    ap.add_argument("--sweep-rows", type=int, default=500_000, help="row cap of the sweep matrices")
    ap.add_argument("--sweep-n", default="16,32,64,128,256")
    ap.add_argument("--sweep-dtypes", default="f64,f32,f16", help="compute precisions of the sweep")
    ap.add_argument("--sweep-members", default="0-63", help="sweep members, e.g. 0-31 or 3,7")
    ap.add_argument("--gcn-train", action="store_true",
                    help="time a two-layer graph-convolution training loop on the 232,965-node graph")
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--no-vendor", action="store_true", help="skip the vendor CSR product timed for context")
    ap.add_argument("--no-other-dtypes", action="store_true",
                    help="skip the same step in the other compute precisions (stencil only)")
    ap.add_argument("--graded-only", action="store_true",
                    help="only the W warm-up and K timed cold steps of the hybrid plan (for profiling)")
    ap.add_argument("--dtype", default=None, choices=["f64", "f32", "f16", "bf16"],
                    help="with --graded-only: the step in this compute precision (default: the workload's)")
    args = ap.parse_args()
    if args.dtype is not None and not args.graded_only:
        ap.error("--dtype applies to --graded-only runs")
    return args


# The paper's own figures (Apple M4 Pro CPU, SuiteSparse matrices, N = 32,
# forward only; Sec. 4.2 and Table 3), quoted beside the bench line as
# context: other hardware, other matrices, other width.
PAPER_CONTEXT = {
    "hardware": "Apple M4 Pro CPU (12 cores, 2 SME units)",
    "n": 32, "pass": "forward only", "matrices": "SuiteSparse (absent here)",
    "fp16_best_matrix_gflops": 1964.9,
    "table3_fp16_gflops_range": [70, 1042],
    "hybrid_vs_csr_only_avg_speedup": 45.64,
    "hybrid_best_share_of_matrices": 0.833,
}


def cpu_model() -> str:
    try:
        for line in Path("/proc/cpuinfo").read_text().splitlines():
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _members(spec):
    out = []
    for part in spec.split(","):
        if "-" in part:
            lo, hi = part.split("-")
            out.extend(range(int(lo), int(hi) + 1))
        elif part:
            out.append(int(part))
    return out


def sweep(args):
    """Forward throughput of AUTO vs CSR-only (and BCSR-only) over the 64
    seeded matrices of the structure sweep (uniform / banded / block-diagonal
    / power law, rows log-uniform in 1k-500k), in each compute precision and
    at each width: one JSON line per (matrix, precision, n) and a summary
    line per precision.  Each plan is timed warm, as the fastest of 6 batches
    of launches (about 2 ms of the CSR-only plan per batch, at most 20
    launches), the three plans' batches interleaved in rotating order (small
    matrices run 7-12 us per launch, where single batches of one plan spread
    by 10 % and more).  Sampled rows of every AUTO result are checked
    against their definition computed row by row in FP64."""
    import numpy as np
    import torch

    import gen
    import paper_2511_08158_amd as hs

    dev = torch.device("cuda:0")
    ns = [int(x) for x in args.sweep_n.split(",")]
    tdt = {"f64": torch.float64, "f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}
    dts = [d for d in args.sweep_dtypes.split(",") if d]
    tol = {"f64": 1e-12, "f32": 1e-5, "f16": 5e-3, "bf16": 5e-3}
    rows = []
    splits = ("auto", "csr", "bcsr")
    for i in _members(args.sweep_members):
        a = gen.config5(i, max_rows=args.sweep_rows)
        spec = a.meta
        vals = torch.tensor(a.vals, device=dev)
        g = np.random.default_rng(i)
        rs = np.sort(g.choice(a.m, min(a.m, 256), replace=False))
        for dname in dts:
            dt = tdt[dname]
            od = torch.float64 if dt == torch.float64 else torch.float32
            # the fixed splits do not depend on n; AUTO is planned per n
            fixed = {sp_: hs.Plan(a.row_ptr, a.col_idx, vals, (a.m, a.k), compute=dt, split=sp_)
                     for sp_ in ("csr", "bcsr")}
            for n in ns:
                b = gen.dense(i, gen.DENSE, a.k, n, "uniform")
                B = torch.tensor(b, device=dev).to(dt)
                plans = {"auto": hs.Plan(a.row_ptr, a.col_idx, vals, (a.m, a.k), compute=dt, split="auto",
                                         n_hint=n), **fixed}
                outs = {}
                for sp_, p in plans.items():
                    outs[sp_] = torch.empty((a.m, n), dtype=od, device=dev)
                    for _ in range(2):
                        p.run(B, out=outs[sp_])
                # launches per batch: about 2 ms of the CSR-only plan, at most 20
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                plans["csr"].run(B, out=outs["csr"])
                e1.record()
                torch.cuda.synchronize()
                reps = int(min(20, max(1, round(2.0 / max(e0.elapsed_time(e1), 1e-3)))))
                best = {sp_: float("inf") for sp_ in splits}
                for rnd in range(6):
                    for sp_ in splits[rnd % 3:] + splits[:rnd % 3]:
                        p = plans[sp_]
                        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                        e0.record()
                        for _ in range(reps):
                            p.run(B, out=outs[sp_])
                        e1.record()
                        torch.cuda.synchronize()
                        best[sp_] = min(best[sp_], e0.elapsed_time(e1) / reps * 1e-3)
                info = plans["auto"].info()
                line = {"i": i, "class": spec["class"], "m": a.m, "nnz": a.nnz, "dtype": dname, "n": n,
                        "auto_gflops": round(2.0 * a.nnz * n / best["auto"] / 1e9, 1),
                        "csr_gflops": round(2.0 * a.nnz * n / best["csr"] / 1e9, 1),
                        "bcsr_gflops": round(2.0 * a.nnz * n / best["bcsr"] / 1e9, 1),
                        "speedup": round(best["csr"] / best["auto"], 3),
                        "vs_best_fixed": round(min(best["csr"], best["bcsr"]) / best["auto"], 3),
                        "rb_bcsr": info["rb_bcsr"], "rb_total": (a.m + 15) // 16, "fill": round(info["fill"], 3)}
                # sampled rows of the AUTO result against their definition,
                # row by row in FP64 on the unrounded operands
                ref = np.stack([a.vals[a.row_ptr[r]:a.row_ptr[r + 1]] @ b[a.col_idx[a.row_ptr[r]:a.row_ptr[r + 1]]]
                                for r in rs])
                got = outs["auto"][torch.as_tensor(rs, device=dev)].double().cpu().numpy()
                line["err"] = float(f"{rel_err(got, ref):.2e}")
                line["err_ok"] = line["err"] <= tol[dname]
                plans["auto"].close()
                del outs, B
                rows.append(line)
                print(json.dumps(line), flush=True)
            for p in fixed.values():
                p.close()
    for dname in dts:
        rr = [r for r in rows if r["dtype"] == dname]
        if not rr:
            continue
        rat = np.array([r["speedup"] for r in rr])
        same = np.array([r["rb_bcsr"] == 0 for r in rr])
        eq = np.where(same, 1.0, rat)
        best_eq = np.where(same, np.array([r["csr_gflops"] / max(r["csr_gflops"], r["bcsr_gflops"]) for r in rr]),
                           np.array([r["vs_best_fixed"] for r in rr]))
        print(json.dumps({"sweep_summary": {
            "dtype": dname, "runs": len(rr),
            "auto_not_slower_share": round(float(np.mean(rat >= 0.98)), 3),
            "auto_not_slower_share_same_plan_equal": round(float(np.mean(eq >= 0.98)), 3),
            "geomean_speedup_auto_vs_csr": round(float(np.exp(np.mean(np.log(rat)))), 3),
            "geomean_speedup_auto_vs_csr_same_plan_equal": round(float(np.exp(np.mean(np.log(eq)))), 3),
            "geomean_auto_vs_best_fixed_same_plan_equal": round(float(np.exp(np.mean(np.log(best_eq)))), 3),
            "max_speedup": round(float(rat.max()), 3), "min_speedup": round(float(rat.min()), 3),
            "runs_auto_is_csr_only_plan": int(same.sum()),
            "timing_spread_same_plan": [round(float(rat[same].min()), 3), round(float(rat[same].max()), 3)]
            if same.any() else None,
            "max_err": max(r["err"] for r in rr), "all_err_ok": all(r["err_ok"] for r in rr)}}), flush=True)


def gcn_train(args):
    """Two-layer graph convolution trained on the synthetic 232,965-node
    graph: H = relu(A (X W1)), logits = A (H W2), cross entropy on seeded
    labels, plain SGD on W1 and W2.  The sparse products run in the library
    through its autograd function (A is constant, so its backward is the
    transposed product alone); the dense products, activation and loss are
    PyTorch.  Reports the epoch time, the sparse products' share of it, the
    plan time against 100 epochs (the paper amortises format conversion over
    training), and the first step's weight gradients against an FP64 scipy
    evaluation of the same network."""
    import numpy as np
    import torch
    import torch.nn.functional as F

    import gen
    import paper_2511_08158_amd as hs

    dev = torch.device("cuda:0")
    a, x = gen.config4()
    hidden, classes = x.shape[1], 16
    g = np.random.default_rng([0, 5])
    w1 = g.standard_normal((x.shape[1], hidden)) / np.sqrt(x.shape[1])
    w2 = g.standard_normal((hidden, classes)) / np.sqrt(hidden)
    lab = g.integers(0, classes, a.m)
    X = torch.tensor(x, device=dev, dtype=torch.float32)
    labels = torch.tensor(lab, device=dev)
    W1 = torch.tensor(w1, device=dev, dtype=torch.float32, requires_grad=True)
    W2 = torch.tensor(w2, device=dev, dtype=torch.float32, requires_grad=True)
    vals = torch.tensor(a.vals, device=dev, dtype=torch.float32)
    rp_d = torch.tensor(a.row_ptr, device=dev, dtype=torch.int32)
    ci_d = torch.tensor(a.col_idx, device=dev, dtype=torch.int32)
    torch.cuda.synchronize()
    # the plan from the graph's CSR pattern resident on the device (the
    # preprocessing the paper times, Sec. 4.5), twice: the first build in a
    # process also pays first-use costs of the runtime
    plan_ms = []
    for _ in range(2):
        t0 = time.perf_counter()
        plan = hs.Plan(rp_d, ci_d, vals, (a.m, a.k), compute=torch.float32, backward=True, n_hint=hidden)
        torch.cuda.synchronize()
        plan_ms.append((time.perf_counter() - t0) * 1e3)
    plan_ms_first = plan_ms[0]
    plan_ms = plan_ms[-1]
    opt = torch.optim.SGD([W1, W2], lr=0.5)

    def forward():
        H = torch.relu(hs.spmm(plan, vals, X @ W1))
        return F.cross_entropy(hs.spmm(plan, vals, H @ W2), labels)

    # first step's gradients against FP64 scipy
    loss0 = forward()
    loss0.backward()
    gw1, gw2 = W1.grad.double().cpu().numpy(), W2.grad.double().cpu().numpy()
    A = a.to_scipy().tocsr()
    z1 = A @ (x @ w1)
    h = np.maximum(z1, 0.0)
    logits = A @ (h @ w2)
    pr = np.exp(logits - logits.max(axis=1, keepdims=True))
    pr /= pr.sum(axis=1, keepdims=True)
    ref_loss = float(-np.mean(np.log(pr[np.arange(a.m), lab])))
    dl = pr
    dl[np.arange(a.m), lab] -= 1.0
    dl /= a.m
    dhw2 = A.T @ dl
    rw2 = h.T @ dhw2
    dz1 = (dhw2 @ w2.T) * (z1 > 0)
    rw1 = x.T @ (A.T @ dz1)
    rel = lambda u, v: float(np.linalg.norm(u - v) / np.linalg.norm(v))

    def epoch():
        opt.zero_grad(set_to_none=True)
        loss = forward()
        loss.backward()
        opt.step()
        return loss

    for _ in range(3):
        epoch()
    torch.cuda.synchronize()
    losses = []
    t0 = time.perf_counter()
    for _ in range(args.epochs):
        losses.append(epoch())
    torch.cuda.synchronize()
    epoch_ms = (time.perf_counter() - t0) / args.epochs * 1e3
    # the sparse products of one epoch alone: two forward products (n = 128,
    # 16) and their two transposed products
    B1 = torch.randn(a.k, hidden, device=dev)
    B2 = torch.randn(a.k, classes, device=dev)
    D1 = torch.randn(a.m, hidden, device=dev)
    D2 = torch.randn(a.m, classes, device=dev)
    reps = 10
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        plan.run(B1)
        plan.run(B2)
        plan.backward(B2, D2, need_dA=False)
        plan.backward(B1, D1, need_dA=False)
    torch.cuda.synchronize()
    sp_ms = (time.perf_counter() - t0) / reps * 1e3
    line = {"gcn_train": {
        "nodes": a.m, "nnz": a.nnz, "features": x.shape[1], "hidden": hidden, "classes": classes,
        "epochs_timed": args.epochs, "epoch_ms": round(epoch_ms, 3),
        "sparse_ms_per_epoch": round(sp_ms, 3), "sparse_share": round(sp_ms / epoch_ms, 3),
        "plan_ms": round(plan_ms, 1), "plan_ms_first_build": round(plan_ms_first, 1),
        "plan_share_100_epochs": round(plan_ms / (plan_ms + 100 * epoch_ms), 4),
        "split": {k: plan.info()[k] for k in ("rows_csr", "rb_bcsr")},
        "loss_first": round(float(loss0), 5), "loss_first_fp64": round(ref_loss, 5),
        "loss_last": round(float(losses[-1]), 5),
        "grad_rel_err_first_step": {"W1": float(f"{rel(gw1, rw1):.2e}"), "W2": float(f"{rel(gw2, rw2):.2e}")},
        "data": "synthetic"}}
    print(json.dumps(line), flush=True)


def copy_probe():
    """A plain copy kernel of known size: 1 GiB read + 1 GiB written per launch."""
    import torch
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(10):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_per_launch": {"read": src.numel() * 4, "write": dst.numel() * 4},
                      "launches": 10}), flush=True)


def kernel_sources_hash() -> str:
    h = hashlib.sha256()
    for p in sorted((ROOT / "paper_2511_08158_amd" / "csrc").iterdir()):
        h.update(p.read_bytes())
    return h.hexdigest()[:16]


def workload(name):
    import gen
    if name == "stencil":
        a, b = gen.config2()
        return a, b, "f32", "block_stencil_65536_n128"
    if name == "gcn":
        a, b = gen.config4()
        return a, b, "f32", "gcn_232965_n128"
    a, b = gen.config3(n=64)
    return a, b, "f16", "powerlaw_1048576_n64"


def alg_bytes_forward(m, k, nnz, n, sv, sb, sc):
    """Compulsory HBM bytes of one product: A once (index + value per entry,
    row pointer), the dense input once, the output once."""
    return nnz * (sv + 4) + 4 * (m + 1) + k * n * sb + m * n * sc


def alg_bytes_sddmm(m, k, nnz, n, sb, sg, sd):
    return nnz * 4 + 4 * (m + 1) + m * n * sg + k * n * sb + nnz * sd


def main():
    args = parse()
    if args.copy_probe:
        copy_probe()
        return
    if args.sweep:
        sweep(args)
        return
    if args.gcn_train:
        gcn_train(args)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); "
              "the library has no multi-GPU path.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import gen
    import paper_2511_08158_amd as hs

    dev = torch.device("cuda:0")
    a, b, dt, wname = workload(args.workload)
    if args.dtype is not None:
        dt = args.dtype
    tdtype = {"f64": torch.float64, "f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}[dt]
    # outputs and dC: FP64 for an FP64 step, FP32 otherwise
    odt = torch.float64 if dt == "f64" else torch.float32
    n = b.shape[1]
    g = gen.dense(0, gen.GRAD, a.m, n)
    vals = torch.tensor(a.vals, device=dev)
    B = torch.tensor(b, device=dev).to(tdtype)
    dC = torch.tensor(g, device=dev, dtype=odt)
    # the input CSR pattern resident on the device, as the values are: the
    # plan time is the format build alone (the upload is reported beside it)
    torch.cuda.synchronize()
    t_up = time.perf_counter()
    rp_d = torch.tensor(a.row_ptr, device=dev, dtype=torch.int32)
    ci_d = torch.tensor(a.col_idx, device=dev, dtype=torch.int32)
    torch.cuda.synchronize()
    upload_ms = (time.perf_counter() - t_up) * 1e3

    def make(split):
        t0 = time.perf_counter()
        p = hs.Plan(rp_d, ci_d, vals, (a.m, a.k), compute=tdtype, split=split, backward=True, n_hint=n)
        torch.cuda.synchronize()
        return p, (time.perf_counter() - t0) * 1e3

    stream = torch.cuda.current_stream()

    def time_steps(plan, steps, warmup):
        C = torch.empty((a.m, n), dtype=torch.float32, device=dev)
        for _ in range(warmup):
            plan.run(B, out=C)
            plan.backward(B, dC)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            plan.run(B, out=C)
            plan.backward(B, dC)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    def step_calls(plan, C, Bx=None, dCx=None):
        """The step's products one by one: the forward, then the backward as
        one call when the library computes both gradients in one pass (one
        kernel), else dB and dA as the two products it runs.  Bx, dCx: the
        operands in another precision (default: the workload's)."""
        Bx = B if Bx is None else Bx
        dCx = dC if dCx is None else dCx
        calls = {"forward": lambda: plan.run(Bx, out=C)}
        if plan.backward_fused(Bx, dCx):
            calls["backward"] = lambda: plan.backward(Bx, dCx)
        else:
            calls["backward_dB"] = lambda: plan.backward(Bx, dCx, need_dB=True, need_dA=False)
            calls["backward_dA"] = lambda: plan.backward(Bx, dCx, need_dB=False, need_dA=True)
        return calls

    def time_kernels(plan, reps):
        """Average duration of each launch, HIP events on the launch stream."""
        C = torch.empty((a.m, n), dtype=torch.float32, device=dev)
        out = {}
        for name, fn in step_calls(plan, C).items():
            for _ in range(3):
                fn()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                fn()
            e1.record(stream)
            torch.cuda.synchronize()
            out[name] = e0.elapsed_time(e1) / reps * 1e3  # us
        return out

    flush_buf = torch.ones(1 << 28, dtype=torch.float32, device=dev)  # 1 GiB

    def flush():
        """Read sweep over 1 GiB: evicts L2 and the MALL, leaves no dirty lines."""
        flush_buf.sum()

    def bracket(ev, fns):
        """Run the products `fns` in order, the first one's first kernel
        recording ev[0] as it starts and the last one's last kernel ev[1] as
        it ends (their own dispatch timestamps): nothing between the kernels
        and no marker before or after them."""
        last = len(fns) - 1
        for j, fn in enumerate(fns):
            hs.set_timing_events(ev[0] if j == 0 else None, ev[1] if j == last else None)
            fn()
        hs.set_timing_events()

    def cold_steps(plan, steps, warmup, per_kernel, Bx=None, dCx=None, out_dtype=torch.float32):
        """`warmup` untimed and `steps` timed cold steps.  Before each step a
        1 GiB read sweep (outside the events) evicts the inputs, the plan and
        the outputs from L2 and the 256 MB MALL.  The step runs from its
        first kernel's start to its last kernel's end, both from the kernels'
        own dispatch timestamps (hybrid_spmm_set_timing_events).  per_kernel:
        each product also records its own start and stop, for per-launch
        durations; a start event delays its kernel's dispatch (about 4.5 us),
        so steps timed this way are not the graded ones.  Returns the
        per-step (and per-launch) durations in us."""
        C = torch.empty((a.m, n), dtype=out_dtype, device=dev)
        calls = step_calls(plan, C, Bx, dCx)
        nev = 2 * len(calls) if per_kernel else 2
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(nev)] for _ in range(warmup + steps)]
        for ev in evs:  # create the events before the timed steps
            for e in ev:
                e.record(stream)
        torch.cuda.synchronize()

        def one(ev):
            flush()
            if per_kernel:
                for j, fn in enumerate(calls.values()):
                    hs.set_timing_events(ev[2 * j], ev[2 * j + 1])
                    fn()
                hs.set_timing_events()
            else:
                bracket(ev, list(calls.values()))

        for ev in evs[:warmup]:
            one(ev)
        torch.cuda.synchronize()
        for ev in evs[warmup:]:
            one(ev)
        torch.cuda.synchronize()
        evs = evs[warmup:]
        out = {"step_us": np.array([ev[0].elapsed_time(ev[-1]) * 1e3 for ev in evs])}
        if per_kernel:
            out["kernels"] = {name: np.array([ev[2 * j].elapsed_time(ev[2 * j + 1]) * 1e3 for ev in evs])
                              for j, name in enumerate(calls)}
        return out

    def step_percentiles(plan, reps, cold):
        """Per-step durations (each step bracketed by its first kernel's start
        and its last kernel's end); cold: a 1 GiB read sweep between steps,
        outside the events."""
        C = torch.empty((a.m, n), dtype=torch.float32, device=dev)
        fns = list(step_calls(plan, C).values())
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for e0, e1 in ev:
            e0.record(stream)
            e1.record(stream)
        torch.cuda.synchronize()
        for i in range(reps + 2):
            if cold:
                flush()
            if i >= 2:
                bracket(ev[i - 2], fns)
            else:
                for fn in fns:
                    fn()
        torch.cuda.synchronize()
        us = np.array([e0.elapsed_time(e1) * 1e3 for e0, e1 in ev])
        return pct(us)

    def pct(us):
        return {q: float(np.percentile(us, p)) for q, p in (("p10", 10), ("p50", 50), ("p90", 90))}

    flops = 6.0 * a.nnz * n
    sv = sb = 4 if dt == "f32" else 2
    per_launch = {
        "forward": alg_bytes_forward(a.m, a.k, a.nnz, n, sv, sb, 4),
        "backward_dB": alg_bytes_forward(a.k, a.m, a.nnz, n, 4, 4, 4),
        "backward_dA": alg_bytes_sddmm(a.m, a.k, a.nnz, n, sb, 4, 4),
    }
    # the one-pass backward: A^T, dC and B read once, dB and dA written once
    per_launch["backward"] = alg_bytes_forward(a.k, a.m, a.nnz, n, 4, 4, 4) + a.k * n * sb + a.nnz * 4

    def step_bytes_of(names):
        """compulsory bytes of a step made of these products"""
        return sum(per_launch[k] for k in names)

    if args.graded_only:
        # the graded measurement alone (the profiled command): W warm-up and
        # K timed cold steps of the hybrid plan
        plan, _ = make("auto")
        cs = cold_steps(plan, args.steps, args.warmup, per_kernel=False, out_dtype=odt)
        ck = cold_steps(plan, args.steps, 2, per_kernel=True, out_dtype=odt)
        t = float(np.median(cs["step_us"])) * 1e-6
        print(json.dumps({"graded_only": True, "workload": wname, "dtype": dt, "steps": args.steps, "warmup": args.warmup,
                          "value": round(flops / t / 1e9, 2), "ms_per_step": round(t * 1e3, 5),
                          "kernels_us_cold_mean": {k: round(float(v.mean()), 2) for k, v in ck["kernels"].items()}}),
              flush=True)
        return

    results = {}
    for split in ("auto", "csr"):
        plan, plan_ms = make(split)
        t_warm = time_steps(plan, args.steps, args.warmup)
        kt_warm = time_kernels(plan, max(10, args.steps))
        # the graded timed region: exactly K cold steps, each bracketed by
        # its first kernel's start and its last kernel's end
        torch.cuda.synchronize()
        cs = cold_steps(plan, args.steps, args.warmup, per_kernel=False)
        torch.cuda.synchronize()
        # per-launch durations for the roofline: K more cold steps of the
        # same kind, each product's kernels timed by their own dispatch
        # timestamps
        ck = cold_steps(plan, args.steps, 2, per_kernel=True)
        reps_p = max(100, args.steps)
        results[split] = {"plan": plan, "t_warm": t_warm, "plan_ms": plan_ms, "kernels_us_warm": kt_warm,
                          "cold": cs, "cold_k": ck, "t": float(np.median(cs["step_us"])) * 1e-6,
                          "info": plan.info(), "pct_warm": step_percentiles(plan, reps_p, False),
                          "pct_cold": step_percentiles(plan, reps_p, True)}
    del flush_buf

    # CPU baseline (the only leg that runs the oracle): whole fwd+bwd passes
    # of the FP64 oracle on the same workload, timed on the host cores, for
    # about --cpu-seconds; the last pass's outputs are the references of the
    # errors below
    hyb = results["auto"]["plan"]
    b_used = B.double().cpu().numpy()
    refs = refs0 = cpu_line = None
    if not args.no_cpu_baseline:
        import oracle as orc
        # the host's share of cores on the GPU machine is 16 threads whatever
        # the affinity mask shows; the threads used are reported as `cores`
        visible = len(os.sched_getaffinity(0))
        threads = min(visible, 16)

        def oracle_pass(nt):
            t0 = time.perf_counter()
            r = (orc.spmm(a.m, a.k, a.row_ptr, a.col_idx, a.vals, b_used, nthreads=nt),
                 orc.spmm_t(a.m, a.k, a.row_ptr, a.col_idx, a.vals, g, nthreads=nt),
                 orc.sddmm(a.m, a.k, a.row_ptr, a.col_idx, g, b_used, nthreads=nt))
            return time.perf_counter() - t0, r

        oracle_pass(threads)  # warm-up
        times, t_start = [], time.perf_counter()
        while len(times) < 3 or (time.perf_counter() - t_start < args.cpu_seconds and len(times) < 50):
            dt_pass, (r_c, r_db, r_da) = oracle_pass(threads)
            times.append(dt_pass)
        tc = float(np.median(times))
        cpu_line = {"value": round(6.0 * a.nnz * n / tc / 1e9, 3), "unit": "GFLOP/s", "cores": threads,
                    "kind": "oracle",
                    "sample": f"median of {len(times)} full fwd+bwd passes (C, dB, dA) of the FP64 oracle on the "
                              f"whole workload after one warm-up pass",
                    "host_cores_visible": visible, "cpu_model": cpu_model()}
        # one single-threaded pass beside it (the oracle sums each row in
        # order whatever the thread count, so the outputs are the same)
        cpu_line["single_thread_value"] = round(6.0 * a.nnz * n / oracle_pass(1)[0] / 1e9, 3)
        refs = {"C": r_c, "dB": r_db, "dA": r_da}
        # the unquantised problem: end-to-end reference of the other precisions
        if dt == "f32" and np.array_equal(b_used, b):
            refs0 = refs
        else:
            refs0 = {"C": orc.spmm(a.m, a.k, a.row_ptr, a.col_idx, a.vals, b, nthreads=threads), "dB": r_db,
                     "dA": orc.sddmm(a.m, a.k, a.row_ptr, a.col_idx, g, b, nthreads=threads)}

    C = hyb.run(B)
    dB, dA = hyb.backward(B, dC)
    torch.cuda.synchronize()
    err = None
    if refs is not None:
        err = {"C": rel_err(C.double().cpu().numpy(), refs["C"]),
               "dB": rel_err(dB.double().cpu().numpy(), refs["dB"]),
               "dA": rel_err(dA.double().cpu().numpy(), refs["dA"])}
    tol = 1e-5 if dt == "f32" else 5e-3

    t_h, t_c = results["auto"]["t"], results["csr"]["t"]
    step_bytes = step_bytes_of(results["auto"]["cold_k"]["kernels"])
    gflops = flops / t_h / 1e9

    # roofline of the dominant kernel of the hybrid step: mean duration of
    # each launch inside the timed cold steps
    kc = {k: float(v.mean()) for k, v in results["auto"]["cold_k"]["kernels"].items()}
    dom = max(kc, key=kc.get)
    achieved = per_launch[dom] / (kc[dom] * 1e-6) / 1e9
    traffic = None
    prof = ROOT / "profiles" / f"traffic_{wname}.json"
    if prof.exists():
        rec = json.loads(prof.read_text())
        if rec.get("sources_hash") == kernel_sources_hash():
            traffic = rec.get("bytes_per_launch", {}).get(dom)

    def rnd(d):
        return {k: round(v, 2) for k, v in d.items()}

    line = {
        "metric": "SpMM GFLOP/s & % HBM roofline, hybrid vs CSR-only, fwd+bwd, at stated error",
        "value": round(gflops, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_h * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dt,
        "data": "synthetic",
        "config": {"workload": wname, "m": a.m, "k": a.k, "nnz": a.nnz, "n": n,
                   "step": "C=A*B; dB=A^T*dC; dA=SDDMM(dC,B)", "split": "auto",
                   "timing": "cold: 1 GiB read sweep between steps outside the events; each step from its first kernel's start to its last kernel's end (dispatch timestamps); median of the K timed steps"},
        "hbm_roofline_frac_step": round(step_bytes / t_h / (HBM_PEAK_GBS * 1e9), 4),
        "csr_only": {"value": round(flops / t_c / 1e9, 2), "ms_per_step": round(t_c * 1e3, 5),
                     "kernels_us_cold_mean": rnd({k: float(v.mean()) for k, v in results["csr"]["cold_k"]["kernels"].items()}),
                     "kernels_us_warm": rnd(results["csr"]["kernels_us_warm"])},
        "speedup_vs_csr_only": round(t_c / t_h, 3),
        "warm": {"value": round(flops / results["auto"]["t_warm"] / 1e9, 2),
                 "ms_per_step": round(results["auto"]["t_warm"] * 1e3, 5),
                 "csr_only_value": round(flops / results["csr"]["t_warm"] / 1e9, 2),
                 "hbm_roofline_frac_step": round(step_bytes / results["auto"]["t_warm"] / (HBM_PEAK_GBS * 1e9), 4),
                 "kernels_us": rnd(results["auto"]["kernels_us_warm"])},
        "step_us_percentiles": {
            mode: {"steps": max(100, args.steps),
                   "auto": rnd(results["auto"][f"pct_{mode}"]),
                   "csr_only": rnd(results["csr"][f"pct_{mode}"]),
                   "gflops_p50": round(flops / (results["auto"][f"pct_{mode}"]["p50"] * 1e-6) / 1e9, 1),
                   "speedup_vs_csr_only_p50": round(results["csr"][f"pct_{mode}"]["p50"] / results["auto"][f"pct_{mode}"]["p50"], 3)}
            for mode in ("warm", "cold")},
        "timed_steps_us": rnd(pct(results["auto"]["cold"]["step_us"])),
        "error": None if err is None else {k: float(f"{v:.3e}") for k, v in err.items()},
        "error_ok": None if err is None else all(v <= tol for v in err.values()),
        "kernels_us": rnd(kc),
        "plan_ms": round(results["auto"]["plan_ms"], 1),
        "csr_upload_ms": round(upload_ms, 1),
        "split": {k: results["auto"]["info"][k] for k in ("rows_csr", "rb_bcsr", "nblk", "fill")},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "alg_bytes_per_launch": per_launch[dom],
                     "timing": "mean kernel duration (its dispatch timestamps) in K cold steps"},
        "context": PAPER_CONTEXT,
    }

    if not args.no_vendor:
        # context only: the vendor CSR product (torch.sparse over hipSPARSE)
        # on the same matrix and B, forward only, HIP events on the stream
        try:
            crow = torch.tensor(a.row_ptr, dtype=torch.int64, device=dev)
            coli = torch.tensor(a.col_idx, dtype=torch.int64, device=dev)
            Av = torch.sparse_csr_tensor(crow, coli, vals.to(tdtype), size=(a.m, a.k))
            Cv = Av @ B
            for _ in range(3):
                Cv = Av @ B
            reps_v = 20
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps_v):
                Cv = Av @ B
            e1.record(stream)
            torch.cuda.synchronize()
            tv = e0.elapsed_time(e1) / reps_v * 1e3
            Ch = hyb.run(B)
            torch.cuda.synchronize()
            line["vendor_csr_forward"] = {
                "library": "torch.sparse CSR @ dense (hipSPARSE)", "us": round(tv, 2),
                "gflops": round(2.0 * a.nnz * n / (tv * 1e-6) / 1e9, 1),
                "hybrid_forward_speedup_warm": round(tv / results["auto"]["kernels_us_warm"]["forward"], 3),
                "agreement_rel_err": float(f"{rel_err(Cv.double().cpu().numpy(), Ch.double().cpu().numpy()):.2e}")}
            del Av, Cv
        except Exception as ex:  # the vendor path is optional context
            line["vendor_csr_forward"] = {"error": str(ex)[:200]}

    if args.workload == "stencil" and not args.no_other_dtypes:
        # the same step in the other precisions of the method: GFLOP/s of the
        # AUTO and CSR-only plans, timed cold like the graded step (median of
        # the timed steps) and warm (back to back, the host's clock), and the
        # end-to-end error of every output against the CPU baseline's FP64
        # outputs on the unrounded inputs (FP16/BF16: B rounded to the type,
        # A scaled per row block, FP32 accumulation and outputs)
        flush_buf = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        other = {}
        for name, cdt, tol_d in (("f64", torch.float64, 1e-12), ("f16", torch.float16, 5e-3),
                                 ("bf16", torch.bfloat16, 5e-3)):
            Bd = torch.tensor(b, device=dev).to(cdt)
            dCd = torch.tensor(g, device=dev) if cdt == torch.float64 else dC
            od = torch.float64 if cdt == torch.float64 else torch.float32
            res_d, warm_d, e = {}, {}, None
            steps_d = max(10, args.steps // 4)
            for split in ("auto", "csr"):
                p = hs.Plan(a.row_ptr, a.col_idx, vals, (a.m, a.k), compute=cdt, split=split, backward=True,
                            n_hint=n)
                Cd = torch.empty((a.m, n), dtype=od, device=dev)
                for _ in range(5):
                    p.run(Bd, out=Cd)
                    p.backward(Bd, dCd)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(steps_d):
                    p.run(Bd, out=Cd)
                    p.backward(Bd, dCd)
                torch.cuda.synchronize()
                warm_d[split] = (time.perf_counter() - t0) / steps_d
                cs_d = cold_steps(p, steps_d, 3, False, Bd, dCd, od)
                res_d[split] = float(np.median(cs_d["step_us"])) * 1e-6
                if split == "auto" and refs0 is not None:
                    Cd = p.run(Bd)
                    dBd, dAd = p.backward(Bd, dCd)
                    torch.cuda.synchronize()
                    e = {"C": rel_err(Cd.double().cpu().numpy(), refs0["C"]),
                         "dB": rel_err(dBd.double().cpu().numpy(), refs0["dB"]),
                         "dA": rel_err(dAd.double().cpu().numpy(), refs0["dA"])}
                p.close()
            other[name] = {"value": round(flops / res_d["auto"] / 1e9, 2),
                           "csr_only": round(flops / res_d["csr"] / 1e9, 2),
                           "speedup_vs_csr_only": round(res_d["csr"] / res_d["auto"], 3),
                           "timing": f"cold, median of {steps_d} steps",
                           "warm_value": round(flops / warm_d["auto"] / 1e9, 2),
                           "warm_csr_only": round(flops / warm_d["csr"] / 1e9, 2),
                           "error": None if e is None else {k: float(f"{v:.3e}") for k, v in e.items()},
                           "error_ok": None if e is None else all(v <= tol_d for v in e.values()),
                           "tol": tol_d}
        line["other_dtypes"] = other

    if cpu_line is not None:
        line["cpu_baseline"] = cpu_line
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
