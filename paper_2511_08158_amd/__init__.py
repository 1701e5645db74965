"""hspmm -- hybrid CSR + BCSR SpMM for the AMD MI355X (gfx950).

Thin Python binding over the C ABI in ``include/hspmm.h``: arguments are
marshalled here, every step of the computation runs in the HIP library
(``libhspmm.so``).  PyTorch supplies device memory and the current stream.

    plan = Plan(row_ptr, col_idx, vals, (m, k), compute=torch.float32,
                split="auto", backward=True)
    C = plan.run(B)                       # C = A B
    dB, dA = plan.backward(B, dC)         # A^T dC, SDDMM(dC, B) on A's pattern
    C = spmm(plan, vals, B)               # autograd.Function (grads for vals, B)
"""
from __future__ import annotations

import ctypes
import itertools
import weakref

import numpy as np
import torch

from . import _lib

__all__ = ["Plan", "spmm", "HspmmError", "DTYPES", "library", "set_timing_events", "check_dense"]

DTYPES = {torch.float64: _lib.F64, torch.float32: _lib.F32, torch.float16: _lib.F16,
          torch.bfloat16: _lib.BF16}
_TORCH_OF = {v: k for k, v in DTYPES.items()}
_NP_OF = {_lib.F64: np.float64, _lib.F32: np.float32, _lib.F16: np.float16, _lib.BF16: np.uint16}


class HspmmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_lib.STATUS.get(code, code)}: {msg}")
        self.code = code
        self.msg = msg


def library():
    """The loaded C library (raises ImportError if it was not built)."""
    return _lib.load()


def _check(rc: int):
    if rc != 0:
        msg = library().hybrid_spmm_last_error().decode(errors="replace")
        raise HspmmError(rc, msg)


def set_timing_events(start=None, stop=None):
    """Make every product this thread launches record the torch.cuda.Event
    `start` as its first kernel begins and `stop` as its last kernel ends
    (the kernels' own timestamps); no arguments clear them.  The events are
    recorded once on the current stream first so that they exist."""
    handles = []
    for e in (start, stop):
        if e is None:
            handles.append(None)
            continue
        if not e.cuda_event:
            e.record()
        handles.append(ctypes.c_void_p(e.cuda_event))
    _check(library().hybrid_spmm_set_timing_events(*handles))


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _out_dtype(compute: int):
    return torch.float64 if compute == _lib.F64 else torch.float32


def check_dense(X, rows, cols, dtype, device, name):
    """Raise HspmmError unless X is a `rows` x `cols` (cols None: any)
    matrix of `dtype` on `device` with unit column stride, the only form the
    C ABI can take as a pointer plus a leading dimension."""
    if not isinstance(X, torch.Tensor):
        raise HspmmError(-1, f"{name} must be a torch tensor")
    if X.device != device:
        raise HspmmError(-1, f"{name} must be on {device}, got {X.device}")
    if X.dtype != dtype:
        raise HspmmError(-3, f"{name} must be {dtype}, got {X.dtype}")
    if X.dim() != 2 or X.shape[0] != rows or (cols is not None and X.shape[1] != cols):
        want = f"{rows} x {'n' if cols is None else cols}"
        raise HspmmError(-1, f"{name} must be a {want} matrix, got shape {tuple(X.shape)}")
    if X.numel() and (X.stride(1) != 1 or X.stride(0) < X.shape[1]):
        raise HspmmError(-1, f"{name} must be row-major with unit column stride")
    return X


def _ld(X):
    return X.stride(0) if X.shape[0] > 0 and X.numel() else X.shape[1]


# every packing of a plan's values gets a fresh token: the autograd function
# compares tokens to know whether the plan still holds the values of the
# forward call it differentiates
_pack_tokens = itertools.count(1)


class Plan:
    """A hybrid plan of a CSR matrix A (m x k) resident on the GPU."""

    def __init__(self, row_ptr, col_idx, vals, shape, compute=torch.float32, split="auto",
                 backward=False, r_boundary=-1, n_hint=128, max_workspace_bytes=0, device=None):
        L = library()
        m, k = int(shape[0]), int(shape[1])
        dev = torch.device(device) if device is not None else (
            vals.device if isinstance(vals, torch.Tensor) and vals.is_cuda else torch.device("cuda"))
        rp = torch.as_tensor(row_ptr).to(device=dev, dtype=torch.int32).contiguous()
        ci = torch.as_tensor(col_idx).to(device=dev, dtype=torch.int32).contiguous()
        v = torch.as_tensor(vals)
        if v.dtype not in DTYPES:
            v = v.to(torch.float64)
        v = v.to(dev).contiguous()
        if rp.numel() != m + 1:
            raise HspmmError(-1, f"row_ptr has {rp.numel()} entries, expected {m + 1}")
        self.m, self.k, self.nnz_input = m, k, int(ci.numel())
        self.compute = DTYPES[compute] if isinstance(compute, torch.dtype) else int(compute)
        self.device = dev
        opts = _lib.PlanOpts(ctypes.sizeof(_lib.PlanOpts), self.compute,
                             _lib.SPLIT[split] if isinstance(split, str) else int(split),
                             16, int(r_boundary), int(n_hint), 1 if backward else 0,
                             int(max_workspace_bytes))
        h = ctypes.c_void_p()
        with torch.cuda.device(dev):
            _check(L.hybrid_spmm_plan(ctypes.byref(h), m, k, self.nnz_input, _ptr(rp), _ptr(ci),
                                      _ptr(v), DTYPES[v.dtype], ctypes.byref(opts), _stream()))
        self._h = h
        self._note_packed(vals, v)
        self.backward_enabled = bool(backward)

    def _note_packed(self, vals, v):
        """Record what the plan now holds: a fresh token, and the caller's
        tensor (weakly) with its version when the library read that tensor
        itself rather than a temporary converted copy."""
        self._pack_token = next(_pack_tokens)
        same = isinstance(vals, torch.Tensor) and v is vals
        self._packed_ref = weakref.ref(vals) if same else None
        self._packed_version = vals._version if same else None

    def holds_values_of(self, vals) -> bool:
        """True if the last packing read exactly this tensor at its current
        version (an unchanged static A needs no re-packing)."""
        r = self._packed_ref
        return r is not None and r() is vals and self._packed_version == vals._version

    # -- lifetime --------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            library().hybrid_spmm_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        if self._h is None or not self._h.value:
            raise HspmmError(-1, "plan is closed")
        return self._h

    # -- compute ---------------------------------------------------------
    @property
    def dense_dtype(self):
        return _TORCH_OF[self.compute]

    @property
    def out_dtype(self):
        return _out_dtype(self.compute)

    def _dense(self, X, rows, name, cols=None, dtype=None):
        return check_dense(X, rows, cols, self.dense_dtype if dtype is None else dtype, self.device, name)

    def run(self, B, out=None):
        """C = A B; B is k x n (row-major, dtype = compute); `out`, if
        given, is an m x n matrix of the output dtype on the plan's device."""
        B = self._dense(B, self.k, "B")
        n = B.shape[1]
        if out is None:
            out = torch.empty((self.m, n), dtype=self.out_dtype, device=self.device)
        else:
            self._dense(out, self.m, "out", cols=n, dtype=self.out_dtype)
        _check(library().hybrid_spmm_run(self.handle, n, _ptr(B), _ld(B), _ptr(out), _ld(out), _stream()))
        return out

    def backward(self, B, dC, need_dB=True, need_dA=True):
        """dB = A^T dC (k x n) and dA[e] = <dC[row(e)], B[col(e)]> in input
        order; dC is an m x n matrix of the output dtype on the plan's device."""
        B = self._dense(B, self.k, "B")
        n = B.shape[1]
        self._dense(dC, self.m, "dC", cols=n, dtype=self.out_dtype)
        dB = torch.empty((self.k, n), dtype=self.out_dtype, device=self.device) if need_dB else None
        dA = torch.empty(self.nnz_input, dtype=self.out_dtype, device=self.device) if need_dA else None
        _check(library().hybrid_spmm_backward(
            self.handle, n, _ptr(B), _ld(B), _ptr(dC), _ld(dC),
            _ptr(dB), n, _ptr(dA), _stream()))
        return dB, dA

    def backward_fused(self, B, dC) -> bool:
        """Whether backward(B, dC) with both gradients takes the one-pass
        path (dB and dA from one gather of each dC row)."""
        B = self._dense(B, self.k, "B")
        n = B.shape[1]
        self._dense(dC, self.m, "dC", cols=n, dtype=self.out_dtype)
        f = ctypes.c_int32()
        _check(library().hybrid_spmm_backward_fused(self.handle, n, _ptr(B), _ld(B), _ptr(dC), _ld(dC),
                                                    None, n, ctypes.byref(f)))
        return bool(f.value)

    def update_values(self, vals):
        if not isinstance(vals, torch.Tensor):
            raise HspmmError(-1, "vals must be a torch tensor")
        v = vals if vals.dtype in DTYPES else vals.to(torch.float64)
        v = v.to(self.device).contiguous()
        if v.dim() != 1 or v.numel() != self.nnz_input:
            raise HspmmError(-1, "vals must be a vector of nnz entries")
        _check(library().hybrid_spmm_update_values(self.handle, _ptr(v), DTYPES[v.dtype], _stream()))
        self._note_packed(vals, v)

    def calibrate(self, B, reps: int = 5) -> dict:
        """Fit the quadratic model (Eq. 2) of forward throughput over
        workgroup partitions of the two parts and apply its argmax (Eq. 3)
        when it measures at least as fast as the default launch."""
        B = self._dense(B, self.k, "B")
        n = B.shape[1]
        C = torch.empty((self.m, n), dtype=self.out_dtype, device=self.device)
        ci = _lib.CalibInfo()
        ci.struct_size = ctypes.sizeof(_lib.CalibInfo)
        _check(library().hybrid_spmm_calibrate(self.handle, n, _ptr(B), B.stride(0) if self.k else n,
                                               _ptr(C), n, int(reps), ctypes.byref(ci), _stream()))
        k = ci.n_candidates
        return {"T": ci.T, "x_max": ci.x_max, "y_max": ci.y_max, "cand_x": list(ci.cand_x[:k]), "cand_y": list(ci.cand_y[:k]),
                "cand_gflops": list(ci.cand_gflops[:k]), "coef": list(ci.coef),
                "best": (ci.best_x, ci.best_y), "best_gflops": ci.best_gflops,
                "default_gflops": ci.default_gflops, "applied": bool(ci.applied)}

    # -- inspection --------------------------------------------------------
    def info(self) -> dict:
        i = _lib.PlanInfo()
        i.struct_size = ctypes.sizeof(_lib.PlanInfo)
        _check(library().hybrid_spmm_plan_info(self.handle, ctypes.byref(i)))
        return {name: getattr(i, name) for name, _ in _lib.PlanInfo._fields_ if name != "struct_size"}

    def export(self, field: str, which: int = 0) -> np.ndarray:
        """Copy one array of the built format to the host (canonical layout)."""
        L = library()
        f = _lib.FIELDS[field]
        nbytes = ctypes.c_int64()
        _check(L.hybrid_spmm_export(self.handle, which, f, None, 0, ctypes.byref(nbytes)))
        if field in ("csr_val", "blk_val"):
            ct = self.compute if which == 0 else (_lib.F64 if self.compute == _lib.F64 else _lib.F32)
            dt = _NP_OF[ct]
        elif field == "rb_scale":
            dt = np.float64
        # the group fields (int32) fall through to the default
        else:
            dt = np.int32
        buf = np.empty(nbytes.value // np.dtype(dt).itemsize, dtype=dt)
        if nbytes.value:
            _check(L.hybrid_spmm_export(self.handle, which, f, buf.ctypes.data_as(ctypes.c_void_p),
                                        nbytes.value, ctypes.byref(nbytes)))
        return buf


class _HybridSpMM(torch.autograd.Function):
    @staticmethod
    def forward(ctx, vals, B, plan):
        # learnable values change every step and are re-packed; a static A
        # (the tensor the plan last read, unchanged since) is not
        if vals.requires_grad or not plan.holds_values_of(vals):
            plan.update_values(vals)
        C = plan.run(B)
        ctx.plan = plan
        ctx.token = plan._pack_token
        ctx.save_for_backward(vals, B)
        ctx.vals_dtype = vals.dtype
        return C

    @staticmethod
    def backward(ctx, dC):
        vals, B = ctx.saved_tensors
        plan = ctx.plan
        need_dA, need_dB = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        if need_dB and plan._pack_token != ctx.token:
            # the plan was re-packed since this forward call (another call
            # with other values, or update_values): dB = A^T dC needs the
            # values this call multiplied with
            plan.update_values(vals)
            ctx.token = plan._pack_token
        dC = dC.to(plan.out_dtype)
        if dC.dim() == 2 and dC.numel() and (dC.stride(1) != 1 or dC.stride(0) < dC.shape[1]):
            dC = dC.contiguous()  # e.g. the broadcast gradient of a sum
        dB, dA = plan.backward(B, dC, need_dB=need_dB, need_dA=need_dA)
        if dA is not None:
            dA = dA.to(ctx.vals_dtype)
        if dB is not None:
            dB = dB.to(B.dtype)
        return dA, dB, None


def spmm(plan: Plan, vals: torch.Tensor, B: torch.Tensor) -> torch.Tensor:
    """C = A(vals) B with gradients for vals (SDDMM) and B (A^T dC)."""
    return _HybridSpMM.apply(vals, B, plan)
