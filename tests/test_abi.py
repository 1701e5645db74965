"""The C-ABI library loads and exports every symbol that include/hspmm.h
declares; struct layouts of the binding match the header.  CPU only: no
compute call is made."""
import ctypes
import re
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parent.parent
HEADER = ROOT / "include" / "hspmm.h"


def declared_functions():
    text = HEADER.read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hybrid_spmm_\w+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for need in ("hybrid_spmm_plan", "hybrid_spmm_run", "hybrid_spmm_backward"):
        assert need in names


def test_library_exports_every_declared_symbol():
    from paper_2511_08158_amd import _lib
    if not _lib.LIB_PATH.exists():
        pytest.fail("libhspmm.so not built (run __graft_entry__.build())")
    L = ctypes.CDLL(str(_lib.LIB_PATH))
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    assert set(_lib.EXPORTED) == set(declared_functions())


def test_version_and_last_error_need_no_gpu():
    from paper_2511_08158_amd import _lib
    L = _lib.load()
    assert b"gfx950" in L.hybrid_spmm_version()
    assert L.hybrid_spmm_last_error() == b""


def test_null_handles_are_rejected_without_a_gpu():
    """Argument errors are detected on the host before any device call."""
    from paper_2511_08158_amd import _lib
    L = _lib.load()
    assert L.hybrid_spmm_run(None, 4, None, 4, None, 4, None) == -1
    assert b"NULL" in L.hybrid_spmm_last_error()
    assert L.hybrid_spmm_plan(None, 1, 1, 0, None, None, None, 1, None, None) == -1
    out = ctypes.c_void_p()
    assert L.hybrid_spmm_plan(ctypes.byref(out), -1, 1, 0, None, None, None, 1, None, None) == -1
    assert L.hybrid_spmm_plan(ctypes.byref(out), 4, 4, 0, None, None, None, 1, None, None) == -1
    opts = _lib.PlanOpts(ctypes.sizeof(_lib.PlanOpts) + 1, 1, 0, 16, -1, 128, 0, 0)
    dummy = ctypes.c_void_p(16)  # never dereferenced: rejected before use
    assert L.hybrid_spmm_plan(ctypes.byref(out), 4, 4, 0, dummy, None, None, 1, ctypes.byref(opts), None) == -1
    assert b"struct_size" in L.hybrid_spmm_last_error()
    assert L.hybrid_spmm_plan(ctypes.byref(out), 4, 4, 0, dummy, None, None, 9, None, None) == -3
    L.hybrid_spmm_destroy(None)


def test_struct_sizes_match_header():
    """Offsets the binding uses equal the C compiler's layout of the header."""
    import subprocess
    import tempfile
    from paper_2511_08158_amd import _lib
    src = (
        '#include <stdio.h>\n#include <stddef.h>\n#include "hspmm.h"\n'
        'int main(){printf("%zu %zu %zu %zu %zu %zu %zu\\n", sizeof(hspmm_plan_opts), sizeof(hspmm_plan_info),'
        ' offsetof(hspmm_plan_opts, max_workspace_bytes), offsetof(hspmm_plan_info, plan_ms),'
        ' offsetof(hspmm_plan_info, t_nblk), sizeof(hspmm_calib_info), offsetof(hspmm_calib_info, applied));'
        ' return 0;}\n')
    with tempfile.TemporaryDirectory() as d:
        c = Path(d) / "t.c"
        c.write_text(src)
        exe = Path(d) / "t"
        subprocess.run(["gcc", "-I", str(ROOT / "include"), str(c), "-o", str(exe)], check=True)
        got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    assert got == [ctypes.sizeof(_lib.PlanOpts), ctypes.sizeof(_lib.PlanInfo),
                   _lib.PlanOpts.max_workspace_bytes.offset, _lib.PlanInfo.plan_ms.offset,
                   _lib.PlanInfo.t_nblk.offset, ctypes.sizeof(_lib.CalibInfo), _lib.CalibInfo.applied.offset]


def test_binding_operand_checks_on_the_host():
    """The binding rejects a dense operand of the wrong device, dtype, shape
    or layout before any pointer reaches the C ABI (host tensors stand in
    for device ones: the check compares devices, no GPU is touched)."""
    import torch

    import paper_2511_08158_amd as hs
    cpu = torch.device("cpu")
    ok = torch.zeros((5, 3))
    assert hs.check_dense(ok, 5, 3, torch.float32, cpu, "X") is ok
    assert hs.check_dense(torch.zeros((8, 6))[:, :3], 8, None, torch.float32, cpu, "X") is not None
    bad = [
        (ok, 5, 3, torch.float32, torch.device("cuda:0")),          # device
        (ok, 5, 3, torch.float64, cpu),                             # dtype
        (ok, 4, 3, torch.float32, cpu),                             # rows
        (ok, 5, 4, torch.float32, cpu),                             # columns
        (torch.zeros((3, 5)).t(), 5, 3, torch.float32, cpu),        # column-major
        (torch.zeros(15), 5, 3, torch.float32, cpu),                # not a matrix
        (torch.zeros((1, 3)).expand(5, 3), 5, 3, torch.float32, cpu),  # rows overlap
        (ok.numpy(), 5, 3, torch.float32, cpu),                     # not a tensor
    ]
    for X, r, c, dt, dv in bad:
        with pytest.raises(hs.HspmmError):
            hs.check_dense(X, r, c, dt, dv, "X")
