"""GPU parity of the window-by-window encoding (matrices of 1 GiB or more)
against the oracle's encoding, bit for bit, through the C ABI.

A 16384 x 8192 FP64 matrix is exactly 1 GiB: the library splits it into 8
windows of 2048 rows (128 MiB each).  The cases cover unique cells (plain
stores) with FP32 and FP64 values, the transposed placement (B -> Y),
duplicate cells with integer values (atomic adds, whose sums are then exact)
and out-of-range records (counted once), and a 0/1 encoding without values.
Each is also checked against the one-pass fill of the same records.
"""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2112_07552_amd import _lib, ops
from paper_2112_07552_amd import workloads as wl

from .gpu_util import cuda_or_skip

pytestmark = pytest.mark.gpu

ROWS, COLS = 16384, 8192
WINDOWS = 8


def _unique_cells(n, rows, cols, seed, dev):
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    cells = torch.randperm(rows * cols, generator=g, device=dev)[:n]
    return (cells // cols).to(torch.int32), (cells % cols).to(torch.int32)


def _traced_encode(group, key, val, rows, cols, transpose, unique):
    """ops.encode with the launch trace on: the matrix and the window count
    of its encode launch record."""
    recs = (_lib.tcu_launch_record * 4)()
    rt = C.CDLL("libamdhip64.so")
    for r in recs:
        a, b = C.c_void_p(), C.c_void_p()
        assert rt.hipEventCreate(C.byref(a)) == 0 and rt.hipEventCreate(C.byref(b)) == 0
        r.begin, r.end = a.value, b.value
    cnt = C.c_int32(0)
    L = _lib.load()
    L.tcu_trace_launches(recs, 4, C.byref(cnt))
    try:
        need = L.tcu_encode_workspace_bytes(C.byref(ops.make_relation(group, key, val, unique)),
                                            rows, cols)
        ws = ops.alloc_workspace(need, group.device)
        X = ops.encode(group, key, val, rows, cols, transpose=transpose, ws=ws, unique=unique)
        st, info = ops.sync_status(ws)
    finally:
        L.tcu_trace_launches(None, 0, None)
    planes = [r.planes for r in recs[:cnt.value] if r.kernel == _lib.TCU_KERNEL_ENCODE]
    for r in recs:
        rt.hipEventDestroy(C.c_void_p(r.begin))
        rt.hipEventDestroy(C.c_void_p(r.end))
    return X, planes, st, info


@pytest.mark.parametrize("dtype,transpose", [(torch.float32, False), (torch.float64, True)])
def test_windowed_encode_unique_cells(orc, dtype, transpose):
    dev = cuda_or_skip()
    n = 1 << 24
    r, c = _unique_cells(n, ROWS, COLS, 11 + int(transpose), dev)
    v = wl.draw_values("uniform", n, 12, 0, device=dev).to(dtype)
    # transpose: the records are B's (key = row, group = column)
    group, key = (c, r) if transpose else (r, c)
    X, planes, st, info = _traced_encode(group, key, v, ROWS, COLS, transpose, True)
    assert st == 0 and planes == [WINDOWS]
    rr, cc = r.cpu().numpy(), c.cpu().numpy()
    Xo, skipped = orc.encode(rr, cc, v.cpu().to(torch.float64).numpy(), ROWS, COLS)
    assert skipped == 0
    assert np.array_equal(X.cpu().numpy(), Xo)
    X1 = ops.encode(group, key, v, ROWS, COLS, transpose=transpose, unique=True, windows=False)
    assert torch.equal(X, X1)


def test_windowed_encode_duplicates_and_skips(orc):
    """Random cells with repeats, integer values (sums exact in any order),
    1% of the records out of range."""
    dev = cuda_or_skip()
    n = 1 << 24
    R = wl.random_relation(n, ROWS, COLS, 13, 1, values="int", lo=-1000, hi=1000, device=dev,
                           bad_fraction=0.01)
    X, planes, st, info = _traced_encode(R.group, R.key, R.val, ROWS, COLS, False, False)
    assert planes == [WINDOWS]
    Xo, skipped = orc.encode(R.group.cpu().numpy(), R.key.cpu().numpy(), R.val.cpu().numpy(),
                             ROWS, COLS)
    assert skipped > 0
    assert st == _lib.TCU_ERR_KEY_RANGE and info["skipped_a"] == skipped
    assert np.array_equal(X.cpu().numpy(), Xo)


def test_windowed_encode_without_values(orc):
    """A 0/1 (multiplicity) encoding: every in-range record adds one."""
    dev = cuda_or_skip()
    n = 1 << 23
    R = wl.random_relation(n, ROWS, COLS, 14, 1, device=dev)
    X, planes, st, _ = _traced_encode(R.group, R.key, None, ROWS, COLS, False, False)
    assert st == 0 and planes == [WINDOWS]
    Xo, _ = orc.encode(R.group.cpu().numpy(), R.key.cpu().numpy(), None, ROWS, COLS)
    assert np.array_equal(X.cpu().numpy(), Xo)


def test_small_matrix_keeps_one_pass():
    dev = cuda_or_skip()
    R = wl.random_relation(1 << 16, 1024, 1024, 15, 1, device=dev)
    _, planes, st, _ = _traced_encode(R.group, R.key, R.val, 1024, 1024, False, False)
    assert st == 0 and planes == [1]
