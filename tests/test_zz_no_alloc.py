"""tcu_join_agg_fwd_noalloc (the forward with the library's own device
array as workspace) against tcu_join_agg_fwd on a caller workspace, through
the C ABI: two calls in a row on one device, the second smaller, C, the pair
count and the status block compared.  Both forms run the same kernels in the
same order: with unique cells (plain stores) the results agree bit for bit;
with duplicate cells the encodings add in FP64 atomics, whose rounding
depends on the order, so there C agrees within 1e-12 of (|X||Y|)[g,h]
(the oracle's product of the absolute values)."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2112_07552_amd import _lib, ops
from paper_2112_07552_amd import workloads as wl
from tests.gpu_util import abs_rel, cuda_or_skip, err_cw, to_orc


def _rel(R, unique):
    return ops.make_relation(R.group, R.key, R.val, unique=unique)


def _regular(L, A, B, M, K, N, prec, tol, with_count, dev, sp):
    nb = L.tcu_workspace_bytes(C.byref(A), C.byref(B), M, K, N, prec,
                               _lib.TCU_WS_COUNT if with_count else 0)
    ws = ops.alloc_workspace(nb, dev)
    Cm = torch.full((M, N), float("nan"), dtype=torch.float64, device=dev)
    cnt = torch.full((M, N), -7, dtype=torch.int32, device=dev) if with_count else None
    _lib.check(L.tcu_join_agg_fwd(C.byref(A), C.byref(B), M, K, N, prec, tol,
                                  C.c_void_p(Cm.data_ptr()),
                                  None if cnt is None else C.c_void_p(cnt.data_ptr()),
                                  C.c_void_p(ws.data_ptr()), ws.numel(), sp), "fwd")
    st, info = ops.sync_status(ws)
    return Cm, cnt, st, info


def _noalloc(L, A, B, M, K, N, prec, tol, with_count, dev, sp):
    Cm = torch.full((M, N), float("nan"), dtype=torch.float64, device=dev)
    cnt = torch.full((M, N), -7, dtype=torch.int32, device=dev) if with_count else None
    status = torch.full((256,), 0xAB, dtype=torch.uint8, device=dev)
    _lib.check(L.tcu_join_agg_fwd_noalloc(C.byref(A), C.byref(B), M, K, N, prec, tol,
                                          C.c_void_p(Cm.data_ptr()),
                                          None if cnt is None else C.c_void_p(cnt.data_ptr()),
                                          C.c_void_p(status.data_ptr()), sp), "fwd_noalloc")
    info = _lib.tcu_status_info()
    st = L.tcu_sync_status(C.c_void_p(status.data_ptr()), sp, C.byref(info))
    return Cm, cnt, st, {"flags": info.flags, "slices": info.slices,
                         "skipped_a": info.skipped_a, "skipped_b": info.skipped_b,
                         "bits": info.bits, "need": info.need, "exceptions": info.exceptions}


CASES = [
    # (name, M, K, N, precision, relation maker): the largest FP64 shape the
    # array holds first, then smaller ones with duplicates, skipped records,
    # counts and the residue form
    ("fp64_max_2048", 2048, 2048, 2048, "fp64", "dense"),
    ("fp64_dups_bad_count", 300, 257, 190, "fp64", "random_bad"),
    ("crt_i8_small", 200, 160, 120, "crt_i8", "dense"),
    ("fp64_smaller", 97, 64, 33, "fp64", "random"),
]


def _inputs(kind, M, K, N, seed, dev):
    if kind == "dense":
        A, B = wl.mm_query(M, K, N, seed=seed, device=dev)
        return A, B, True
    bad = 0.02 if kind == "random_bad" else 0.0
    A = wl.random_relation(3 * M * K // 2, M, K, seed, 1, device=dev, bad_fraction=bad)
    B = wl.random_relation(3 * K * N // 2, N, K, seed, 2, device=dev, bad_fraction=bad)
    return A, B, False


@pytest.mark.gpu
def test_noalloc_matches_workspace_forward_on_consecutive_calls(orc):
    dev = cuda_or_skip()
    L = _lib.load()
    sp = C.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    for i, (name, M, K, N, precision, kind) in enumerate(CASES):
        print(f"noalloc case {name}: M={M} K={K} N={N} {precision}", flush=True)
        A, B, unique = _inputs(kind, M, K, N, 40 + i, dev)
        rA, rB = _rel(A, unique), _rel(B, unique)
        prec = ops.PRECISIONS[precision]
        tol = 1e-12 if precision != "fp64" else 0.0
        with_count = kind == "random_bad"
        nb = L.tcu_workspace_bytes(C.byref(rA), C.byref(rB), M, K, N, prec, 0)
        assert 0 < nb <= _lib.TCU_NOALLOC_MAX_BYTES, name
        C0, n0, st0, i0 = _regular(L, rA, rB, M, K, N, prec, tol, with_count, dev, sp)
        C1, n1, st1, i1 = _noalloc(L, rA, rB, M, K, N, prec, tol, with_count, dev, sp)
        torch.cuda.synchronize()
        assert st1 == st0, name
        assert i1 == i0, name
        if kind == "random_bad":
            assert st1 == _lib.TCU_ERR_KEY_RANGE and i1["skipped_a"] > 0 and i1["skipped_b"] > 0
        else:
            assert st1 == _lib.TCU_OK, name
        a, b = C0.cpu().numpy(), C1.cpu().numpy()
        assert np.isfinite(b).all(), name
        if unique:
            assert np.array_equal(a.view(np.int64), b.view(np.int64)), name
        else:
            S, _, _ = orc.join_agg(abs_rel(orc, to_orc(orc, A)), abs_rel(orc, to_orc(orc, B)),
                                   M, K, N)
            assert err_cw(b, a, S) <= 1e-12, name
        if with_count:
            assert torch.equal(n0, n1), name
            assert int(n1.min()) >= 0


@pytest.mark.gpu
def test_noalloc_rejects_shapes_beyond_its_array():
    dev = cuda_or_skip()
    L = _lib.load()
    sp = C.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    A, B = wl.mm_query(8, 8, 8, seed=1, device=dev)
    rA, rB = _rel(A, True), _rel(B, True)
    Cm = torch.zeros((2200, 2200), dtype=torch.float64, device=dev)
    assert L.tcu_join_agg_fwd_noalloc(C.byref(rA), C.byref(rB), 2200, 2048, 2200, 0, 0.0,
                                      C.c_void_p(Cm.data_ptr()), None, None,
                                      sp) == _lib.TCU_ERR_WORKSPACE
    assert bool((Cm == 0).all())
