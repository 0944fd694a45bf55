"""Host-side checks of libtcudb.so that need no GPU.

The library must load, export every entry point include/tcudb.h declares,
size workspaces, and reject invalid arguments before touching the device.
"""
import ctypes as C
import os
import re

import pytest

from paper_2112_07552_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "tcudb.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tcu_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def test_exports_every_declared_symbol(lib):
    names = header_functions()
    assert len(names) >= 8
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(_lib.EXPORTS)


def test_version_and_status_strings(lib):
    assert b"gfx950" in lib.tcu_version()
    for code in range(-7, 1):
        s = lib.tcu_status_str(code).decode()
        assert s and s != "unknown status"
    assert lib.tcu_status_str(-99).decode() == "unknown status"


def rel(n, dtype=_lib.TCU_F64, ptr=0x1000, flags=0):
    return _lib.tcu_relation(n, ptr if n else None, ptr if n else None, ptr, dtype, flags)


def test_workspace_bytes(lib):
    A, B = rel(10), rel(10)
    M, K, N = 100, 37, 50
    fwd = lib.tcu_workspace_bytes(C.byref(A), C.byref(B), M, K, N, 0, 0)
    align = lambda x: (x + 255) // 256 * 256
    assert fwd == 256 + align(M * K * 8) + align(K * N * 8)
    bwd = lib.tcu_workspace_bytes(C.byref(A), C.byref(B), M, K, N, 0, _lib.TCU_WS_BACKWARD)
    # backward: separate dX (M x K) and dY (K x N) buffers
    assert bwd == fwd + align(M * K * 8) + align(K * N * 8)
    assert lib.tcu_workspace_bytes(C.byref(A), C.byref(B), 0, K, N, 0, 0) == 0
    assert lib.tcu_workspace_bytes(C.byref(A), C.byref(B), M, K, N, 7, 0) == 0


def test_fp64_workspace_holds_split_partials(lib):
    """FP64 products with few output tiles split their contraction: at 1024^3
    (64 tiles of 128 x 128) four 256-deep parts, each a 1024 x 1024 FP64
    partial product in the workspace; at 4096^3 (1024 tiles) none."""
    A, B = rel(1 << 20), rel(1 << 20)
    mb = 1024 * 1024 * 8
    assert lib.tcu_workspace_bytes(C.byref(A), C.byref(B), 1024, 1024, 1024, 0, 0) == \
        256 + 2 * mb + 4 * mb
    assert lib.tcu_gemm_f64_workspace_bytes(1024, 1024, 1024) == 4 * mb
    assert lib.tcu_workspace_bytes(C.byref(A), C.byref(B), 1024, 1024, 1024, 0,
                                   _lib.TCU_WS_BACKWARD) == 256 + 4 * mb + 4 * mb
    big = lib.tcu_workspace_bytes(None, None, 4096, 4096, 4096, 0, 0)
    assert big == 256 + 2 * 4096 * 4096 * 8


def _window_scratch(n, rows, cols, vb):
    """The window-by-window encoding's scratch as documented in encode.hip:
    window totals and offsets, a run table of windows x workgroups (8192
    records each), and per slot (records plus up to 31 per run) a 4-byte
    cell offset and a value."""
    align = lambda x: (x + 255) // 256 * 256
    wrows = min(max(1, (128 << 20) // (cols * 8)), rows)
    wrows = max(wrows, -(-rows // 1024))
    nw = -(-rows // wrows)
    nwg = -(-n // 8192)
    table = nw * nwg
    slots = n + 31 * table
    return align((2 * 1024 + 1) * 8) + align(4 * table) + align(4 * slots) + align(vb * slots)


def test_encode_window_scratch_sizes(lib):
    """Encodings of 1 GiB or more get the partition's scratch; smaller ones
    none (a one-pass fill needs only the status block)."""
    n = 1 << 30
    for dtype, vb in ((_lib.TCU_F32, 4), (_lib.TCU_F64, 8)):
        R = rel(n, dtype)
        assert lib.tcu_encode_workspace_bytes(C.byref(R), 32768, 32768) == \
            256 + _window_scratch(n, 32768, 32768, vb)
    # 64 windows of 512 rows, 131072 workgroups: 8 GiB of slots for FP32 values
    assert _window_scratch(n, 32768, 32768, 4) < 10.5 * 2 ** 30
    # no values (a 0/1 encoding): cell offsets only
    R0 = _lib.tcu_relation(n, 0x1000, 0x1000, None, _lib.TCU_F64, 0)
    assert lib.tcu_encode_workspace_bytes(C.byref(R0), 32768, 32768) == \
        256 + _window_scratch(n, 32768, 32768, 0)
    # below 1 GiB: one pass, status block only
    R = rel(1 << 24)
    assert lib.tcu_encode_workspace_bytes(C.byref(R), 4096, 4096) == 256
    assert lib.tcu_encode_workspace_bytes(C.byref(R), 8192, 16383) == 256
    assert lib.tcu_encode_workspace_bytes(C.byref(R), 16384, 8192) == \
        256 + _window_scratch(1 << 24, 16384, 8192, 8)
    # a tall matrix is cut into at most 1024 windows
    tall = (1 << 31) - 1
    assert lib.tcu_encode_workspace_bytes(C.byref(R), tall, 128) == \
        256 + _window_scratch(1 << 24, tall, 128, 8)
    assert lib.tcu_encode_workspace_bytes(C.byref(R), 0, 8192) == 0
    # the operator's workspace holds the larger operand's scratch when given
    # the relations, and none without them
    A, B = rel(n, _lib.TCU_F32), rel(n // 2, _lib.TCU_F64)
    M = K = N = 32768
    with_rel = lib.tcu_workspace_bytes(C.byref(A), C.byref(B), M, K, N, 3, _lib.TCU_WS_BACKWARD)
    without = lib.tcu_workspace_bytes(None, None, M, K, N, 3, _lib.TCU_WS_BACKWARD)
    assert with_rel - without == max(_window_scratch(n, M, K, 4), _window_scratch(n // 2, K, N, 8))
    small_a, small_b = rel(1 << 24), rel(1 << 24)
    assert lib.tcu_workspace_bytes(C.byref(small_a), C.byref(small_b), 4096, 4096, 4096, 0, 0) == \
        lib.tcu_workspace_bytes(None, None, 4096, 4096, 4096, 0, 0)


def test_argument_errors_return_before_launch(lib):
    A, B = rel(10), rel(10)
    cbuf = C.c_void_p(0x2000)
    # NULL C
    assert lib.tcu_join_agg_fwd(C.byref(A), C.byref(B), 4, 4, 4, 0, 0.0, None, None,
                                C.c_void_p(0x100000), 1 << 20, None) == _lib.TCU_ERR_ARG
    # bad shapes
    assert lib.tcu_join_agg_fwd(C.byref(A), C.byref(B), 0, 4, 4, 0, 0.0, cbuf, None,
                                C.c_void_p(0x100000), 1 << 20, None) == _lib.TCU_ERR_ARG
    # negative record count
    bad = rel(10); bad.n = -1
    assert lib.tcu_join_agg_fwd(C.byref(bad), C.byref(B), 4, 4, 4, 0, 0.0, cbuf, None,
                                C.c_void_p(0x100000), 1 << 20, None) == _lib.TCU_ERR_ARG
    # NULL key column with records
    nok = _lib.tcu_relation(5, 0x1000, None, None, 0)
    assert lib.tcu_join_agg_fwd(C.byref(nok), C.byref(B), 4, 4, 4, 0, 0.0, cbuf, None,
                                C.c_void_p(0x100000), 1 << 20, None) == _lib.TCU_ERR_ARG
    # bad dtype
    bd = rel(10, dtype=5)
    assert lib.tcu_join_agg_fwd(C.byref(bd), C.byref(B), 4, 4, 4, 0, 0.0, cbuf, None,
                                C.c_void_p(0x100000), 1 << 20, None) == _lib.TCU_ERR_ARG
    # workspace: NULL, misaligned, too small
    assert lib.tcu_join_agg_fwd(C.byref(A), C.byref(B), 4, 4, 4, 0, 0.0, cbuf, None,
                                None, 1 << 20, None) == _lib.TCU_ERR_WORKSPACE
    assert lib.tcu_join_agg_fwd(C.byref(A), C.byref(B), 4, 4, 4, 0, 0.0, cbuf, None,
                                C.c_void_p(0x100010), 1 << 20, None) == _lib.TCU_ERR_WORKSPACE
    assert lib.tcu_join_agg_fwd(C.byref(A), C.byref(B), 4, 4, 4, 0, 0.0, cbuf, None,
                                C.c_void_p(0x100000), 300, None) == _lib.TCU_ERR_WORKSPACE
    # unknown relation flag
    bf = rel(10, flags=4)
    assert lib.tcu_join_agg_fwd(C.byref(bf), C.byref(B), 4, 4, 4, 0, 0.0, cbuf, None,
                                C.c_void_p(0x100000), 1 << 20, None) == _lib.TCU_ERR_ARG
    # backward: NULL dC, unknown flag, small workspace
    assert lib.tcu_join_agg_bwd(C.byref(A), C.byref(B), 4, 4, 4, 0, 0.0, None, cbuf, cbuf, 0,
                                C.c_void_p(0x100000), 1 << 20, None) == _lib.TCU_ERR_ARG
    assert lib.tcu_join_agg_bwd(C.byref(A), C.byref(B), 4, 4, 4, 0, 0.0, cbuf, cbuf, cbuf, 2,
                                C.c_void_p(0x100000), 1 << 20, None) == _lib.TCU_ERR_ARG
    fwd_only = lib.tcu_workspace_bytes(C.byref(A), C.byref(B), 64, 64, 64, 0, 0)
    assert lib.tcu_join_agg_bwd(C.byref(A), C.byref(B), 64, 64, 64, 0, 0.0, cbuf, cbuf, cbuf, 0,
                                C.c_void_p(0x100000), fwd_only, None) == _lib.TCU_ERR_WORKSPACE
    # gemm: bad transpose flag, negative size, short leading dimension
    assert lib.tcu_gemm_f64(2, 0, 4, 4, 4, cbuf, 4, cbuf, 4, cbuf, 4, None) == _lib.TCU_ERR_ARG
    assert lib.tcu_gemm_f64(0, 0, -1, 4, 4, cbuf, 4, cbuf, 4, cbuf, 4, None) == _lib.TCU_ERR_ARG
    assert lib.tcu_gemm_f64(0, 0, 4, 4, 8, cbuf, 4, cbuf, 4, cbuf, 4, None) == _lib.TCU_ERR_ARG
    assert lib.tcu_gemm_f64(0, 0, 4, 4, 4, cbuf, 4, cbuf, 4, cbuf, 3, None) == _lib.TCU_ERR_ARG
    # m == 0: nothing to do, nothing launched
    assert lib.tcu_gemm_f64(0, 0, 0, 4, 4, None, 4, None, 4, None, 4, None) == _lib.TCU_OK
    # encode: bad transpose, NULL out
    assert lib.tcu_encode(C.byref(A), 3, 4, 4, cbuf, C.c_void_p(0x100000), 256, None) == _lib.TCU_ERR_ARG
    assert lib.tcu_encode(C.byref(A), 0, 4, 4, None, C.c_void_p(0x100000), 256, None) == _lib.TCU_ERR_ARG
    assert lib.tcu_sync_status(None, None, None) == _lib.TCU_ERR_WORKSPACE


MODULI = [256, 255, 253, 251, 247, 241, 239, 233, 229, 227, 223, 217, 211, 199, 197]


def _plan(lib, p, k, tol, need, u):
    bits = C.c_int32(-1)
    r = lib.tcu_mixed_plan(p, k, tol, need, u, C.byref(bits))
    return r, bits.value


def test_mixed_plan_host_only(lib):
    """Step a0's host part: the plan from a product's certificate."""
    import math
    for p in (_lib.TCU_PREC_SPLIT_BF16, _lib.TCU_PREC_SPLIT_I8):
        assert _plan(lib, p, 4096, 1e-12, 0, 1.0)[0] == 1        # all-zero product
        for need in range(1, 9):
            assert _plan(lib, p, 4096, 1e-12, need, 100.0)[0] == need
        assert _plan(lib, p, 4096, 1e-12, 9, 1.0)[0] == _lib.TCU_ERR_INFEASIBLE
        assert _plan(lib, p, 4096, 1e-12, 255, 1.0)[0] == _lib.TCU_ERR_INFEASIBLE
    crt = _lib.TCU_PREC_CRT_I8
    # the modulus count: the smallest L with prod m_i > 2 |P| (1 + 2^-38) for
    # every |P| <= 2^(2b) U, U = min(max(u, 1), k) -- the reconstruction
    # rounds S / M to within 2^-40 of itself -- checked in exact integers
    # (the library's 1e-6-bit margin is a factor 1 + 6.9e-7)
    from fractions import Fraction
    for k, need, u in ((4096, 42, 4096.0), (4096, 46, 136.0), (32768, 48, 325.0),
                       (32768, 51, 370.2), (1, 2, 0.9), (257, 53, 257.0), (100, 20, 1e9),
                       (5000, 0, 0.0), (3570, 41, 3570.0)):
        b = max(need, 1)
        U = Fraction(min(max(u, 1.0), float(k)))
        bound = 2 * 2 ** (2 * b) * U * (1 + Fraction(1, 2 ** 38))
        want = next((L for L in range(1, 16) if math.prod(MODULI[:L]) > bound), None)
        got, bits = _plan(lib, crt, k, 1e-12, need, u)
        if want is None:
            assert got == _lib.TCU_ERR_INFEASIBLE
        else:
            # the margin can only add a modulus when prod m_i sits within a
            # factor 1 + 6.9e-7 of the bound, which none of these cases does
            assert (got, bits) == (want, b), (k, need, u)
            assert math.prod(MODULI[:got]) > bound
    # a case the former M > 4 |P| rule planned one modulus wider: 2^(2*20+1) * 100
    # lies below the first six moduli's product, 2^(2*20+2) * 100 above it
    assert _plan(lib, crt, 100, 1e-12, 20, 1e9)[0] == 6
    # every modulus count is reachable
    seen = ({_plan(lib, crt, 131071, 1e-12, b, 131071.0)[0] for b in range(1, 54)} |
            {_plan(lib, crt, 1, 1e-12, b, 1.0)[0] for b in range(1, 54)})
    assert sorted(seen - {_lib.TCU_ERR_INFEASIBLE}) == list(range(1, 16))
    assert _plan(lib, crt, 4096, 1e-12, 54, 1.0)[0] == _lib.TCU_ERR_INFEASIBLE
    assert _plan(lib, crt, 131072, 1e-12, 10, 1.0)[0] == _lib.TCU_ERR_INFEASIBLE  # int32 sums
    for p in (crt, _lib.TCU_PREC_SPLIT_I8):
        assert _plan(lib, p, 64, 2.0 ** -51, 3, 1.0)[0] == _lib.TCU_ERR_INFEASIBLE  # tol floor
        assert _plan(lib, p, 64, 0.0, 3, 1.0) == _plan(lib, p, 64, 1e-12, 3, 1.0)
        assert _plan(lib, p, 0, 1e-9, 3, 1.0)[0] == _lib.TCU_ERR_ARG
    assert _plan(lib, _lib.TCU_PREC_FP64, 64, 1e-9, 3, 1.0)[0] == _lib.TCU_ERR_ARG


def test_split_argument_errors(lib):
    buf = C.c_void_p(0x100000)
    # bad axis, S out of range, padding not a multiple of 128 / 64, FP64 precision
    assert lib.tcu_split(buf, 10, 10, 10, 2, 2, 3, buf, 128, 64, buf, buf, 1 << 20, None) == _lib.TCU_ERR_ARG
    assert lib.tcu_split(buf, 10, 10, 10, 0, 2, 9, buf, 128, 64, buf, buf, 1 << 20, None) == _lib.TCU_ERR_ARG
    assert lib.tcu_split(buf, 10, 10, 10, 0, 2, 3, buf, 100, 64, buf, buf, 1 << 20, None) == _lib.TCU_ERR_ARG
    assert lib.tcu_split(buf, 10, 10, 10, 0, 2, 3, buf, 128, 60, buf, buf, 1 << 20, None) == _lib.TCU_ERR_ARG
    assert lib.tcu_split(buf, 10, 10, 10, 0, 0, 3, buf, 128, 64, buf, buf, 1 << 20, None) == _lib.TCU_ERR_ARG
    assert lib.tcu_split(buf, 10, 10, 5, 0, 2, 3, buf, 128, 64, buf, buf, 1 << 20, None) == _lib.TCU_ERR_ARG
    # workspace too small for the line maxima
    assert lib.tcu_split(buf, 10, 10, 10, 0, 2, 3, buf, 128, 64, buf, buf, 300, None) == _lib.TCU_ERR_WORKSPACE


def test_mixed_forms_workspace_and_infeasible(lib):
    A, B = rel(10), rel(10)
    fp64 = lib.tcu_workspace_bytes(C.byref(A), C.byref(B), 300, 200, 100, 0, 0)
    i8 = lib.tcu_workspace_bytes(C.byref(A), C.byref(B), 300, 200, 100, 2, 0)
    bf = lib.tcu_workspace_bytes(C.byref(A), C.byref(B), 300, 200, 100, 1, 0)
    assert fp64 < i8 < bf
    # an unreachable tolerance is refused before any launch
    cbuf = C.c_void_p(0x2000)
    assert lib.tcu_join_agg_fwd(C.byref(A), C.byref(B), 4, 4, 4, 2, 1e-18, cbuf, None,
                                C.c_void_p(0x100000), 1 << 30, None) == _lib.TCU_ERR_INFEASIBLE


def test_queries_bsr_nonzero_host_argument_errors(lib):
    """Argument checks of the later entry points, all before any HIP call."""
    buf = (C.c_double * 16)()
    p = C.cast(buf, C.c_void_p)
    cnt = C.c_int64(-1)
    dev = C.c_void_p(0x100000)
    # nonzero: negative extents, ld < cols, missing count, one-sided map
    assert lib.tcu_nonzero(p, -1, 4, 4, p, p, None, None, 4, C.byref(cnt), dev, 1 << 20,
                           None) == _lib.TCU_ERR_ARG
    assert lib.tcu_nonzero(p, 4, 4, 3, p, p, None, None, 4, C.byref(cnt), dev, 1 << 20,
                           None) == _lib.TCU_ERR_ARG
    assert lib.tcu_nonzero(p, 4, 4, 4, p, p, None, None, 4, None, dev, 1 << 20,
                           None) == _lib.TCU_ERR_ARG
    assert lib.tcu_nonzero(p, 4, 4, 4, p, p, p, None, 4, C.byref(cnt), dev, 1 << 20,
                           None) == _lib.TCU_ERR_ARG
    assert lib.tcu_nonzero(p, 4, 4, 4, p, p, None, None, 4, C.byref(cnt), None, 0,
                           None) == _lib.TCU_ERR_WORKSPACE
    assert lib.tcu_nonzero_workspace_bytes(-1, 5) == 0
    # host-resident GEMM: shapes, leading dimensions, block size, device buffer
    assert lib.tcu_gemm_f64_host(-1, 4, 4, p, 4, p, 4, p, 4, dev, 1 << 30, 0,
                                 None) == _lib.TCU_ERR_ARG
    assert lib.tcu_gemm_f64_host(4, 4, 4, p, 3, p, 4, p, 4, dev, 1 << 30, 0,
                                 None) == _lib.TCU_ERR_ARG
    assert lib.tcu_gemm_f64_host(4, 4, 4, p, 4, p, 4, p, 4, dev, 1 << 30, 100,
                                 None) == _lib.TCU_ERR_ARG
    assert lib.tcu_gemm_f64_host(4, 4, 4, None, 4, p, 4, p, 4, dev, 1 << 30, 0,
                                 None) == _lib.TCU_ERR_ARG
    assert lib.tcu_gemm_f64_host(4, 4, 4, p, 4, p, 4, p, 4, None, 1 << 30, 0,
                                 None) == _lib.TCU_ERR_WORKSPACE
    assert lib.tcu_gemm_f64_host(4, 4, 4, p, 4, p, 4, p, 4, dev, 1000, 0,
                                 None) == _lib.TCU_ERR_WORKSPACE
    assert lib.tcu_gemm_f64_host(4, 4, 4, p, 4, p, 4, p, 4, dev, 48 * 128 * 128 - 8, 128,
                                 None) == _lib.TCU_ERR_WORKSPACE
    assert lib.tcu_gemm_f64_host(0, 4, 4, p, 4, p, 4, p, 4, None, 0, 0, None) == _lib.TCU_OK
    # row form and block-sparse form: bad shapes
    A = _lib.tcu_relation(0, None, None, None, _lib.TCU_F64, 0)
    assert lib.tcu_join_agg_row(C.byref(A), C.byref(A), 0, 4, p, None, dev, 1 << 20,
                                None) == _lib.TCU_ERR_ARG
    assert lib.tcu_join_agg_row_workspace_bytes(4, 0) == 0
    assert lib.tcu_join_agg_bsr(C.byref(A), C.byref(A), 4, 0, 4, p, dev, 1 << 20,
                                None) == _lib.TCU_ERR_ARG
    assert lib.tcu_join_agg_bsr_workspace_bytes(C.byref(A), C.byref(A), 0, 4, 4) == 0
    assert lib.tcu_dict_encode(None, 5, None, 0, None, None, None, C.byref(cnt), dev, 1 << 20,
                               None) == _lib.TCU_ERR_ARG
    assert lib.tcu_dict_workspace_bytes(-3) == 0


def test_block_sparse_choice_host_only(lib):
    """The dense / block-sparse cost model (Sections 4.2.4, 4.3) runs on the
    host only.  For Q1 pair counts (one record per tuple, n tuples per side)
    it must pick the dense form while few distinct keys make the encodings
    dense, the block-sparse form once the key domain is large, switch only
    once as K grows, and agree with the winners measured on MI355X at the
    calibration points next to the switch."""
    fake = C.c_void_p(0x1000)  # never dereferenced

    def rel(n):
        return _lib.tcu_relation(n, fake, fake, None, _lib.TCU_F64, 0)

    def pick(n, K):
        a, b = rel(n), rel(n)
        return lib.tcu_block_sparse_preferred(C.byref(a), C.byref(b), n, K, n)

    for n in (4096, 8192, 16384):
        picks = [pick(n, K) for K in (32, 128, 512, 1024, 2048, 4096, 16384, 1 << 20)]
        assert picks[0] == 0 and picks[-1] == 1
        assert picks == sorted(picks)  # one switch, dense -> block-sparse
    # measured on MI355X (dense ms / block-sparse ms): n = 4096: K = 1024
    # 0.53 / 0.77, K = 2006 1.19 / 0.75; n = 8192: K = 512 1.01 / 1.47,
    # K = 1024 1.95 / 1.22
    assert pick(4096, 1024) == 0 and pick(4096, 2006) == 1
    assert pick(8192, 512) == 0 and pick(8192, 1024) == 1
    bad = rel(-1)
    good = rel(10)
    assert lib.tcu_block_sparse_preferred(C.byref(bad), C.byref(good), 4, 4, 4) == _lib.TCU_ERR_ARG
    assert lib.tcu_block_sparse_preferred(C.byref(good), C.byref(good), 0, 4, 4) == _lib.TCU_ERR_ARG


def test_mfma_peak_host_only(lib):
    """The peak probe's operation counts and argument checks need no GPU:
    2048 workgroups of four waves, eight instructions per wave and round."""
    assert lib.tcu_mfma_peak_out_bytes() >= 2048 * 256 * 8
    waves = 2048 * 4 * 8
    assert lib.tcu_mfma_peak_ops(0, 3) == waves * 3 * 2.0 * 16 * 16 * 4
    assert lib.tcu_mfma_peak_ops(1, 3) == waves * 3 * 2.0 * 32 * 32 * 32
    assert lib.tcu_mfma_peak_ops(2, 1) == lib.tcu_mfma_peak_ops(1, 1)
    assert lib.tcu_mfma_peak_ops(3, 1) == 0.0 and lib.tcu_mfma_peak_ops(0, 0) == 0.0
    fake = C.c_void_p(0x1000)  # never dereferenced
    assert lib.tcu_mfma_peak(3, 1, fake, None) == _lib.TCU_ERR_ARG
    assert lib.tcu_mfma_peak(0, 0, fake, None) == _lib.TCU_ERR_ARG
    assert lib.tcu_mfma_peak(1, 4, None, None) == _lib.TCU_ERR_ARG


def test_noalloc_rejects_before_touching_the_device(lib):
    A, B = rel(10), rel(10)
    cbuf = C.c_void_p(0x2000)
    # shapes whose workspace exceeds the library's array: refused on the host
    assert lib.tcu_join_agg_fwd_noalloc(C.byref(A), C.byref(B), 4096, 4096, 4096, 0, 0.0, cbuf,
                                        None, None, None) == _lib.TCU_ERR_WORKSPACE
    # invalid shapes, precision and a misaligned status buffer
    assert lib.tcu_join_agg_fwd_noalloc(C.byref(A), C.byref(B), 0, 4, 4, 0, 0.0, cbuf, None,
                                        None, None) == _lib.TCU_ERR_ARG
    assert lib.tcu_join_agg_fwd_noalloc(C.byref(A), C.byref(B), 4, 4, 4, 9, 0.0, cbuf, None,
                                        None, None) == _lib.TCU_ERR_ARG
    assert lib.tcu_join_agg_fwd_noalloc(C.byref(A), C.byref(B), 4, 4, 4, 0, 0.0, cbuf, None,
                                        C.c_void_p(0x1010), None) == _lib.TCU_ERR_ARG
    # the largest FP64 shape it holds
    need = lib.tcu_workspace_bytes(C.byref(A), C.byref(B), 2048, 2048, 2048, 0, 0)
    assert need <= _lib.TCU_NOALLOC_MAX_BYTES
    assert lib.tcu_workspace_bytes(C.byref(A), C.byref(B), 2200, 2048, 2200, 0, 0) > \
        _lib.TCU_NOALLOC_MAX_BYTES


def test_ops_out_shape_and_device_checked(monkeypatch):
    """ops.encode / ops.gemm_f64 refuse an `out` whose shape or device differs
    from what the library writes (host-side, before any library call)."""
    import torch
    from paper_2112_07552_amd import ops

    monkeypatch.setattr(ops, "_need_cuda", lambda *a, **k: None)  # CPU tensors stand in
    out = torch.empty((3, 4), dtype=torch.float64)
    ops._need_out(out, (3, 4), "cpu")
    for shape in ((4, 3), (3, 5), (12,)):
        with pytest.raises(ValueError):
            ops._need_out(out, shape, "cpu")
    with pytest.raises(ValueError):
        ops._need_out(out, (3, 4), "meta")


def test_gemm_split_workspace_sizes(lib):
    """The split contraction applies to outputs of few tiles with a long
    contraction; its workspace holds one partial product per chunk."""
    assert lib.tcu_gemm_f64_workspace_bytes(4096, 4096, 4096) == 0   # enough tiles
    assert lib.tcu_gemm_f64_workspace_bytes(1, 32, 512) == 0         # short contraction
    nb = lib.tcu_gemm_f64_workspace_bytes(1, 32, 32768)
    assert nb > 0 and nb % (1 * 32 * 8) == 0 and nb // (32 * 8) >= 2
    assert lib.tcu_gemm_f64_workspace_bytes(0, 32, 32768) == 0
    cbuf = C.c_void_p(0x2000)
    # argument errors return before any launch
    assert lib.tcu_gemm_f64_ws(2, 0, 1, 32, 32768, cbuf, 32768, cbuf, 32, cbuf, 32, cbuf, nb,
                               None) == _lib.TCU_ERR_ARG
    assert lib.tcu_gemm_f64_ws(0, 0, 1, 32, 32768, cbuf, 32768, cbuf, 32, cbuf, 31, cbuf, nb,
                               None) == _lib.TCU_ERR_ARG
    assert lib.tcu_gemm_f64_ws(0, 0, 1, 32, 32768, cbuf, 32768, cbuf, 32, cbuf, 32, None, nb,
                               None) == _lib.TCU_ERR_WORKSPACE
    assert lib.tcu_gemm_f64_ws(0, 0, 1, 32, 32768, cbuf, 32768, cbuf, 32, cbuf, 32, cbuf, nb - 1,
                               None) == _lib.TCU_ERR_WORKSPACE
