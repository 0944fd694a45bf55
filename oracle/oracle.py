"""Python face of the FP64 CPU oracle (oracle.c) for the TCUDB join-aggregate.

TEST INFRASTRUCTURE ONLY: the checker that the HIP path is compared with.
Only the tests, the smoke check and the benchmark's CPU-baseline leg use it;
the product path never imports it.  It shares no code with the HIP library.

Relations are passed as (group, key, val) for A and (key, group, val) for B,
numpy arrays of int32, int32 and float64 (val may be None: COUNT, all ones).
Notation follows the matrix multiplication query of Section 2.3: A holds
records (g, k, v), B holds records (k, h, w) and
    C[g,h] = sum over joined pairs with a.group = g, b.group = h of v * w.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import NamedTuple, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

_i32p = C.POINTER(C.c_int32)
_i64p = C.POINTER(C.c_int64)
_f64p = C.POINTER(C.c_double)


class Rel(NamedTuple):
    """One relation as a struct of arrays.

    For A: group = g (A.col_num in the MM query), key = k (A.row_num).
    For B: group = h (B.row_num), key = k (B.col_num).
    """
    group: np.ndarray
    key: np.ndarray
    val: Optional[np.ndarray]

    @property
    def n(self) -> int:
        return int(self.group.shape[0])


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b  # type: ignore
            _b.build()
        L = C.CDLL(LIB_PATH)
        rel = [C.c_int64, _i32p, _i32p, _f64p, C.c_int64, _i32p, _i32p, _f64p,
               C.c_int32, C.c_int32, C.c_int32]
        L.orc_encode.argtypes = [C.c_int64, _i32p, _i32p, _f64p, C.c_int32, C.c_int32, _f64p]
        L.orc_encode.restype = C.c_int64
        L.orc_join_agg_rows.argtypes = rel + [C.c_int64, _i32p, _f64p, _i64p, C.c_int]
        L.orc_join_agg_rows.restype = C.c_int
        L.orc_join_agg_cells.argtypes = rel + [C.c_int64, _i32p, _i32p, _f64p, _i64p, C.c_int]
        L.orc_join_agg_cells.restype = C.c_int
        L.orc_freivalds.argtypes = rel + [_f64p, _f64p, C.c_int]
        L.orc_freivalds.restype = C.c_int
        L.orc_grad.argtypes = rel + [_f64p, C.c_int, C.c_int64, _i64p, _f64p, C.c_int]
        L.orc_grad.restype = C.c_int
        L.orc_split.argtypes = [C.c_int32, C.c_int32, _f64p, C.c_int, C.c_int, C.c_int,
                                _i32p, _f64p]
        L.orc_split.restype = C.c_int64
        L.orc_dict.argtypes = [C.c_int64, _i64p, C.c_int64, _i64p, _i32p, _i32p, _i64p]
        L.orc_dict.restype = C.c_int64
        L.orc_trunc_product.argtypes = [C.c_int32, C.c_int32, C.c_int32, _f64p, _f64p, C.c_int,
                                        _f64p, C.c_int]
        L.orc_trunc_product.restype = C.c_int
        L.orc_certificate.argtypes = [C.c_int32, C.c_int32, C.c_int32, _f64p, _f64p, C.c_double,
                                      _f64p, C.POINTER(C.c_uint32), C.POINTER(C.c_uint32),
                                      _f64p, _i64p, _f64p, C.c_int]
        L.orc_certificate.restype = C.c_int
        _lib = L
    return _lib


def _p(a, t):
    if a is None:
        return None
    return a.ctypes.data_as(t)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _rel_args(A: Rel, B: Rel, M: int, K: int, N: int, keep: list):
    ag, ak, av = _i32(A.group), _i32(A.key), _f64(A.val)
    bk, bh, bw = _i32(B.key), _i32(B.group), _f64(B.val)
    keep += [ag, ak, av, bk, bh, bw]
    return [A.n, _p(ag, _i32p), _p(ak, _i32p), _p(av, _f64p),
            B.n, _p(bk, _i32p), _p(bh, _i32p), _p(bw, _f64p), M, K, N]


def threads_default() -> int:
    return len(os.sched_getaffinity(0))


def encode(row, col, val, R: int, Ccols: int):
    """Dense R x Ccols encoding: out[row,col] = sum of val (Section 3.1/3.3).

    Returns (matrix, number of skipped out-of-range records)."""
    row, col, val = _i32(row), _i32(col), _f64(val)
    out = np.empty((R, Ccols), dtype=np.float64)
    skipped = lib().orc_encode(row.shape[0], _p(row, _i32p), _p(col, _i32p), _p(val, _f64p),
                               R, Ccols, _p(out, _f64p))
    return out, int(skipped)


def encode_A(A: Rel, M: int, K: int):
    """X (M x K): X[g,k] = sum of a.val over A records (g, k)."""
    return encode(A.group, A.key, A.val, M, K)


def encode_B(B: Rel, K: int, N: int):
    """Y (K x N): Y[k,h] = sum of b.val over B records (k, h)."""
    return encode(B.key, B.group, B.val, K, N)


def join_agg(A: Rel, B: Rel, M: int, K: int, N: int, rows=None, with_count=False,
             threads: Optional[int] = None):
    """C (and the exact pair count) for all groups g, or for `rows` only.

    Returns (C, count or None, threads_used)."""
    keep: list = []
    args = _rel_args(A, B, M, K, N, keep)
    if rows is None:
        nr, rp = M, None
    else:
        rows = _i32(rows)
        nr, rp = rows.shape[0], _p(rows, _i32p)
    out = np.empty((nr, N), dtype=np.float64)
    cnt = np.empty((nr, N), dtype=np.int64) if with_count else None
    used = lib().orc_join_agg_rows(*args, nr if rows is not None else 0, rp, _p(out, _f64p),
                                   _p(cnt, _i64p), threads or threads_default())
    if used < 0:
        raise MemoryError("oracle: allocation failed")
    return out, cnt, used


def join_agg_cells(A: Rel, B: Rel, M: int, K: int, N: int, cg, ch,
                   threads: Optional[int] = None):
    """C and the pair count at cells (cg[i], ch[i]).  Returns (vals, counts)."""
    keep: list = []
    args = _rel_args(A, B, M, K, N, keep)
    cg, ch = _i32(cg), _i32(ch)
    out = np.empty(cg.shape[0], dtype=np.float64)
    cnt = np.empty(cg.shape[0], dtype=np.int64)
    used = lib().orc_join_agg_cells(*args, cg.shape[0], _p(cg, _i32p), _p(ch, _i32p),
                                    _p(out, _f64p), _p(cnt, _i64p), threads or threads_default())
    if used < 0:
        raise MemoryError("oracle: allocation failed")
    return out, cnt


def freivalds(A: Rel, B: Rel, M: int, K: int, N: int, r, threads: Optional[int] = None):
    """C @ r evaluated from the records in O(nA + nB) (Freivalds' check)."""
    keep: list = []
    args = _rel_args(A, B, M, K, N, keep)
    r = _f64(r)
    out = np.empty(M, dtype=np.float64)
    used = lib().orc_freivalds(*args, _p(r, _f64p), _p(out, _f64p), threads or threads_default())
    if used < 0:
        raise MemoryError("oracle: allocation failed")
    return out


def grad(A: Rel, B: Rel, M: int, K: int, N: int, W, which: str, idx=None,
         threads: Optional[int] = None):
    """Closed-form gradient of sum(W * C) w.r.t. A.val ('A') or B.val ('B').

    `idx` selects records (all when None)."""
    keep: list = []
    args = _rel_args(A, B, M, K, N, keep)
    W = np.ascontiguousarray(W, dtype=np.float64)
    assert W.shape == (M, N)
    n = A.n if which == "A" else B.n
    if idx is not None:
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        nidx, ip = idx.shape[0], _p(idx, _i64p)
    else:
        nidx, ip = n, None
    out = np.empty(nidx, dtype=np.float64)
    used = lib().orc_grad(*args, _p(W, _f64p), 0 if which == "A" else 1, nidx, ip,
                          _p(out, _f64p), threads or threads_default())
    if used < 0:
        raise MemoryError("oracle: allocation failed")
    return out


def split(X, axis: int, nslices: int, bits: int = 8):
    """Fixed-point slices of X with one power-of-two scale per row (axis 0)
    or per column (axis 1).  Returns (exps int32, slices float64 [s, R, L])."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    R, L = X.shape
    exps = np.empty(R if axis == 0 else L, dtype=np.int32)
    sl = np.empty((nslices, R, L), dtype=np.float64)
    bad = lib().orc_split(R, L, _p(X, _f64p), axis, nslices, bits, _p(exps, _i32p), _p(sl, _f64p))
    if bad:
        raise FloatingPointError(f"oracle.split: non-finite value in line {bad - 1}")
    return exps, sl


def dictionary(a, b):
    """dom(ID) of Section 3.1 for two int64 columns: (dict sorted distinct
    values, codes of a, codes of b), codes = ranks in dict."""
    a = np.ascontiguousarray(a, dtype=np.int64)
    b = np.ascontiguousarray(b, dtype=np.int64)
    ca = np.empty(a.shape[0], dtype=np.int32)
    cb = np.empty(b.shape[0], dtype=np.int32)
    d = np.empty(max(1, a.shape[0] + b.shape[0]), dtype=np.int64)
    k = lib().orc_dict(a.shape[0], _p(a, _i64p), b.shape[0], _p(b, _i64p), _p(ca, _i32p),
                       _p(cb, _i32p), _p(d, _i64p))
    if k < 0:
        raise MemoryError("oracle: allocation failed")
    return d[:k].copy(), ca, cb


def join3(a_id1, b_id1, b_id2, c_id2):
    """Query Q2 of Section 3.2 by its definition: every (a, b, c) with
    A[a].ID1 = B[b].ID1 and B[b].ID2 = C[c].ID2.  Returns an int64 array of
    shape (t, 3), rows sorted lexicographically.

    For each B tuple, the matching A tuples and C tuples are found by sorting
    A on ID1 and C on ID2 and taking equal ranges (library sort and binary
    search as steps); the output is their product, per B tuple."""
    a = np.ascontiguousarray(a_id1, dtype=np.int64)
    b1 = np.ascontiguousarray(b_id1, dtype=np.int64)
    b2 = np.ascontiguousarray(b_id2, dtype=np.int64)
    c = np.ascontiguousarray(c_id2, dtype=np.int64)
    oa = np.argsort(a, kind="stable")
    oc = np.argsort(c, kind="stable")
    sa, sc = a[oa], c[oc]
    a_lo, a_hi = np.searchsorted(sa, b1, "left"), np.searchsorted(sa, b1, "right")
    c_lo, c_hi = np.searchsorted(sc, b2, "left"), np.searchsorted(sc, b2, "right")
    out = []
    for b in range(b1.shape[0]):
        na, nc = a_hi[b] - a_lo[b], c_hi[b] - c_lo[b]
        if na == 0 or nc == 0:
            continue
        aa = oa[a_lo[b]:a_hi[b]]
        cc = oc[c_lo[b]:c_hi[b]]
        t = np.empty((na * nc, 3), dtype=np.int64)
        t[:, 0] = np.repeat(aa, nc)
        t[:, 1] = b
        t[:, 2] = np.tile(cc, na)
        out.append(t)
    if not out:
        return np.empty((0, 3), dtype=np.int64)
    t = np.concatenate(out)
    return t[np.lexsort((t[:, 2], t[:, 1], t[:, 0]))]


def trunc_product(X, Y, bits: int, threads: Optional[int] = None):
    """(X' Y') 2^(e_g + f_h - 2 bits), X' and Y' the per-row / per-column
    truncations of X and Y to `bits`-bit integers, the integer product exact
    (128-bit) and rounded once: what the CRT mixed form reconstructs."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    Y = np.ascontiguousarray(Y, dtype=np.float64)
    M, K = X.shape
    K2, N = Y.shape
    assert K == K2
    out = np.empty((M, N), dtype=np.float64)
    r = lib().orc_trunc_product(M, K, N, _p(X, _f64p), _p(Y, _f64p), bits, _p(out, _f64p),
                                threads or threads_default())
    if r == -1:
        raise FloatingPointError("oracle.trunc_product: non-finite input or bad bits")
    if r < 0:
        raise MemoryError("oracle: allocation failed")
    return out



def certificate(X, Y, tcrt: float, tdig, with_detail: bool = False,
                threads: Optional[int] = None):
    """The certificate of the mixed-form product X Y (oracle.c,
    orc_certificate): returns (need_bits, need_slices, (umax_x, umax_y)) (255:
    no width or digit count certifies some cell) and,
    with_detail, also T (M x N int64) and the normalised line sums (rows of
    X, then columns of Y).  tdig: 9 tolerances indexed by the digit count
    (entry 0 unused)."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    Y = np.ascontiguousarray(Y, dtype=np.float64)
    M, K = X.shape
    K2, N = Y.shape
    assert K == K2
    td = np.ascontiguousarray(tdig, dtype=np.float64)
    assert td.shape == (9,)
    nb, ns = C.c_uint32(0), C.c_uint32(0)
    umax = np.zeros(2)
    T = np.empty((M, N), dtype=np.int64) if with_detail else None
    sums = np.empty(M + N) if with_detail else None
    r = lib().orc_certificate(M, K, N, _p(X, _f64p), _p(Y, _f64p), float(tcrt), _p(td, _f64p),
                              C.byref(nb), C.byref(ns), _p(umax, _f64p), _p(T, _i64p),
                              _p(sums, _f64p), threads or threads_default())
    if r == -1:
        raise FloatingPointError("oracle.certificate: non-finite input")
    if r < 0:
        raise MemoryError("oracle: allocation failed")
    out = (nb.value, ns.value, (float(umax[0]), float(umax[1])))
    return out + (T, sums) if with_detail else out
