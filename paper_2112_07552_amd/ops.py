"""Torch-facing calls of the join-aggregate operator (TCUDB Sections 2.3, 3.3).

Each function checks tensor placement and dtypes, allocates outputs and the
workspace with torch, and calls the C ABI of libtcudb.so on the current HIP
stream.  No arithmetic of the operator happens here.

Relation layout (struct of arrays, all on one GPU):
  A: a_group (int32, g in [0,M)), a_key (int32, k in [0,K)), a_val (f64/f32 or None)
  B: b_key (int32, k in [0,K)), b_group (int32, h in [0,N)), b_val (f64/f32 or None)
  C[g,h] = sum over joined pairs (a.k == b.k) with a.g == g, b.h == h of a.v * b.w
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Tuple

import torch

from . import _lib
from ._lib import TcuError, check

PRECISIONS = {"fp64": _lib.TCU_PREC_FP64, "split_bf16": _lib.TCU_PREC_SPLIT_BF16,
              "split_i8": _lib.TCU_PREC_SPLIT_I8, "crt_i8": _lib.TCU_PREC_CRT_I8}


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(device: torch.device):
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _need_cuda(t: torch.Tensor, name: str, dtypes) -> None:
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype not in dtypes:
        raise TypeError(f"{name} must have dtype in {dtypes}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _need_out(out: torch.Tensor, shape, device) -> None:
    """A caller-supplied output must have exactly the shape the library
    writes (it writes every element of that shape), on the inputs' device."""
    _need_cuda(out, "out", (torch.float64,))
    if tuple(out.shape) != tuple(shape):
        raise ValueError(f"out must have shape {tuple(shape)}, got {tuple(out.shape)}")
    if out.device != torch.device(device):
        raise ValueError(f"out must be on {device}, got {out.device}")


def make_relation(group: torch.Tensor, key: torch.Tensor, val: Optional[torch.Tensor],
                  unique: bool = False):
    """tcu_relation for one relation.  unique=True declares that no two
    records share a (group, key) cell (a table storing a matrix)."""
    _need_cuda(group, "group", (torch.int32,))
    _need_cuda(key, "key", (torch.int32,))
    n = group.numel()
    if key.numel() != n:
        raise ValueError("group and key lengths differ")
    dtype = _lib.TCU_F64
    if val is not None:
        _need_cuda(val, "val", (torch.float64, torch.float32))
        if val.numel() != n:
            raise ValueError("val length differs from group/key")
        if val.device != group.device or key.device != group.device:
            raise ValueError("columns of a relation must be on one device")
        dtype = _lib.TCU_F32 if val.dtype == torch.float32 else _lib.TCU_F64
    rel = _lib.tcu_relation(n, group.data_ptr() if n else None, key.data_ptr() if n else None,
                            val.data_ptr() if (val is not None and n) else None, dtype,
                            _lib.TCU_REL_UNIQUE_CELLS if unique else 0)
    return rel


def workspace_bytes(A, B, M: int, K: int, N: int, precision: str = "fp64",
                    backward: bool = False, count: bool = False) -> int:
    flags = (_lib.TCU_WS_BACKWARD if backward else 0) | (_lib.TCU_WS_COUNT if count else 0)
    nb = _lib.load().tcu_workspace_bytes(C.byref(A), C.byref(B), M, K, N,
                                          PRECISIONS[precision], flags)
    if nb == 0:
        raise TcuError(_lib.TCU_ERR_ARG, "tcu_workspace_bytes")
    return int(nb)


def alloc_workspace(nbytes: int, device) -> torch.Tensor:
    ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
    if ws.data_ptr() % 256:
        raise RuntimeError("torch returned a workspace that is not 256-byte aligned")
    return ws


def mixed_plan(precision: str, k: int, tol: float, need: int, u: float):
    """Step a0 host plan of one mixed-form product from its certificate (the
    largest per-cell need and the bound u on the normalised line sums):
    (slice or modulus count, truncation bits or 0); raises TcuError
    (TCU_ERR_INFEASIBLE) when no plan exists."""
    bits = C.c_int32(0)
    r = _lib.load().tcu_mixed_plan(PRECISIONS[precision], int(k), float(tol), int(need),
                                   float(u), C.byref(bits))
    if r < 0:
        raise TcuError(r, "tcu_mixed_plan")
    return r, bits.value


def _pad(x: int, m: int) -> int:
    return (x + m - 1) // m * m


def split(Z: torch.Tensor, axis: int, precision: str, S: int, ws: Optional[torch.Tensor] = None):
    """Step a0 device part: (exps int32 [lines], slices [S, lines_pad, len_pad]
    in the library's blocked layout, raw dtype int8 or int16 (BF16 bits))."""
    _need_cuda(Z, "Z", (torch.float64,))
    rows, cols = Z.shape
    lines, length = (rows, cols) if axis == 0 else (cols, rows)
    lines_pad, len_pad = _pad(lines, 128), _pad(length, 64)
    dt = torch.int8 if precision == "split_i8" else torch.int16
    slices = torch.empty((S, lines_pad * len_pad), dtype=dt, device=Z.device)
    exps = torch.empty(lines, dtype=torch.int32, device=Z.device)
    need = 256 + 8 * lines_pad
    if ws is None or ws.numel() < need:
        ws = alloc_workspace(need, Z.device)
    check(_lib.load().tcu_split(_ptr(Z), rows, cols, Z.shape[1], axis, PRECISIONS[precision], S,
                                _ptr(slices), lines_pad, len_pad, _ptr(exps), _ptr(ws),
                                ws.numel(), _stream(Z.device)), "tcu_split")
    return exps, slices, (lines_pad, len_pad), ws


def unblock_slices(slices: torch.Tensor, lines: int, length: int, lines_pad: int, len_pad: int,
                   precision: str) -> torch.Tensor:
    """Reorder the blocked layout [S][t / KSTEP][(t % KSTEP) / HALF][line][t % HALF]
    to [S][line][t] (index bookkeeping only)."""
    kstep = 32 if precision == "split_i8" else 16
    half = kstep // 2
    S = slices.shape[0]
    v = slices.reshape(S, len_pad // kstep, 2, lines_pad, half).permute(0, 3, 1, 2, 4)
    return v.reshape(S, lines_pad, len_pad)[:, :lines, :length]


def encode(group, key, val, rows: int, cols: int, transpose: bool = False,
           out: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None,
           unique: bool = False, windows: bool = True) -> torch.Tensor:
    """Step a1 (Sections 3.1/3.3): dense FP64 encoding of one relation.

    transpose=False: out[group, key] (A -> X);  True: out[key, group] (B -> Y).
    windows: give the library the scratch with which it fills a matrix of
    1 GiB or more one window of rows at a time (tcu_encode_workspace_bytes);
    False, or a smaller `ws`, fills it in one pass (same result)."""
    rel = make_relation(group, key, val, unique)
    dev = group.device
    if out is None:
        out = torch.empty((rows, cols), dtype=torch.float64, device=dev)
    _need_out(out, (rows, cols), dev)
    if ws is None:
        need = _lib.load().tcu_encode_workspace_bytes(C.byref(rel), rows, cols) if windows else 0
        ws = alloc_workspace(max(256, need), dev)
    check(_lib.load().tcu_encode(C.byref(rel), int(transpose), rows, cols, _ptr(out), _ptr(ws),
                                 ws.numel(), _stream(dev)), "tcu_encode")
    return out


def gemm_f64(A: torch.Tensor, B: torch.Tensor, trans_a: bool = False, trans_b: bool = False,
             out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Step a2 alone: op(A) @ op(B) in FP64 on the matrix cores."""
    _need_cuda(A, "A", (torch.float64,))
    _need_cuda(B, "B", (torch.float64,))
    m, k = (A.shape[1], A.shape[0]) if trans_a else (A.shape[0], A.shape[1])
    kb, n = (B.shape[1], B.shape[0]) if trans_b else (B.shape[0], B.shape[1])
    if k != kb:
        raise ValueError(f"inner dimensions differ: {k} vs {kb}")
    if B.device != A.device:
        raise ValueError("A and B must be on one device")
    if out is None:
        out = torch.empty((m, n), dtype=torch.float64, device=A.device)
    _need_out(out, (m, n), A.device)
    L = _lib.load()
    nb = int(L.tcu_gemm_f64_workspace_bytes(m, n, k)) if m and n and k else 0
    if nb > 0:
        # few output tiles: the contraction is split over workgroups
        ws = alloc_workspace(nb, A.device)
        check(L.tcu_gemm_f64_ws(int(trans_a), int(trans_b), m, n, k, _ptr(A), A.shape[1],
                                _ptr(B), B.shape[1], _ptr(out), n, _ptr(ws), ws.numel(),
                                _stream(A.device)), "tcu_gemm_f64_ws")
        return out
    check(L.tcu_gemm_f64(int(trans_a), int(trans_b), m, n, k, _ptr(A), A.shape[1],
                         _ptr(B), B.shape[1], _ptr(out), n, _stream(A.device)), "tcu_gemm_f64")
    return out


def gemm_f64_host(A: torch.Tensor, B: torch.Tensor, out: Optional[torch.Tensor] = None,
                  dev_bytes: int = 1 << 30, block: int = 0, device=None) -> torch.Tensor:
    """Section 4.2.3: C = A @ B with A, B, C in host memory (FP64 CPU tensors,
    preferably pinned), streamed through `dev_bytes` of device memory in
    blocks (block = 0: the largest multiple of 128 that fits)."""
    for t, name in ((A, "A"), (B, "B")):
        if t.device.type != "cpu" or t.dtype != torch.float64 or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float64 CPU tensor")
    m, k = A.shape
    kb, n = B.shape
    if k != kb:
        raise ValueError(f"inner dimensions differ: {k} vs {kb}")
    if out is None:
        out = torch.empty((m, n), dtype=torch.float64, pin_memory=True)
    dev = torch.device("cuda:0") if device is None else torch.device(device)
    buf = alloc_workspace(int(dev_bytes), dev)
    check(_lib.load().tcu_gemm_f64_host(m, n, k, _ptr(A), k, _ptr(B), n, _ptr(out), n, _ptr(buf),
                                        buf.numel(), int(block), _stream(dev)),
          "tcu_gemm_f64_host")
    return out


def join_agg_fwd(a_group, a_key, a_val, b_key, b_group, b_val, M: int, K: int, N: int,
                 precision: str = "fp64", tol: float = 0.0, with_count: bool = False,
                 ws: Optional[torch.Tensor] = None, unique: bool = False,
                 for_backward: bool = False
                 ) -> Tuple[torch.Tensor, Optional[torch.Tensor], torch.Tensor]:
    """Steps a1-a3: returns (C, count or None, workspace).

    for_backward=True sizes the workspace so that join_agg_bwd can reuse the
    encodings it holds (saved_encodings=True)."""
    A = make_relation(a_group, a_key, a_val, unique)
    B = make_relation(b_group, b_key, b_val, unique)
    dev = a_group.device
    need = workspace_bytes(A, B, M, K, N, precision, count=with_count, backward=for_backward)
    if ws is None or ws.numel() < need:
        ws = alloc_workspace(need, dev)
    Cm = torch.empty((M, N), dtype=torch.float64, device=dev)
    cnt = torch.empty((M, N), dtype=torch.int32, device=dev) if with_count else None
    check(_lib.load().tcu_join_agg_fwd(C.byref(A), C.byref(B), M, K, N, PRECISIONS[precision],
                                       tol, _ptr(Cm), _ptr(cnt), _ptr(ws), ws.numel(),
                                       _stream(dev)), "tcu_join_agg_fwd")
    return Cm, cnt, ws


def join_agg_bwd(a_group, a_key, a_val, b_key, b_group, b_val, M: int, K: int, N: int,
                 dC: torch.Tensor, need_a: bool = True, need_b: bool = True,
                 precision: str = "fp64", tol: float = 0.0, ws: Optional[torch.Tensor] = None,
                 unique: bool = False, saved_encodings: bool = False):
    """Step a4: returns (dA_val or None, dB_val or None, workspace), FP64.

    saved_encodings=True: `ws` is the workspace of the forward on these same
    inputs (sized with for_backward=True) and still holds X and Y."""
    A = make_relation(a_group, a_key, a_val, unique)
    B = make_relation(b_group, b_key, b_val, unique)
    dev = a_group.device
    _need_cuda(dC, "dC", (torch.float64,))
    if tuple(dC.shape) != (M, N):
        raise ValueError(f"dC must be {M} x {N}")
    need = workspace_bytes(A, B, M, K, N, precision, backward=True)
    if saved_encodings and (ws is None or ws.numel() < need):
        raise ValueError("saved_encodings needs the forward's workspace sized for backward")
    if ws is None or ws.numel() < need:
        ws = alloc_workspace(need, dev)
    dA = torch.empty(A.n, dtype=torch.float64, device=dev) if need_a else None
    dB = torch.empty(B.n, dtype=torch.float64, device=dev) if need_b else None
    flags = _lib.TCU_BWD_SAVED_ENCODINGS if saved_encodings else 0
    check(_lib.load().tcu_join_agg_bwd(C.byref(A), C.byref(B), M, K, N, PRECISIONS[precision],
                                       tol, _ptr(dC), _ptr(dA), _ptr(dB), flags, _ptr(ws),
                                       ws.numel(), _stream(dev)), "tcu_join_agg_bwd")
    return dA, dB, ws


def sync_status(ws: torch.Tensor) -> Tuple[int, dict]:
    """Synchronise and read the workspace status block of the last call."""
    info = _lib.tcu_status_info()
    st = _lib.load().tcu_sync_status(_ptr(ws), _stream(ws.device), C.byref(info))
    return st, {"flags": info.flags, "slices": info.slices,
                "skipped_a": info.skipped_a, "skipped_b": info.skipped_b,
                "bits": info.bits, "need": info.need, "exceptions": info.exceptions}


def _checkpoint_needed(M: int, K: int, N: int, device) -> bool:
    """Keep X and Y for backward unless they would take more than half of the
    device memory that is free now."""
    enc = 8 * (M * K + K * N + max(M * K, K * N))
    free, _ = torch.cuda.mem_get_info(device)
    return enc > free // 2


def dict_encode(a: torch.Tensor, b: torch.Tensor):
    """dom(ID) of Section 3.1 for two int64 columns on the GPU: returns
    (dict: sorted distinct values, codes_a int32, codes_b int32)."""
    _need_cuda(a, "a", (torch.int64,))
    _need_cuda(b, "b", (torch.int64,))
    dev = a.device
    n = a.numel() + b.numel()
    ws = alloc_workspace(int(_lib.load().tcu_dict_workspace_bytes(n)), dev)
    ca = torch.empty(a.numel(), dtype=torch.int32, device=dev)
    cb = torch.empty(b.numel(), dtype=torch.int32, device=dev)
    d = torch.empty(max(n, 1), dtype=torch.int64, device=dev)
    k = C.c_int64(0)
    check(_lib.load().tcu_dict_encode(_ptr(a) if a.numel() else None, a.numel(),
                                      _ptr(b) if b.numel() else None, b.numel(),
                                      _ptr(ca) if a.numel() else None,
                                      _ptr(cb) if b.numel() else None, _ptr(d), C.byref(k),
                                      _ptr(ws), ws.numel(), _stream(dev)), "tcu_dict_encode")
    return d[:k.value], ca, cb


def join_agg_row(a_key, a_val, b_key, b_group, b_val, K: int, N: int, with_count: bool = False):
    """Q3 / Q4 of Section 3.3 in re-associated form (A is one group):
    returns (c [N] FP64, count [N] int64 or None, workspace)."""
    dev = a_key.device
    A = make_relation(a_key, a_key, a_val)  # the group column is not read
    B = make_relation(b_group, b_key, b_val)
    ws = alloc_workspace(int(_lib.load().tcu_join_agg_row_workspace_bytes(K, N)), dev)
    c = torch.empty(N, dtype=torch.float64, device=dev)
    cnt = torch.empty(N, dtype=torch.int64, device=dev) if with_count else None
    check(_lib.load().tcu_join_agg_row(C.byref(A), C.byref(B), K, N, _ptr(c), _ptr(cnt),
                                       _ptr(ws), ws.numel(), _stream(dev)), "tcu_join_agg_row")
    return c, cnt, ws


def join_agg_bsr(a_group, a_key, a_val, b_key, b_group, b_val, M: int, K: int, N: int,
                 unique: bool = False) -> Tuple[torch.Tensor, torch.Tensor]:
    """The operator on 16 x 16 block-sparse encodings (Section 4.2.4):
    returns (C [M, N] FP64, workspace).  Blocks once per relation."""
    A = make_relation(a_group, a_key, a_val, unique)
    B = make_relation(b_group, b_key, b_val, unique)
    dev = a_group.device
    ws = alloc_workspace(int(_lib.load().tcu_join_agg_bsr_workspace_bytes(
        C.byref(A), C.byref(B), M, K, N)), dev)
    Cm = torch.empty((M, N), dtype=torch.float64, device=dev)
    check(_lib.load().tcu_join_agg_bsr(C.byref(A), C.byref(B), M, K, N, _ptr(Cm), _ptr(ws),
                                       ws.numel(), _stream(dev)), "tcu_join_agg_bsr")
    return Cm, ws


def block_sparse_preferred(a_group, a_key, a_val, b_key, b_group, b_val, M: int, K: int,
                           N: int) -> bool:
    """The library's cost-model choice (Sections 4.2.4, 4.2.2): True when the
    block-sparse operator is predicted faster than the dense FP64 one."""
    A = make_relation(a_group, a_key, a_val)
    B = make_relation(b_group, b_key, b_val)
    r = int(_lib.load().tcu_block_sparse_preferred(C.byref(A), C.byref(B), M, K, N))
    if r < 0:
        check(r, "tcu_block_sparse_preferred")
    return r == 1


def join_agg_auto(a_group, a_key, a_val, b_key, b_group, b_val, M: int, K: int, N: int,
                  unique: bool = False) -> Tuple[torch.Tensor, str]:
    """The operator in the form the cost model picks: returns (C [M, N] FP64,
    "block_sparse" or "dense")."""
    args = (a_group, a_key, a_val, b_key, b_group, b_val, M, K, N)
    if block_sparse_preferred(*args):
        return join_agg_bsr(*args, unique=unique)[0], "block_sparse"
    return join_agg_fwd(*args, unique=unique)[0], "dense"


def nonzero(M: torch.Tensor, col_map: Optional[torch.Tensor] = None,
            capacity: Optional[int] = None):
    """The matrix-to-table conversion of Section 3.2: (rows, cols, keys) of
    the nonzero cells of M in row-major order, int32; keys = col_map[cols]
    (None without a map).  Scans again with a larger output if `capacity`
    (default: a 2^22-entry guess) was too small."""
    if not isinstance(M, torch.Tensor) or M.device.type != "cuda" or M.dtype != torch.float64:
        raise ValueError("M must be a float64 CUDA (HIP) tensor")
    if M.dim() != 2 or (M.numel() and (M.stride(1) != 1 or M.stride(0) < M.shape[1])):
        raise ValueError("M must be a 2-D row-major matrix (unit column stride)")
    rows, cols = M.shape
    dev = M.device
    if col_map is not None:
        _need_cuda(col_map, "col_map", (torch.int32,))
        if col_map.numel() != cols:
            raise ValueError("col_map needs one entry per column")
    L = _lib.load()
    ws = alloc_workspace(int(L.tcu_nonzero_workspace_bytes(rows, cols)), dev)
    cap = min(rows * cols, 1 << 22) if capacity is None else int(capacity)
    while True:
        r = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        c = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        k = torch.empty(max(cap, 1), dtype=torch.int32, device=dev) if col_map is not None else None
        count = C.c_int64(0)
        check(L.tcu_nonzero(_ptr(M) if M.numel() else None, rows, cols, M.stride(0) if rows else cols,
                            _ptr(r), _ptr(c), _ptr(col_map), _ptr(k), cap, C.byref(count),
                            _ptr(ws), ws.numel(), _stream(dev)), "tcu_nonzero")
        if count.value <= cap:
            n = count.value
            return r[:n], c[:n], (None if k is None else k[:n])
        cap = count.value


def join3(a_id1: torch.Tensor, b_id1: torch.Tensor, b_id2: torch.Tensor, c_id2: torch.Tensor):
    """Query Q2 of Section 3.2, A(ID1) JOIN B(ID1, ID2) JOIN C(ID2), in the
    order A -> B -> C: C1 = mat(A) mat(B)^T, its nonzeros as the table AB,
    re-encoded by B.ID2, then C3 = mat(AB) mat(C)^T.  Returns (pair_a,
    pair_b, C3): C3[i, j] = 1 iff (A tuple pair_a[i], B tuple pair_b[i],
    C tuple j) is a result tuple."""
    dev = a_id1.device
    d1, ka, kb1 = dict_encode(a_id1, b_id1)
    d2, kb2, kc = dict_encode(b_id2, c_id2)
    n, m, mc = a_id1.numel(), b_id1.numel(), c_id2.numel()
    K1, K2 = max(1, d1.numel()), max(1, d2.numel())
    empty = torch.empty(0, dtype=torch.int32, device=dev)
    if n == 0 or m == 0:
        return empty, empty, torch.zeros((0, mc), dtype=torch.float64, device=dev)
    ta = torch.arange(n, dtype=torch.int32, device=dev)
    tb = torch.arange(m, dtype=torch.int32, device=dev)
    C1, _, ws = join_agg_fwd(ta, ka, None, kb1, tb, None, n, K1, m, unique=True)
    pa, pb, keys = nonzero(C1, col_map=kb2)
    del C1
    n2 = pa.numel()
    if n2 == 0 or mc == 0:
        return pa, pb, torch.zeros((n2, mc), dtype=torch.float64, device=dev)
    t2 = torch.arange(n2, dtype=torch.int32, device=dev)
    tc = torch.arange(mc, dtype=torch.int32, device=dev)
    C3, _, _ = join_agg_fwd(t2, keys, None, kc, tc, None, n2, K2, mc, unique=True)
    return pa, pb, C3


def join3_chain(a_id1: torch.Tensor, b_id1: torch.Tensor, b_id2: torch.Tensor,
                c_id2: torch.Tensor) -> torch.Tensor:
    """Q2 with B projected out (Section 3.2): mat(A) mat(B)^T mat(C)^T with
    mat(B) the ID1 x ID2 incidence of B, no table conversion in between.
    Returns R (n_A x n_C) FP64: R[a, c] = number of B tuples joining a and c."""
    dev = a_id1.device
    d1, ka, kb1 = dict_encode(a_id1, b_id1)
    d2, kb2, kc = dict_encode(b_id2, c_id2)
    n, mc = a_id1.numel(), c_id2.numel()
    K1, K2 = max(1, d1.numel()), max(1, d2.numel())
    ta = torch.arange(n, dtype=torch.int32, device=dev)
    tc = torch.arange(mc, dtype=torch.int32, device=dev)
    X1, _, _ = join_agg_fwd(ta, ka, None, kb1, kb2, None, n, K1, K2)   # n x K2
    Y = encode(tc, kc, None, K2, mc, transpose=True, unique=True)      # K2 x n_C
    return gemm_f64(X1, Y)


class JoinAgg(torch.autograd.Function):
    """C = join-aggregate(A, B) with the hand-written adjoint as backward.

    checkpoint=None keeps the forward's encodings X and Y for backward when
    they fit comfortably in HBM, and otherwise saves only the record columns
    and re-encodes in backward (activation checkpointing); True / False force
    one or the other."""

    @staticmethod
    def forward(ctx, a_group, a_key, a_val, b_key, b_group, b_val, M, K, N, precision, tol,
                unique, checkpoint):
        if checkpoint is None:
            checkpoint = _checkpoint_needed(M, K, N, a_group.device)
        Cm, _, ws = join_agg_fwd(a_group, a_key, a_val, b_key, b_group, b_val, M, K, N,
                                 precision, tol, unique=unique, for_backward=not checkpoint)
        ctx.save_for_backward(a_group, a_key, a_val, b_key, b_group, b_val)
        ctx.shape = (M, K, N)
        ctx.precision, ctx.tol, ctx.unique = precision, tol, unique
        ctx.ws = None if checkpoint else ws
        return Cm

    @staticmethod
    def backward(ctx, dC):
        a_group, a_key, a_val, b_key, b_group, b_val = ctx.saved_tensors
        M, K, N = ctx.shape
        need_a = a_val is not None and ctx.needs_input_grad[2]
        need_b = b_val is not None and ctx.needs_input_grad[5]
        dA = dB = None
        if need_a or need_b:
            dA, dB, _ = join_agg_bwd(a_group, a_key, a_val, b_key, b_group, b_val, M, K, N,
                                     dC.contiguous().to(torch.float64), need_a, need_b,
                                     ctx.precision, ctx.tol, ws=ctx.ws, unique=ctx.unique,
                                     saved_encodings=ctx.ws is not None)
        ctx.ws = None
        if dA is not None:
            dA = dA.to(a_val.dtype)
        if dB is not None:
            dB = dB.to(b_val.dtype)
        return (None, None, dA, None, None, dB) + (None,) * 7


def join_agg(a_group, a_key, a_val, b_key, b_group, b_val, M: int, K: int, N: int,
             precision: str = "fp64", tol: float = 0.0, unique: bool = False,
             checkpoint: Optional[bool] = None) -> torch.Tensor:
    """Differentiable C = join-aggregate (gradients for the value columns)."""
    return JoinAgg.apply(a_group, a_key, a_val, b_key, b_group, b_val, M, K, N, precision, tol,
                         unique, checkpoint)
