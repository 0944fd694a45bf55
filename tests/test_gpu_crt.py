"""The CRT mixed form (residues modulo small coprime moduli on the int8
matrix cores, Chinese-remainder reconstruction) against the oracle.

Two checks per case:
  * the reconstruction is exact arithmetic: C must equal the oracle's
    product of the same per-line integer truncations (exact 128-bit sum,
    one rounding) up to the two roundings of the FP64 reconstruction;
  * against the true product, the planned bound
    |C - C*| <= tol * K * max|X[g,:]| * max|Y[:,h]| holds cell by cell.
"""
import numpy as np
import pytest
import torch

from paper_2112_07552_amd import ops
from paper_2112_07552_amd import workloads as wl

from .gpu_util import abs_rel, cuda_or_skip, err_cw, to_orc

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("M,K,N,kind,tol", [
    (64, 96, 80, "uniform", 1e-12),
    (300, 257, 129, "loguniform", 1e-12),    # ragged tiles and k-steps
    (1, 5000, 3, "mixture", 1e-12),          # a single row, long contraction
    (513, 1, 700, "uniform", 1e-9),          # K = 1
    (1024, 1024, 1024, "loguniform", 1e-12),
    (200, 131, 260, "uniform", 1e-6),        # few moduli
])
def test_crt_reconstructs_truncated_product(orc, M, K, N, kind, tol):
    dev = cuda_or_skip()
    A, B = wl.mm_query(M, K, N, seed=M + K + N, values=kind, device=dev)
    Cg, _, ws = ops.join_agg_fwd(A.group, A.key, A.val, B.key, B.group, B.val, M, K, N,
                                 precision="crt_i8", tol=tol, unique=True)
    st, info = ops.sync_status(ws)
    L, bits = ops.crt_plan(K, tol)
    assert st == 0 and info["slices"] == L
    RA, RB = to_orc(orc, A), to_orc(orc, B)
    X, _ = orc.encode_A(RA, M, K)
    Y, _ = orc.encode_B(RB, K, N)
    T = orc.trunc_product(X, Y, bits)
    C = Cg.cpu().numpy()
    assert np.all(np.abs(C - T) <= 2.0 ** -50 * np.abs(T))
    # the planned bound against the true product (oracle, Dot2)
    Co, _, _ = orc.join_agg(RA, RB, M, K, N)
    bound = tol * K * np.outer(np.abs(X).max(axis=1), np.abs(Y).max(axis=0))
    assert np.all(np.abs(C - Co) <= bound)


def test_crt_long_contraction_and_zero_lines(orc):
    """K = 100000 (13-14 moduli, int32 sums up to 2^31), zero rows and columns."""
    dev = cuda_or_skip()
    M, K, N = 40, 100_000, 50
    A = wl.random_relation(300_000, M, K, 57, 1, device=dev, values="loguniform")
    B = wl.random_relation(300_000, N, K, 57, 2, device=dev, values="loguniform")
    A = wl.Relation(torch.where(A.group == 7, torch.full_like(A.group, M + 1), A.group), A.key,
                    A.val)  # row 7 empty (its records out of range, reported)
    Cg, _, ws = ops.join_agg_fwd(A.group, A.key, A.val, B.key, B.group, B.val, M, K, N,
                                 precision="crt_i8", tol=1e-12)
    st, info = ops.sync_status(ws)
    assert st == ops._lib.TCU_ERR_KEY_RANGE and info["skipped_a"] > 0
    C = Cg.cpu().numpy()
    assert np.all(C[7] == 0.0)
    RA, RB = to_orc(orc, A), to_orc(orc, B)
    X, _ = orc.encode_A(RA, M, K)
    Y, _ = orc.encode_B(RB, K, N)
    _, bits = ops.crt_plan(K, 1e-12)
    T = orc.trunc_product(X, Y, bits)
    assert np.all(np.abs(C - T) <= 2.0 ** -50 * np.abs(T))
    Co, _, _ = orc.join_agg(RA, RB, M, K, N)
    So, _, _ = orc.join_agg(abs_rel(orc, RA), abs_rel(orc, RB), M, K, N)
    bound = 1e-12 * K * np.outer(np.abs(X).max(axis=1), np.abs(Y).max(axis=0))
    assert np.all(np.abs(C - Co) <= bound)


def test_crt_plan_limits():
    cuda_or_skip()
    assert ops.crt_plan(4096, 1e-12) == (13, 42)
    with pytest.raises(ops.TcuError):
        ops.crt_plan(131072, 1e-12)   # int32 sums would no longer be exact
    with pytest.raises(ops.TcuError):
        ops.crt_plan(100, 1e-17)      # beyond 53-bit inputs


# one tolerance per modulus count the plan can pick (K = 1 reaches L = 2,
# K = 257 the counts 3 .. 15): the reconstruction has one kernel instance per
# count, and each must rebuild the truncated product
_L_SWEEP = [(1, 0.1)] + [(257, t) for t in (0.1, 1e-2, 1e-3, 1e-4, 1e-5, 1e-7, 1e-8, 1e-9,
                                            1e-10, 1e-11, 1e-13, 1e-14, 1e-15)]


@pytest.mark.parametrize("K,tol", _L_SWEEP)
def test_crt_every_modulus_count(orc, K, tol):
    dev = cuda_or_skip()
    M, N = 70, 90
    A, B = wl.mm_query(M, K, N, seed=K + 7, values="loguniform", device=dev)
    Cg, _, ws = ops.join_agg_fwd(A.group, A.key, A.val, B.key, B.group, B.val, M, K, N,
                                 precision="crt_i8", tol=tol, unique=True)
    st, info = ops.sync_status(ws)
    L, bits = ops.crt_plan(K, tol)
    assert st == 0 and info["slices"] == L
    RA, RB = to_orc(orc, A), to_orc(orc, B)
    X, _ = orc.encode_A(RA, M, K)
    Y, _ = orc.encode_B(RB, K, N)
    T = orc.trunc_product(X, Y, bits)
    C = Cg.cpu().numpy()
    assert np.all(np.abs(C - T) <= 2.0 ** -50 * np.abs(T))
    Co, _, _ = orc.join_agg(RA, RB, M, K, N)
    bound = tol * K * np.outer(np.abs(X).max(axis=1), np.abs(Y).max(axis=0))
    assert np.all(np.abs(C - Co) <= bound)


def test_crt_sweep_covers_every_count():
    """The sweep above reaches every modulus count from 2 to the maximum
    (the plan never picks one modulus); host-side plan only."""
    counts = sorted(ops.crt_plan(K, tol)[0] for K, tol in _L_SWEEP)
    assert counts == list(range(2, 16))
