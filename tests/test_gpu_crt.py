"""The CRT mixed form (residues modulo small coprime moduli on the int8
matrix cores, Chinese-remainder reconstruction) against the oracle.

Two checks per case:
  * the reconstruction is exact arithmetic: C must equal the oracle's
    product of the same per-line integer truncations (the width the plan
    reports; exact 128-bit sum, one rounding) up to the roundings of the
    FP64 reconstruction;
  * against the true product, the certified guarantee
    |C - C*| <= tol (|X||Y|)[g,h] holds cell by cell (err_cw <= tol).
"""
import numpy as np
import pytest
import torch

from paper_2112_07552_amd import ops
from paper_2112_07552_amd import workloads as wl

from .gpu_util import abs_rel, cuda_or_skip, err_cw, to_orc

pytestmark = pytest.mark.gpu


def run_crt(orc, A, B, M, K, N, tol, unique):
    Cg, _, ws = ops.join_agg_fwd(A.group, A.key, A.val, B.key, B.group, B.val, M, K, N,
                                 precision="crt_i8", tol=tol, unique=unique)
    st, info = ops.sync_status(ws)
    C = Cg.cpu().numpy()
    RA, RB = to_orc(orc, A), to_orc(orc, B)
    X, _ = orc.encode_A(RA, M, K)
    Y, _ = orc.encode_B(RB, K, N)
    Co, _, _ = orc.join_agg(RA, RB, M, K, N)
    So, _, _ = orc.join_agg(abs_rel(orc, RA), abs_rel(orc, RB), M, K, N)
    return C, st, info, X, Y, Co, So


def check_reconstruction(orc, C, info, X, Y):
    """C is the oracle's product of the truncations to info['bits'] bits."""
    assert info["flags"] & ops._lib.TCU_FLAG_FALLBACK == 0 and info["exceptions"] == 0
    assert 1 <= info["slices"] <= 15 and 1 <= info["bits"] <= 53
    T = orc.trunc_product(X, Y, info["bits"])
    assert np.all(np.abs(C - T) <= 2.0 ** -50 * np.abs(T))


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
    C, st, info, X, Y, Co, So = run_crt(orc, A, B, M, K, N, tol, True)
    assert st == 0
    check_reconstruction(orc, C, info, X, Y)
    assert err_cw(C, Co, So) <= tol


def _sparse_long(dev):
    M, K, N = 40, 100_000, 50
    A = wl.random_relation(300_000, M, K, 57, 1, device=dev, values="loguniform")
    B = wl.random_relation(300_000, N, K, 57, 2, device=dev, values="loguniform")
    A = wl.Relation(torch.where(A.group == 7, torch.full_like(A.group, M + 1), A.group), A.key,
                    A.val)  # row 7 empty (its records out of range, reported)
    return A, B, M, K, N


def test_crt_long_contraction_and_zero_lines(orc):
    """K = 100000 (int32 sums up to 2^31), sparse encodings, an empty row."""
    dev = cuda_or_skip()
    A, B, M, K, N = _sparse_long(dev)
    C, st, info, X, Y, Co, So = run_crt(orc, A, B, M, K, N, 1e-9, False)
    assert st == ops._lib.TCU_ERR_KEY_RANGE and info["skipped_a"] > 0
    assert np.all(C[7] == 0.0)
    check_reconstruction(orc, C, info, X, Y)
    assert err_cw(C, Co, So) <= 1e-9


def test_crt_falls_back_to_fp64_without_a_certified_plan(orc):
    """The same sparse log-uniform product at 1e-12: some cell's certificate
    needs more bits than 53-bit truncations and 15 moduli provide, so the
    residue form cannot certify it and the product runs in FP64 (flagged),
    within the FP64 form's accuracy of its C."""
    dev = cuda_or_skip()
    A, B, M, K, N = _sparse_long(dev)
    C, st, info, X, Y, Co, So = run_crt(orc, A, B, M, K, N, 1e-12, False)
    assert info["flags"] & ops._lib.TCU_FLAG_FALLBACK and info["slices"] == 0
    C64, _, _ = ops.join_agg_fwd(A.group, A.key, A.val, B.key, B.group, B.val, M, K, N)
    # duplicate cells add in FP64 atomics (order-dependent last bits), so
    # compare within the FP64 form's own accuracy
    assert err_cw(C, C64.cpu().numpy(), So) <= 1e-13
    assert err_cw(C, Co, So) <= 1e-12


@pytest.mark.parametrize("precision", ["crt_i8", "split_i8", "split_bf16"])
def test_uncertifiable_cell_runs_in_fp64(orc, precision):
    """A cell whose terms all pair a value below 2^-7 of its row's maximum
    with a nonzero (magnitude code 0, so no lower bound of |X||Y| there):
    the product cannot be certified and runs in FP64, exactly as the FP64
    form (unique cells: the same encodings)."""
    dev = cuda_or_skip()
    # X row 0: 1e6 at key 0, 1e-6 at key 1; Y column 0: nonzero only at key 1
    g = torch.tensor([0, 0, 1, 1], dtype=torch.int32, device=dev)
    k = torch.tensor([0, 1, 0, 1], dtype=torch.int32, device=dev)
    v = torch.tensor([1e6, 1e-6, 2.0, 3.0], dtype=torch.float64, device=dev)
    h = torch.tensor([0, 1, 1], dtype=torch.int32, device=dev)
    kb = torch.tensor([1, 0, 1], dtype=torch.int32, device=dev)
    w = torch.tensor([5.0, 7.0, 11.0], dtype=torch.float64, device=dev)
    Cm, _, ws = ops.join_agg_fwd(g, k, v, kb, h, w, 2, 2, 2, precision=precision, tol=1e-12,
                                 unique=True)
    st, info = ops.sync_status(ws)
    assert st == 0 and info["flags"] == ops._lib.TCU_FLAG_FALLBACK and info["need"] == 255
    C64, _, _ = ops.join_agg_fwd(g, k, v, kb, h, w, 2, 2, 2, unique=True)
    assert torch.equal(Cm, C64)


# Tolerances that drive the plan through every modulus count.  With K = 1
# and U[-1,1) values, every cell's certificate ratio lies in [2/t, 4/t], so
# t = 1.5 2^-j gives a width of j + 2 bits and, with line sums below 1, the
# count is the first L whose moduli exceed 2 (j + 2) + 1 bits: j = 0, 3, 7,
# ..., 47, 49 give L = 1 .. 14.  K = 1024 adds log2 of the line sums (about
# 9 bits) and reaches L = 15.  The reconstruction has one kernel instance per
# count.
_L_SWEEP = [(1, 1.5 * 2.0 ** -j) for j in (0, 3, 7, 11, 15, 19, 23, 27, 31, 35, 39, 43, 47, 49)] \
    + [(1024, 1.5 * 2.0 ** -49)]


@pytest.mark.parametrize("K,tol", _L_SWEEP)
def test_crt_modulus_counts(orc, K, tol):
    dev = cuda_or_skip()
    M, N = 70, 90
    A, B = wl.mm_query(M, K, N, seed=K + 7, values="uniform", device=dev)
    C, st, info, X, Y, Co, So = run_crt(orc, A, B, M, K, N, tol, True)
    assert st == 0
    check_reconstruction(orc, C, info, X, Y)
    assert err_cw(C, Co, So) <= tol
    _seen_counts.append(info["slices"])


_seen_counts = []


def test_crt_sweep_covered_every_count():
    """Runs after the sweep above: every modulus count 1 .. 15 occurred."""
    cuda_or_skip()
    if len(_seen_counts) != len(_L_SWEEP):
        pytest.skip("the sweep did not run in this session")
    assert sorted(_seen_counts) == list(range(1, 16))


@pytest.mark.parametrize("precision", ["crt_i8", "split_i8"])
@pytest.mark.parametrize("M,K,N,kind,tol", [
    (300, 257, 129, "loguniform", 1e-12),
    (200, 1000, 170, "mixture", 1e-12),
    (150, 700, 260, "uniform", 1e-9),
])
def test_certificate_need_matches_the_oracle(orc, precision, M, K, N, kind, tol):
    """The plan's certificate (step a0) against the oracle's, written from its
    definition without rounding margins: the device's need is the oracle's,
    or one more where the device's margins (relative 2^-20 on the line sums,
    2^-40 on the comparison) tip a cell over a power of two."""
    dev = cuda_or_skip()
    A, B = wl.mm_query(M, K, N, seed=M + 3 * K, values=kind, device=dev)
    Cg, _, ws = ops.join_agg_fwd(A.group, A.key, A.val, B.key, B.group, B.val, M, K, N,
                                 precision=precision, tol=tol, unique=True)
    st, info = ops.sync_status(ws)
    assert st == 0
    RA, RB = to_orc(orc, A), to_orc(orc, B)
    X, _ = orc.encode_A(RA, M, K)
    Y, _ = orc.encode_B(RB, K, N)
    lib = ops._lib.load()
    # the tolerances the device compares against (tcudb.h, tcu_mixed_plan)
    tcrt = (tol - 2.0 ** -52) * (1 - 2.0 ** -40)
    if precision == "crt_i8":
        tdig = [0.0] * 9
    else:
        # int8 digits: one FP64 addition per diagonal for K <= 16384
        tdig = [0.0] + [(tol - S * 2.0 ** -52) * (1 - 2.0 ** -40) for S in range(1, 9)]
    nb, ns, umax = orc.certificate(X, Y, tcrt, tdig)
    want = nb if precision == "crt_i8" else ns
    assert info["need"] in (want, want + 1), (info, want)
    assert info["exceptions"] == 0  # products this small never scan for them
    if info["flags"] & ops._lib.TCU_FLAG_FALLBACK == 0:
        # the plan the host derives from the oracle's need (same u up to the margin)
        got = ops.mixed_plan(precision, K, tol, info["need"], min(umax) * (1 + 2.0 ** -20))
        assert got[0] == info["slices"]
        if precision == "crt_i8":
            assert got[1] == info["bits"]


def test_crt_product_in_several_launches(orc):
    """A product with more workgroups than one launch takes: 8604^2 cells in
    34 x 34 tiles and 15 moduli run as two launches per k-chunk (14 moduli,
    then 1).  Sampled whole rows are still the oracle's product of the
    truncations, and within the tolerance of the oracle's C."""
    dev = cuda_or_skip()
    M = N = 8604
    K = 1024
    tol = 1.5 * 2.0 ** -49
    A, B = wl.mm_query(M, K, N, seed=21, values="uniform", device=dev)
    Cg, _, ws = ops.join_agg_fwd(A.group, A.key, A.val, B.key, B.group, B.val, M, K, N,
                                 precision="crt_i8", tol=tol, unique=True)
    st, info = ops.sync_status(ws)
    assert st == 0 and info["flags"] == 0 and info["slices"] == 15
    rows = np.sort(np.random.default_rng(5).choice(M, 48, replace=False))
    C = Cg[torch.as_tensor(rows, device=dev)].cpu().numpy()
    RA, RB = to_orc(orc, A), to_orc(orc, B)
    X, _ = orc.encode_A(RA, M, K)
    Y, _ = orc.encode_B(RB, K, N)
    # each row's truncation depends on that row alone
    T = orc.trunc_product(np.ascontiguousarray(X[rows]), Y, info["bits"])
    assert np.all(np.abs(C - T) <= 2.0 ** -50 * np.abs(T))
    Co, _, _ = orc.join_agg(RA, RB, M, K, N, rows=rows)
    So, _, _ = orc.join_agg(abs_rel(orc, RA), abs_rel(orc, RB), M, K, N, rows=rows)
    assert err_cw(C, Co, So) <= tol


def test_crt_wide_tiles_ragged(orc):
    """Outputs of 16384 columns or more run on 256 x 384 tiles (residue
    products and certificate); 16500 columns leave a ragged last tile.  The
    result is the oracle's product of the truncations, within tol of C."""
    dev = cuda_or_skip()
    M, K, N = 96, 700, 16500
    A, B = wl.mm_query(M, K, N, seed=23, values="loguniform", device=dev)
    C, st, info, X, Y, Co, So = run_crt(orc, A, B, M, K, N, 1e-12, True)
    assert st == 0
    check_reconstruction(orc, C, info, X, Y)
    assert err_cw(C, Co, So) <= 1e-12
