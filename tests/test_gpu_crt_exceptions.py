"""The residue form's reconstruction at the edge of its modulus plan, and
its exception path: cells recomputed one by one when that lets the rest
of the product run with fewer moduli, or at all.

  * Near M / 2: every entry 1 - 2^-53 makes every cell's truncated integer
    product P = K (2^b - 1)^2, as large as the plan's bound |P| <=
    2^(2b) K allows.  At K = 3570 and 41 bits the plan takes 12 moduli with
    |P| / M = 0.4994, so q = round(S / M) must come out right within 2^-39
    of a half.
  * Exceptions: a product whose cells the certificate bounds at about 43
    bits, except one cell it cannot bound (the row's and the column's
    supports meet only at an entry below 2^-7 of its row's maximum, whose
    magnitude code is 0).  Without exceptions the whole product would run
    in FP64; with them it runs on the int8 matrix cores and that one cell is
    recomputed as a compensated dot product.
"""
import numpy as np
import pytest
import torch

from paper_2112_07552_amd import ops

from .gpu_util import abs_rel, cuda_or_skip, dense_relation_from_matrix, err_cw, to_orc

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_reconstruction_at_half_the_modulus_product(orc, sign):
    dev = cuda_or_skip()
    M, K, N = 64, 3570, 64
    v = 1.0 - 2.0 ** -53
    X = torch.full((M, K), sign * v, dtype=torch.float64, device=dev)
    Y = torch.full((K, N), v, dtype=torch.float64, device=dev)
    A = dense_relation_from_matrix(X, False)
    B = dense_relation_from_matrix(Y, True)
    Cg, _, ws = ops.join_agg_fwd(A.group, A.key, A.val, B.key, B.group, B.val, M, K, N,
                                 precision="crt_i8", tol=1e-12, unique=True)
    st, info = ops.sync_status(ws)
    assert st == 0 and info["flags"] == 0 and info["exceptions"] == 0
    # 2 * 41 + log2(3570) + 1 = 94.8017 bits against 94.8033 for 12 moduli
    assert info["bits"] == 41 and info["slices"] == 12, info
    C = Cg.cpu().numpy()
    want = sign * 3570.0 * (1.0 - 2.0 ** -41) ** 2  # P 2^-82, P = K (2^41 - 1)^2
    assert np.all(C == want)
    Xo, Yo = X.cpu().numpy(), Y.cpu().numpy()
    T = orc.trunc_product(Xo, Yo, 41)
    assert np.array_equal(C, T)
    RA, RB = to_orc(orc, A), to_orc(orc, B)
    Co, _, _ = orc.join_agg(RA, RB, M, K, N)
    So, _, _ = orc.join_agg(abs_rel(orc, RA), abs_rel(orc, RB), M, K, N)
    assert err_cw(C, Co, So) <= 1e-12


def _one_uncertifiable_cell(dev, M, K, N, g, h, k1):
    gen = torch.Generator(device=dev)
    gen.manual_seed(77)
    X = torch.rand((M, K), generator=gen, dtype=torch.float64, device=dev) * 2 - 1
    Y = torch.rand((K, N), generator=gen, dtype=torch.float64, device=dev) * 2 - 1
    X[g, K // 2:] = 0.0          # row g lives on the first half of the keys ...
    X[g, k1] = 1e-9              # ... and one tiny entry in the second (code 0)
    Y[: K // 2, h] = 0.0         # column h lives on the second half
    return X, Y


def test_uncertifiable_cell_is_recomputed_alone(orc):
    dev = cuda_or_skip()
    M, K, N = 2048, 1024, 2048
    g, h, k1 = 1000, 1500, 700
    X, Y = _one_uncertifiable_cell(dev, M, K, N, g, h, k1)
    A = dense_relation_from_matrix(X, False)
    B = dense_relation_from_matrix(Y, True)
    Cg, _, ws = ops.join_agg_fwd(A.group, A.key, A.val, B.key, B.group, B.val, M, K, N,
                                 precision="crt_i8", tol=1e-12, unique=True)
    st, info = ops.sync_status(ws)
    assert st == 0 and info["need"] == 255, info
    assert info["flags"] & ops._lib.TCU_FLAG_FALLBACK == 0, info
    assert info["exceptions"] == 1 and 1 <= info["slices"] <= 15, info
    rows = np.unique(np.concatenate([[g], np.random.default_rng(3).choice(M, 40, replace=False)]))
    C = Cg[torch.as_tensor(rows, device=dev)].cpu().numpy()
    RA, RB = to_orc(orc, A), to_orc(orc, B)
    Co, _, _ = orc.join_agg(RA, RB, M, K, N, rows=rows)
    So, _, _ = orc.join_agg(abs_rel(orc, RA), abs_rel(orc, RB), M, K, N, rows=rows)
    assert err_cw(C, Co, So) <= 1e-12
    # the recomputed cell: 1e-9 * Y[k1, h], within a rounding or two
    ig = int(np.searchsorted(rows, g))
    exact = 1e-9 * float(Y[k1, h])
    assert abs(C[ig, h] - exact) <= 2.0 ** -51 * abs(exact)
    # every other sampled cell is the residue form's: the product of the
    # truncations to the plan's width
    Xo, Yo = X.cpu().numpy(), Y.cpu().numpy()
    T = orc.trunc_product(np.ascontiguousarray(Xo[rows]), Yo, info["bits"])
    mask = np.ones_like(T, dtype=bool)
    mask[ig, h] = False
    assert np.all(np.abs(C - T)[mask] <= 2.0 ** -50 * np.abs(T)[mask])
    # the truncated product misses the cell by far more than the tolerance
    assert abs(T[ig, h] - exact) > 1e-9 * abs(exact)


def test_exceptions_leave_small_products_alone(orc):
    """The same structure at 128 x 64 x 128: a scan and a second read-back
    cost more than FP64 there, so the product falls back to FP64 whole."""
    dev = cuda_or_skip()
    M, K, N = 128, 64, 128
    X, Y = _one_uncertifiable_cell(dev, M, K, N, 5, 7, 40)
    A = dense_relation_from_matrix(X, False)
    B = dense_relation_from_matrix(Y, True)
    Cg, _, ws = ops.join_agg_fwd(A.group, A.key, A.val, B.key, B.group, B.val, M, K, N,
                                 precision="crt_i8", tol=1e-12, unique=True)
    st, info = ops.sync_status(ws)
    assert st == 0 and info["flags"] & ops._lib.TCU_FLAG_FALLBACK and info["exceptions"] == 0
    C64, _, _ = ops.join_agg_fwd(A.group, A.key, A.val, B.key, B.group, B.val, M, K, N,
                                 unique=True)
    assert torch.equal(Cg, C64)


def test_adjoint_products_recompute_their_uncertifiable_cells(orc):
    """The adjoint's products dX = dC Y^T and dY = X^T dC each hold one cell
    the certificate cannot bound (the same construction on dC's row g* and
    Y's row k*, and on X's column k0 and dC's column h0).  Both products run
    in the residue form with that cell recomputed alone; the two gradient
    records that read those cells, and a sample of the others, match the
    oracle's closed form within tol."""
    dev = cuda_or_skip()
    M = K = N = 2048
    gs, ks, h1 = 100, 300, 1500     # dX cell (gs, ks): dC row gs meets Y row ks at h1 only
    k0, h0, g1 = 700, 200, 1800     # dY cell (k0, h0): X column k0 meets dC column h0 at g1 only
    gen = torch.Generator(device=dev)
    gen.manual_seed(91)
    X = torch.rand((M, K), generator=gen, dtype=torch.float64, device=dev) * 2 - 1
    Y = torch.rand((K, N), generator=gen, dtype=torch.float64, device=dev) * 2 - 1
    W = torch.rand((M, N), generator=gen, dtype=torch.float64, device=dev) * 2 - 1
    W[gs, N // 2:] = 0.0
    W[gs, h1] = 1e-9
    Y[ks, : N // 2] = 0.0
    X[M // 2:, k0] = 0.0
    X[g1, k0] = 1e-9
    W[: M // 2, h0] = 0.0
    A = dense_relation_from_matrix(X, False)
    B = dense_relation_from_matrix(Y, True)
    dA, dB, ws = ops.join_agg_bwd(A.group, A.key, A.val, B.key, B.group, B.val, M, K, N, W,
                                  precision="crt_i8", tol=1e-12, unique=True)
    st, info = ops.sync_status(ws)  # the last product: dY
    assert st == 0 and info["need"] == 255, info
    assert info["flags"] & ops._lib.TCU_FLAG_FALLBACK == 0 and info["exceptions"] >= 1, info
    ia = np.unique(np.concatenate([[gs * K + ks],
                                   np.random.default_rng(4).choice(M * K, 2000, replace=False)]))
    ib = np.unique(np.concatenate([[k0 * N + h0],
                                   np.random.default_rng(5).choice(K * N, 2000, replace=False)]))
    RA, RB = to_orc(orc, A), to_orc(orc, B)
    Wn = W.cpu().numpy()
    ga = orc.grad(RA, RB, M, K, N, Wn, "A", idx=ia)
    gb = orc.grad(RA, RB, M, K, N, Wn, "B", idx=ib)
    sa = orc.grad(abs_rel(orc, RA), abs_rel(orc, RB), M, K, N, np.abs(Wn), "A", idx=ia)
    sb = orc.grad(abs_rel(orc, RA), abs_rel(orc, RB), M, K, N, np.abs(Wn), "B", idx=ib)
    dAn, dBn = dA.cpu().numpy()[ia], dB.cpu().numpy()[ib]
    assert err_cw(dAn, ga, sa) <= 1e-12
    assert err_cw(dBn, gb, sb) <= 1e-12
    # the two recomputed cells, within a rounding or two of their one term
    exact_a = 1e-9 * float(Y[ks, h1])
    exact_b = 1e-9 * float(W[g1, h0])
    got_a = float(dA[gs * K + ks])
    got_b = float(dB[k0 * N + h0])
    assert abs(got_a - exact_a) <= 2.0 ** -51 * abs(exact_a)
    assert abs(got_b - exact_b) <= 2.0 ** -51 * abs(exact_b)


def test_exceptions_at_ragged_corners_of_wide_tiles(orc):
    """Rows 0 and m - 1 and columns 0 and n - 1 restricted as above: the four
    corner cells (ragged last row block, ragged last 256 x 384 tile column)
    cannot be bounded and are recomputed alone; everything else is the
    residue form's."""
    dev = cuda_or_skip()
    M, K, N = 300, 1024, 16500
    k1 = 700
    gen = torch.Generator(device=dev)
    gen.manual_seed(93)
    X = torch.rand((M, K), generator=gen, dtype=torch.float64, device=dev) * 2 - 1
    Y = torch.rand((K, N), generator=gen, dtype=torch.float64, device=dev) * 2 - 1
    for g in (0, M - 1):
        X[g, K // 2:] = 0.0
        X[g, k1] = 1e-9
    for h in (0, N - 1):
        Y[: K // 2, h] = 0.0
    A = dense_relation_from_matrix(X, False)
    B = dense_relation_from_matrix(Y, True)
    Cg, _, ws = ops.join_agg_fwd(A.group, A.key, A.val, B.key, B.group, B.val, M, K, N,
                                 precision="crt_i8", tol=1e-12, unique=True)
    st, info = ops.sync_status(ws)
    assert st == 0 and info["need"] == 255, info
    assert info["flags"] & ops._lib.TCU_FLAG_FALLBACK == 0 and info["exceptions"] >= 4, info
    rows = np.unique(np.concatenate([[0, M - 1], np.random.default_rng(6).choice(M, 30, replace=False)]))
    C = Cg[torch.as_tensor(rows, device=dev)].cpu().numpy()
    RA, RB = to_orc(orc, A), to_orc(orc, B)
    Co, _, _ = orc.join_agg(RA, RB, M, K, N, rows=rows)
    So, _, _ = orc.join_agg(abs_rel(orc, RA), abs_rel(orc, RB), M, K, N, rows=rows)
    assert err_cw(C, Co, So) <= 1e-12
    for g in (0, M - 1):
        for h in (0, N - 1):
            exact = 1e-9 * float(Y[k1, h])
            got = C[int(np.searchsorted(rows, g)), h]
            assert abs(got - exact) <= 2.0 ** -51 * abs(exact), (g, h, got, exact)
