"""Pins of the FP64 CPU oracle against what the paper and mathematics fix.

None of these checks retypes the oracle's own evaluation: each compares it with
an independent route (exact rational brute force over all record pairs, a
library matrix product, the paper's closed forms of Section 3.3, exact integer
arithmetic, algebraic invariances), chosen so that a dropped term, a wrong
index, a swapped operand or a lost duplicate fails at least one of them.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
import torch

from paper_2112_07552_amd import workloads as wl

from .paper_tables import error_table

U = 2.0 ** -53  # unit roundoff of binary64


def to_rel(orc, R):
    return orc.Rel(R.group.numpy(), R.key.numpy(), None if R.val is None else R.val.numpy())


def brute_force(A, B, M, N, K=None):
    """SQL nested-loop evaluation with exact rationals: every pair (a, b).

    Records with a key outside [0, K) or a group outside its range are not
    part of the operator's input (the operator skips and reports them)."""
    C = {}
    cnt = {}
    absum = {}
    for i in range(A.n):
        g, k = int(A.group[i]), int(A.key[i])
        if not (0 <= g < M) or (K is not None and not (0 <= k < K)):
            continue
        v = Fraction(1) if A.val is None else Fraction(float(A.val[i]))
        for j in range(B.n):
            kb, h = int(B.key[j]), int(B.group[j])
            if kb != k or not (0 <= h < N):
                continue
            w = Fraction(1) if B.val is None else Fraction(float(B.val[j]))
            C[(g, h)] = C.get((g, h), Fraction(0)) + v * w
            cnt[(g, h)] = cnt.get((g, h), 0) + 1
            absum[(g, h)] = absum.get((g, h), Fraction(0)) + abs(v * w)
    return C, cnt, absum


def small_case(seed, nA, nB, M, K, N, values="uniform", bad=0.0, nulls=False):
    A = wl.random_relation(nA, M, K, seed, 1, values=values, bad_fraction=bad)
    B = wl.random_relation(nB, N, K, seed, 2, values=values, bad_fraction=bad)
    if nulls:
        A = wl.Relation(A.group, A.key, None)
    return A, B


def check_against_brute(orc, A, B, M, K, N):
    C, cnt, _ = orc.join_agg(to_rel(orc, A), to_rel(orc, B), M, K, N, with_count=True)
    exact, ecnt, absum = brute_force(A, B, M, N, K)
    for g in range(M):
        for h in range(N):
            e = exact.get((g, h), Fraction(0))
            npairs = ecnt.get((g, h), 0)
            assert cnt[g, h] == npairs, (g, h)
            err = abs(Fraction(float(C[g, h])) - e)
            bound = Fraction(U) * abs(e) + Fraction(2 * (npairs * U) ** 2) * absum.get((g, h), 0)
            assert err <= bound, (g, h, float(err), float(bound))


@pytest.mark.parametrize("seed,nA,nB,M,K,N", [
    (0, 40, 50, 5, 4, 6),      # duplicates of (g,k) and (k,h)
    (1, 64, 64, 3, 9, 2),      # keys present in only one relation
    (2, 30, 60, 1, 3, 7),      # M = 1
    (3, 60, 30, 6, 1, 5),      # K = 1: every pair joins
    (4, 50, 50, 4, 5, 1),      # N = 1
    (5, 0, 20, 3, 3, 3),       # empty A
    (6, 20, 0, 3, 3, 3),       # empty B
    (7, 64, 64, 8, 40, 8),     # sparse join: most keys unmatched
])
def test_brute_force_values(orc, seed, nA, nB, M, K, N):
    A, B = small_case(seed, nA, nB, M, K, N)
    check_against_brute(orc, A, B, M, K, N)


def test_brute_force_out_of_range_records_skipped(orc):
    A, B = small_case(11, 64, 64, 4, 6, 5, bad=0.3)
    assert int(((A.group < 0) | (A.group >= 4) | (A.key < 0) | (A.key >= 6)).sum()) > 0
    check_against_brute(orc, A, B, 4, 6, 5)


def test_brute_force_count_semantics(orc):
    """NULL value column = COUNT (Section 3.3): C equals the pair count."""
    A, B = small_case(12, 50, 60, 4, 5, 6)
    A = wl.Relation(A.group, A.key, None)
    B = wl.Relation(B.group, B.key, None)
    C, cnt, _ = orc.join_agg(to_rel(orc, A), to_rel(orc, B), 4, 5, 6, with_count=True)
    _, ecnt, _ = brute_force(A, B, 4, 6, 5)
    for g in range(4):
        for h in range(6):
            assert C[g, h] == ecnt.get((g, h), 0) == cnt[g, h]


def test_cells_match_brute_force(orc):
    A, B = small_case(13, 64, 64, 5, 6, 7, bad=0.1)
    exact, ecnt, _ = brute_force(A, B, 5, 7, 6)
    cg = np.array([g for g in range(-1, 6) for h in range(-1, 8)], dtype=np.int32)
    ch = np.array([h for g in range(-1, 6) for h in range(-1, 8)], dtype=np.int32)
    vals, cnts = orc.join_agg_cells(to_rel(orc, A), to_rel(orc, B), 5, 6, 7, cg, ch)
    for c in range(cg.shape[0]):
        e = exact.get((int(cg[c]), int(ch[c])), Fraction(0))
        assert abs(Fraction(float(vals[c])) - e) <= Fraction(U) * abs(e) + Fraction(1, 2**100)
        assert cnts[c] == ecnt.get((int(cg[c]), int(ch[c])), 0)


@pytest.mark.parametrize("M,K,N", [(64, 48, 80), (128, 128, 128), (1, 200, 3)])
def test_dense_tables_match_library_dgemm(orc, M, K, N):
    """Full dense tables: the join-aggregate equals a matrix product of the
    encodings (Section 3.3); numpy's DGEMM is an independent route."""
    A, B = wl.mm_query(M, K, N, seed=5)
    X = np.zeros((M, K))
    X[A.group.numpy(), A.key.numpy()] = A.val.numpy()
    Y = np.zeros((K, N))
    Y[B.key.numpy(), B.group.numpy()] = B.val.numpy()
    C, _, _ = orc.join_agg(to_rel(orc, A), to_rel(orc, B), M, K, N)
    ref = X @ Y
    scale = np.abs(X) @ np.abs(Y)
    assert np.all(np.abs(C - ref) <= 2 * K * U * scale + 1e-300)


@pytest.mark.parametrize("lo,hi", [(lo, hi) for lo, hi, _ in error_table()[1] if hi <= 2**15])
def test_integer_values_exact(orc, lo, hi):
    """Integer-valued inputs (the rows of Table "error", Section 5.4.1, read
    from tests/golden/): every partial sum is an integer below 2^53, so C is
    exact; int64 matmul is the exact reference."""
    M = K = N = 96
    A, B = wl.mm_query(M, K, N, seed=6, values="int", lo=lo, hi=hi)
    Xi = np.zeros((M, K), dtype=np.int64)
    Xi[A.group.numpy(), A.key.numpy()] = A.val.numpy().astype(np.int64)
    Yi = np.zeros((K, N), dtype=np.int64)
    Yi[B.key.numpy(), B.group.numpy()] = B.val.numpy().astype(np.int64)
    C, _, _ = orc.join_agg(to_rel(orc, A), to_rel(orc, B), M, K, N)
    assert np.array_equal(C, (Xi @ Yi).astype(np.float64))


def test_error_table_rows_against_exact_integers(orc):
    """Every row of Table "error" (Section 5.4.1, tests/golden/): on integer
    inputs of that range the oracle's MAPE against exact big-integer C is at
    most the paper's figure at every size; below 2^15 it is 0, and for the
    +-2^31 row (products up to 2^62, not representable in binary64) the
    compensated dot product stays within a few units in the last place."""
    sizes, rows = error_table()
    assert sizes == [2048, 4096, 8192, 16384, 32768]
    M = K = N = 40
    for lo, hi, paper in rows:
        A, B = wl.mm_query(M, K, N, seed=9, values="int", lo=lo, hi=hi)
        Xo = np.zeros((M, K), dtype=object)
        Yo = np.zeros((K, N), dtype=object)
        for g, k, v in zip(A.group.tolist(), A.key.tolist(), A.val.tolist()):
            Xo[g, k] = int(v)
        for k, h, v in zip(B.key.tolist(), B.group.tolist(), B.val.tolist()):
            Yo[k, h] = int(v)
        exact = Xo.dot(Yo)                       # Python integers, exact
        C, _, _ = orc.join_agg(to_rel(orc, A), to_rel(orc, B), M, K, N)
        rel = [abs(Fraction(float(c)) - e) / abs(e)
               for c, e in zip(C.ravel().tolist(), exact.ravel().tolist()) if e != 0]
        mape = 100.0 * float(sum(rel) / len(rel))
        assert all(mape <= p for p in paper)
        if hi <= 2**15:
            assert mape == 0.0
        else:
            assert max(rel) <= 4 * Fraction(U), float(max(rel))


def test_lemma_q3_column_sums(orc):
    """Lemma Q3 (Section 3.3): 1^T C = (1^T X) Y, i.e. summing C over g equals
    grouping A by key first.  Evaluated exactly with rationals."""
    M, K, N = 7, 9, 8
    A, B = small_case(21, 64, 64, M, K, N)
    C, _, _ = orc.join_agg(to_rel(orc, A), to_rel(orc, B), M, K, N)
    hA = [Fraction(0)] * K
    for i in range(A.n):
        if 0 <= int(A.group[i]) < M and 0 <= int(A.key[i]) < K:
            hA[int(A.key[i])] += Fraction(float(A.val[i]))
    col = [Fraction(0)] * N
    for j in range(B.n):
        k, h = int(B.key[j]), int(B.group[j])
        if 0 <= k < K and 0 <= h < N:
            col[h] += hA[k] * Fraction(float(B.val[j]))
    for h in range(N):
        s = sum(Fraction(float(C[g, h])) for g in range(M))
        assert abs(s - col[h]) <= Fraction(4 * U) * sum(abs(Fraction(float(C[g, h]))) for g in range(M)) + Fraction(1, 2**200)


def test_q4_total(orc):
    """Q4 (Section 3.3): the total of C equals sum_k hA[k] hB[k] with hA, hB
    the per-key sums of each relation's values (matrix-vector reductions)."""
    M, K, N = 6, 11, 5
    A, B = small_case(22, 64, 64, M, K, N)
    C, _, _ = orc.join_agg(to_rel(orc, A), to_rel(orc, B), M, K, N)
    hA = [Fraction(0)] * K
    hB = [Fraction(0)] * K
    for i in range(A.n):
        if 0 <= int(A.group[i]) < M and 0 <= int(A.key[i]) < K:
            hA[int(A.key[i])] += Fraction(float(A.val[i]))
    for j in range(B.n):
        if 0 <= int(B.group[j]) < N and 0 <= int(B.key[j]) < K:
            hB[int(B.key[j])] += Fraction(float(B.val[j]))
    total = sum(hA[k] * hB[k] for k in range(K))
    s = sum(Fraction(float(x)) for x in C.ravel())
    assert abs(s - total) <= Fraction(4 * U) * sum(abs(Fraction(float(x))) for x in C.ravel()) + Fraction(1, 2**200)


def test_identity_relation_gives_encoding(orc):
    """A = identity records (g = k, value 1): C equals B's encoding exactly."""
    K, N = 50, 40
    B = wl.random_relation(500, N, K, 31, 2)
    idx = torch.arange(K, dtype=torch.int32)
    A = wl.Relation(idx, idx.clone(), torch.ones(K, dtype=torch.float64))
    C, _, _ = orc.join_agg(to_rel(orc, A), to_rel(orc, B), K, K, N)
    # B's encoding computed as exact rationals, then rounded once
    Y = [[Fraction(0)] * N for _ in range(K)]
    for j in range(B.n):
        Y[int(B.key[j])][int(B.group[j])] += Fraction(float(B.val[j]))
    for k in range(K):
        for h in range(N):
            assert C[k, h] == float(Y[k][h])


def test_bilinear_scaling_exact(orc):
    M, K, N = 32, 24, 40
    A, B = small_case(41, 600, 700, M, K, N)
    C, _, _ = orc.join_agg(to_rel(orc, A), to_rel(orc, B), M, K, N)
    A2 = wl.Relation(A.group, A.key, A.val * 2.0)
    B4 = wl.Relation(B.group, B.key, B.val * 0.25)
    C2, _, _ = orc.join_agg(to_rel(orc, A2), to_rel(orc, B4), M, K, N)
    assert np.array_equal(C2, C * 0.5)


def test_role_swap_transposes(orc):
    M, K, N = 20, 17, 30
    A, B = small_case(42, 500, 400, M, K, N)
    C, cnt, _ = orc.join_agg(to_rel(orc, A), to_rel(orc, B), M, K, N, with_count=True)
    # B as the left relation (group h, key k), A as the right one (key k, group g)
    Ct, cntt, _ = orc.join_agg(to_rel(orc, B), to_rel(orc, A), N, K, M, with_count=True)
    assert np.array_equal(cnt, cntt.T)
    scale = np.abs(C) + 1e-300
    assert np.all(np.abs(C - Ct.T) <= 2 * U * scale + 1e-30)


def test_record_order_invariance(orc):
    M, K, N = 24, 20, 28
    A, B = small_case(43, 800, 900, M, K, N)
    C, cnt, _ = orc.join_agg(to_rel(orc, A), to_rel(orc, B), M, K, N, with_count=True)
    g = torch.Generator().manual_seed(0)
    pa, pb = torch.randperm(A.n, generator=g), torch.randperm(B.n, generator=g)
    A2 = wl.Relation(A.group[pa], A.key[pa], A.val[pa])
    B2 = wl.Relation(B.group[pb], B.key[pb], B.val[pb])
    C2, cnt2, _ = orc.join_agg(to_rel(orc, A2), to_rel(orc, B2), M, K, N, with_count=True)
    assert np.array_equal(cnt, cnt2)
    assert np.all(np.abs(C - C2) <= 2 * U * np.abs(C) + 1e-30)


def test_rows_subset_and_cells_agree_with_full(orc):
    M, K, N = 40, 30, 36
    A, B = small_case(44, 2000, 2000, M, K, N, bad=0.05)
    rA, rB = to_rel(orc, A), to_rel(orc, B)
    C, cnt, _ = orc.join_agg(rA, rB, M, K, N, with_count=True)
    rows = np.array([39, 0, 7, 7, 22], dtype=np.int32)
    Cr, cntr, _ = orc.join_agg(rA, rB, M, K, N, rows=rows, with_count=True)
    assert np.array_equal(Cr, C[rows]) and np.array_equal(cntr, cnt[rows])
    rng = np.random.default_rng(0)
    cg = rng.integers(0, M, 300).astype(np.int32)
    ch = rng.integers(0, N, 300).astype(np.int32)
    v, c = orc.join_agg_cells(rA, rB, M, K, N, cg, ch)
    assert np.array_equal(c, cnt[cg, ch])
    assert np.all(np.abs(v - C[cg, ch]) <= 2 * U * np.abs(C[cg, ch]) + 1e-30)


def test_freivalds_matches_full_product(orc):
    M, K, N = 50, 45, 55
    A, B = small_case(45, 3000, 3000, M, K, N, bad=0.05)
    rA, rB = to_rel(orc, A), to_rel(orc, B)
    C, _, _ = orc.join_agg(rA, rB, M, K, N)
    r = np.where(np.random.default_rng(1).random(N) < 0.5, -1.0, 1.0)
    lhs = np.array([math.fsum(C[g] * r) for g in range(M)])
    rhs = orc.freivalds(rA, rB, M, K, N, r)
    tol = 4 * U * (np.abs(C) @ np.ones(N)) + 1e-30
    assert np.all(np.abs(lhs - rhs) <= tol)


def test_encode_definition(orc):
    """Encoding (Section 3.1/3.3): X[g,k] is the sum of the values placed at
    (g,k); exact rationals, duplicates included, out-of-range skipped."""
    M, K = 9, 7
    A = wl.random_relation(300, M, K, 51, 1, bad_fraction=0.1)
    X, skipped = orc.encode_A(to_rel(orc, A), M, K)
    ref = [[Fraction(0)] * K for _ in range(M)]
    nbad = 0
    for i in range(A.n):
        g, k = int(A.group[i]), int(A.key[i])
        if 0 <= g < M and 0 <= k < K:
            ref[g][k] += Fraction(float(A.val[i]))
        else:
            nbad += 1
    assert skipped == nbad > 0
    for g in range(M):
        for k in range(K):
            # plain left-to-right sum: within a few roundings of the exact value
            assert abs(Fraction(float(X[g, k])) - ref[g][k]) <= Fraction(64 * U) * 8


def test_encode_dense_is_bit_exact_placement(orc):
    M, K = 33, 65
    A, _ = wl.mm_query(M, K, 3, seed=9)
    X, skipped = orc.encode_A(to_rel(orc, A), M, K)
    assert skipped == 0
    ref = np.full((M, K), np.nan)
    ref[A.group.numpy(), A.key.numpy()] = A.val.numpy()
    assert np.array_equal(X, ref)


def test_dictionary_matches_library_unique(orc):
    """dom(ID) of Section 3.1: numpy's unique (sort + dedup) is an
    independent route to the sorted distinct values and the ranks."""
    rng = np.random.default_rng(7)
    a = rng.integers(-50, 50, 300).astype(np.int64)
    b = np.concatenate([rng.integers(-2**63, 2**63 - 1, 200, dtype=np.int64),
                        np.array([np.iinfo(np.int64).min, np.iinfo(np.int64).max, 0, 0],
                                 dtype=np.int64)])
    d, ca, cb = orc.dictionary(a, b)
    ref, inv = np.unique(np.concatenate([a, b]), return_inverse=True)
    assert np.array_equal(d, ref)
    assert np.array_equal(np.concatenate([ca, cb]), inv.astype(np.int32))
    d, ca, cb = orc.dictionary(a[:0], b[:3])
    assert np.array_equal(d, np.unique(b[:3])) and ca.shape == (0,)


def test_join3_matches_nested_loops(orc):
    """Q2 (three-way join) against the triple loop over all tuple triples."""
    rng = np.random.default_rng(41)
    for na, nb, nc, d1, d2 in ((30, 40, 35, 6, 5), (0, 10, 10, 3, 3), (12, 0, 9, 4, 4),
                               (20, 25, 0, 3, 3), (50, 1, 50, 2, 2)):
        a = rng.integers(0, d1, na) * 1000003 - 7
        b1 = rng.integers(0, d1, nb) * 1000003 - 7
        b2 = rng.integers(0, d2, nb) * 999983 + 11
        c = rng.integers(0, d2, nc) * 999983 + 11
        want = sorted((i, j, k) for i in range(na) for j in range(nb) for k in range(nc)
                      if a[i] == b1[j] and b2[j] == c[k])
        got = orc.join3(a, b1, b2, c)
        assert [tuple(r) for r in got.tolist()] == want
