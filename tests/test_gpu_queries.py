"""The Q1/Q3/Q4 family of Sections 3.1 and 3.3 on the GPU against the oracle.

Dictionary encoding (dom(ID), Section 3.1) is integer work: bit-exact.
Q1 (two-way join) is the operator with one group per tuple and COUNT
encodings: exact integer counts, and a pair is in the join iff its count
is positive.  Q3 (SUM ... GROUP BY B.Val over the join) and Q4 (SUM of
products without GROUP BY) run in re-associated form (A's histogram over
keys, then one pass over B) and must match the oracle's SQL sum with all of
A in one group.
"""
import numpy as np
import pytest
import torch

from paper_2112_07552_amd import ops
from paper_2112_07552_amd import workloads as wl

from .gpu_util import abs_rel, cuda_or_skip, err_cw

pytestmark = pytest.mark.gpu

I64MIN, I64MAX = np.iinfo(np.int64).min, np.iinfo(np.int64).max


@pytest.mark.parametrize("na,nb,distinct", [(1000, 1500, 37), (0, 100, 10), (100, 0, 10),
                                            (1 << 20, 1 << 20, 32), (300_000, 200_000, 250_000)])
def test_dictionary_bit_exact(orc, na, nb, distinct):
    dev = cuda_or_skip()
    a = wl.id_column(na, distinct, 60, 1)
    b = wl.id_column(nb, distinct, 60, 2)  # same pool: the domains overlap
    if na > 3:
        a[0], a[1], a[2] = I64MIN, I64MAX, -1
    d, ca, cb = ops.dict_encode(a.to(dev), b.to(dev))
    od, oca, ocb = orc.dictionary(a.numpy(), b.numpy())
    assert np.array_equal(d.cpu().numpy(), od)
    assert np.array_equal(ca.cpu().numpy(), oca)
    assert np.array_equal(cb.cpu().numpy(), ocb)


@pytest.mark.parametrize("n", [4096, 32768])
def test_q1_join_indicator_exact(orc, n):
    """Q1: A(ID), B(ID) with n = m tuples over 32 distinct IDs (the paper's
    microbenchmark shape, Section 5.2).  C = mat(A) mat(B)^T counts the
    joined pairs; tuple pair (i, j) is in the join iff C[i,j] > 0."""
    dev = cuda_or_skip()
    m = n
    ida = wl.id_column(n, 32, 61, 1)
    idb = wl.id_column(m, 32, 61, 2)
    _, ka, kb = ops.dict_encode(ida.to(dev), idb.to(dev))
    K = int(max(ka.max(), kb.max())) + 1
    ga = torch.arange(n, dtype=torch.int32, device=dev)
    hb = torch.arange(m, dtype=torch.int32, device=dev)
    Cm, cnt, ws = ops.join_agg_fwd(ga, ka, None, kb, hb, None, n, K, m, with_count=True,
                                   unique=True)
    assert ops.sync_status(ws)[0] == 0
    rows = np.arange(3, n, n // 128, dtype=np.int32)
    got = cnt[torch.as_tensor(rows, device=dev)].cpu().numpy()
    joined = (ida.numpy()[rows, None] == idb.numpy()[None, :])
    assert np.array_equal(got > 0, joined)
    RA = orc.Rel(ga.cpu().numpy(), ka.cpu().numpy(), None)
    RB = orc.Rel(hb.cpu().numpy(), kb.cpu().numpy(), None)
    _, oc, _ = orc.join_agg(RA, RB, n, K, m, rows=rows, with_count=True)
    assert np.array_equal(got, oc)
    assert torch.equal(Cm, cnt.to(torch.float64))
    # the join size (the number of result tuples of Q1) from the reduction
    assert int(cnt.sum(dtype=torch.int64)) == int(
        sum(np.count_nonzero(idb.numpy() == v) * c
            for v, c in zip(*np.unique(ida.numpy(), return_counts=True))))


def q3_case(orc, n_a, n_b, n_ids, n_groups, seed, weighted=False, bad=0.0):
    """SUM(A.Val), COUNT and AVG grouped by B.Val over A JOIN B ON ID.

    weighted=True multiplies each pair by a B-side weight as well (the
    operator's general form with M = 1)."""
    dev = cuda_or_skip()
    ida = wl.id_column(n_a, n_ids, seed, 1)
    idb = wl.id_column(n_b, n_ids, seed, 2)
    bval = wl.id_column(n_b, n_groups, seed, 7)      # B.Val: the GROUP BY column
    _, ka, kb = ops.dict_encode(ida.to(dev), idb.to(dev))
    groups, gb, _ = ops.dict_encode(bval.to(dev), bval[:0].to(dev))
    N = int(groups.numel())
    K = max(1, int(ka.max()) + 1 if n_a else 1, int(kb.max()) + 1 if n_b else 1)
    av = wl.draw_values("uniform", n_a, seed, 3, device=dev)
    bw = wl.draw_values("uniform", n_b, seed, 4, device=dev) if weighted else None
    if bad:
        kb = kb.clone()
        kb[::int(1 / bad)] = K + 5
    c, cnt, ws = ops.join_agg_row(ka, av, kb, gb, bw, K, N, with_count=True)
    st, info = ops.sync_status(ws)
    RA = orc.Rel(np.zeros(n_a, dtype=np.int32), ka.cpu().numpy(), av.cpu().numpy())
    RB = orc.Rel(gb.cpu().numpy(), kb.cpu().numpy(), None if bw is None else bw.cpu().numpy())
    Co, co, _ = orc.join_agg(RA, RB, 1, K, N, with_count=True)
    So, _, _ = orc.join_agg(abs_rel(orc, RA), abs_rel(orc, RB), 1, K, N)
    c, cnt = c.cpu().numpy(), cnt.cpu().numpy()
    assert np.array_equal(cnt, co[0])
    assert err_cw(c, Co[0], So[0]) <= 1e-12
    # AVG = SUM / COUNT (Section 3.3), for the groups with joined pairs
    has = co[0] > 0
    avg = c[has] / cnt[has]
    assert np.all(np.abs(avg - Co[0][has] / co[0][has]) <= 2e-12 * So[0][has] / co[0][has])
    return st, info


@pytest.mark.parametrize("n_a,n_b,n_ids,n_groups", [
    (32768, 32768, 32, 32),            # microbenchmark: 32 distinct join values
    (4096, 4096, 4096, 64),            # microbenchmark: 4096 records, many distinct values
    (20_000, 30_000, 1024, 5000),      # group array beyond the LDS-privatised size
    (100_000, 50_000, 10_000, 1500),   # key histogram in global memory
    (1 << 22, 1 << 22, 1 << 20, 3000), # millions of records, sparse join
    (0, 1000, 16, 8),                  # empty A: every group sums to 0
])
def test_q3_group_sum_and_avg(orc, n_a, n_b, n_ids, n_groups):
    st, _ = q3_case(orc, n_a, n_b, n_ids, n_groups, seed=62)
    assert st == 0


def test_q3_weighted(orc):
    st, _ = q3_case(orc, 30_000, 40_000, 500, 3000, seed=65, weighted=True)
    assert st == 0


def test_q3_out_of_range_keys_reported(orc):
    st, info = q3_case(orc, 50_000, 60_000, 64, 40, seed=63, bad=0.01)
    assert st == ops._lib.TCU_ERR_KEY_RANGE and info["skipped_b"] > 0


@pytest.mark.parametrize("n,n_ids", [(32768, 32), (1 << 22, 1 << 21)])
def test_q4_total(orc, n, n_ids):
    """Q4: SUM(A.Val * B.Val) over the join: N = 1, every B record in group 0."""
    dev = cuda_or_skip()
    ida, idb = wl.id_column(n, n_ids, 64, 1), wl.id_column(n, n_ids, 64, 2)
    _, ka, kb = ops.dict_encode(ida.to(dev), idb.to(dev))
    K = int(max(ka.max(), kb.max())) + 1
    av = wl.draw_values("uniform", n, 64, 3, device=dev)
    bw = wl.draw_values("uniform", n, 64, 4, device=dev)
    g0 = torch.zeros(n, dtype=torch.int32, device=dev)
    c, cnt, ws = ops.join_agg_row(ka, av, kb, g0, bw, K, 1, with_count=True)
    assert ops.sync_status(ws)[0] == 0
    RA = orc.Rel(np.zeros(n, np.int32), ka.cpu().numpy(), av.cpu().numpy())
    RB = orc.Rel(np.zeros(n, np.int32), kb.cpu().numpy(), bw.cpu().numpy())
    Co, co, _ = orc.join_agg(RA, RB, 1, K, 1, with_count=True)
    So, _, _ = orc.join_agg(abs_rel(orc, RA), abs_rel(orc, RB), 1, K, 1)
    assert int(cnt.cpu()[0]) == int(co[0, 0])
    assert abs(float(c.cpu()[0]) - Co[0, 0]) <= 1e-12 * So[0, 0]


@pytest.mark.parametrize("n_ids", [32, 4096])
def test_q3_q4_literal_matrix_form(orc, n_ids):
    """Lemma Q3 as written: 1^T x (mat(A) mat(B)^T), one row of mat(A) per
    A tuple, with the ones-vector reduction as a second product on the FP64
    matrix cores; Q4 adds the reduction on the right.  4096 records per
    table (the microbenchmark size), 32 or 4096 distinct join values."""
    dev = cuda_or_skip()
    n = 4096
    ida, idb = wl.id_column(n, n_ids, 66, 1), wl.id_column(n, n_ids, 66, 2)
    bval = wl.id_column(n, 64, 66, 7)
    _, ka, kb = ops.dict_encode(ida.to(dev), idb.to(dev))
    _, gb, _ = ops.dict_encode(bval.to(dev), bval[:0].to(dev))
    K = int(max(ka.max(), kb.max())) + 1
    N = int(gb.max()) + 1
    av = wl.draw_values("uniform", n, 66, 3, device=dev)
    bw = wl.draw_values("uniform", n, 66, 4, device=dev)
    tuples = torch.arange(n, dtype=torch.int32, device=dev)
    ones = torch.ones((1, n), dtype=torch.float64, device=dev)
    # Q3: rows = A tuples, columns = B.Val groups, B side 0/1 (COUNT encoding)
    Cfull, _, ws = ops.join_agg_fwd(tuples, ka, av, kb, gb, None, n, K, N)
    assert ops.sync_status(ws)[0] == 0
    q3 = ops.gemm_f64(ones, Cfull).cpu().numpy()[0]
    RA = orc.Rel(np.zeros(n, np.int32), ka.cpu().numpy(), av.cpu().numpy())
    RB = orc.Rel(gb.cpu().numpy(), kb.cpu().numpy(), None)
    Co, _, _ = orc.join_agg(RA, RB, 1, K, N)
    So, _, _ = orc.join_agg(abs_rel(orc, RA), abs_rel(orc, RB), 1, K, N)
    assert err_cw(q3, Co[0], So[0]) <= 1e-12
    # Q4: rows = A tuples, columns = B tuples, then 1^T C 1
    Ct, _, ws = ops.join_agg_fwd(tuples, ka, av, kb, tuples, bw, n, K, n, unique=True)
    assert ops.sync_status(ws)[0] == 0
    col = ops.gemm_f64(Ct, torch.ones((n, 1), dtype=torch.float64, device=dev))
    q4 = float(ops.gemm_f64(ones, col).cpu()[0, 0])
    RB4 = orc.Rel(np.zeros(n, np.int32), kb.cpu().numpy(), bw.cpu().numpy())
    C4, _, _ = orc.join_agg(RA, RB4, 1, K, 1)
    S4, _, _ = orc.join_agg(abs_rel(orc, RA), abs_rel(orc, RB4), 1, K, 1)
    assert abs(q4 - C4[0, 0]) <= 1e-12 * S4[0, 0]
