"""The block-sparse form (16 x 16 tiles, empty tiles skipped; Section 4.2.4)
against the oracle and against the dense form.

The oracle evaluates the SQL sum over joined record pairs; the tile
structure is invisible to it.  Bars as for the dense form: err_cw <= 1e-12
against (|X||Y|), cells without a joined pair exactly 0, integer (COUNT)
results exact."""
import numpy as np
import pytest
import torch

from paper_2112_07552_amd import ops
from paper_2112_07552_amd import workloads as wl

from .gpu_util import TOL, abs_rel, cuda_or_skip, err_cw, to_orc

pytestmark = pytest.mark.gpu


def check_rows(orc, A, B, M, K, N, Cg, rows=None):
    RA, RB = to_orc(orc, A), to_orc(orc, B)
    Co, _, _ = orc.join_agg(RA, RB, M, K, N, rows=rows)
    So, _, _ = orc.join_agg(abs_rel(orc, RA), abs_rel(orc, RB), M, K, N, rows=rows)
    got = Cg if rows is None else Cg[rows]
    return err_cw(got, Co, So)


@pytest.mark.parametrize("M,K,N,na,nb,seed", [
    (300, 5000, 200, 4000, 5000, 1),     # ragged tile edges, duplicates
    (16, 16, 16, 300, 300, 2),           # one tile each
    (1, 100_000, 1, 500, 700, 3),        # single group, huge sparse key domain
    (1000, 1_000_000, 1000, 20_000, 20_000, 4),
])
def test_bsr_random_relations(orc, M, K, N, na, nb, seed):
    dev = cuda_or_skip()
    A = wl.random_relation(na, M, K, seed, 1, device=dev)
    B = wl.random_relation(nb, N, K, seed, 2, device=dev)
    Cg, ws = ops.join_agg_bsr(A.group, A.key, A.val, B.key, B.group, B.val, M, K, N)
    assert ops.sync_status(ws)[0] == 0
    Cg = Cg.cpu().numpy()
    assert check_rows(orc, wl.Relation(*[t.cpu() for t in A]), wl.Relation(*[t.cpu() for t in B]),
                      M, K, N, Cg) <= TOL


def test_bsr_matches_dense_form_exactly_on_integers(orc):
    """Integer values: every partial sum is exact, so the block-sparse and
    dense forms agree bit for bit."""
    dev = cuda_or_skip()
    M, K, N = 200, 3000, 150
    A = wl.random_relation(6000, M, K, 5, 1, values="int", lo=-100, hi=100, device=dev)
    B = wl.random_relation(6000, N, K, 5, 2, values="int", lo=-100, hi=100, device=dev)
    Cb, ws = ops.join_agg_bsr(A.group, A.key, A.val, B.key, B.group, B.val, M, K, N)
    assert ops.sync_status(ws)[0] == 0
    Cd, _, ws2 = ops.join_agg_fwd(A.group, A.key, A.val, B.key, B.group, B.val, M, K, N)
    assert ops.sync_status(ws2)[0] == 0
    assert torch.equal(Cb, Cd)


def test_bsr_out_of_range_and_unique(orc):
    dev = cuda_or_skip()
    M, K, N = 64, 4096, 48
    A = wl.random_relation(3000, M, K, 6, 1, device=dev, bad_fraction=0.05)
    B = wl.random_relation(3000, N, K, 6, 2, device=dev, bad_fraction=0.05)
    Cg, ws = ops.join_agg_bsr(A.group, A.key, A.val, B.key, B.group, B.val, M, K, N)
    st, info = ops.sync_status(ws)
    assert st == ops._lib.TCU_ERR_KEY_RANGE and info["skipped_a"] > 0 and info["skipped_b"] > 0
    Ac, Bc = wl.Relation(*[t.cpu() for t in A]), wl.Relation(*[t.cpu() for t in B])
    assert check_rows(orc, Ac, Bc, M, K, N, Cg.cpu().numpy()) <= TOL
    # unique cells: a dense table's records in random order
    Xd, Yd = wl.mm_query(40, 37, 29, seed=7, device=dev)
    Cu, ws = ops.join_agg_bsr(Xd.group, Xd.key, Xd.val, Yd.key, Yd.group, Yd.val, 40, 37, 29,
                              unique=True)
    assert ops.sync_status(ws)[0] == 0
    Xc, Yc = wl.Relation(*[t.cpu() for t in Xd]), wl.Relation(*[t.cpu() for t in Yd])
    assert check_rows(orc, Xc, Yc, 40, 37, 29, Cu.cpu().numpy()) <= TOL


def test_bsr_empty_relation_gives_zero():
    dev = cuda_or_skip()
    A = wl.random_relation(0, 33, 70, 8, 1, device=dev)
    B = wl.random_relation(500, 21, 70, 8, 2, device=dev)
    Cg, ws = ops.join_agg_bsr(A.group, A.key, A.val, B.key, B.group, B.val, 33, 70, 21)
    assert ops.sync_status(ws)[0] == 0
    assert torch.all(Cg == 0)


@pytest.mark.parametrize("n,k", [(4096, 4096), (16384, 1 << 20)])
def test_bsr_q1_counts_many_distinct_values(orc, n, k):
    """Q1 in the many-distinct-values regime (Section 5.2): one record per
    tuple, k distinct IDs.  C is the exact pair-count matrix."""
    dev = cuda_or_skip()
    ida, idb = wl.id_column(n, k, 67, 1, device=dev), wl.id_column(n, k, 67, 2, device=dev)
    _, ka, kb = ops.dict_encode(ida, idb)
    K = int(max(ka.max(), kb.max())) + 1
    t = torch.arange(n, dtype=torch.int32, device=dev)
    Cb, ws = ops.join_agg_bsr(t, ka, None, kb, t, None, n, K, n, unique=True)
    assert ops.sync_status(ws)[0] == 0
    rows = np.arange(5, n, n // 64, dtype=np.int32)
    got = Cb[torch.as_tensor(rows, device=dev)].cpu().numpy()
    RA = orc.Rel(t.cpu().numpy(), ka.cpu().numpy(), None)
    RB = orc.Rel(t.cpu().numpy(), kb.cpu().numpy(), None)
    _, oc, _ = orc.join_agg(RA, RB, n, K, n, rows=rows, with_count=True)
    assert np.array_equal(got, oc.astype(np.float64))
    # the total: the join size
    ia, ib = ida.cpu().numpy(), idb.cpu().numpy()
    va, ca = np.unique(ia, return_counts=True)
    vb, cb = np.unique(ib, return_counts=True)
    common, xa, xb = np.intersect1d(va, vb, return_indices=True)
    assert float(Cb.sum()) == float(np.sum(ca[xa] * cb[xb]))


def test_bsr_local_graph(orc):
    """A graph with locality (road-network-like, about 2 edges per node):
    adjacency times a weighted node-feature relation, 8192 nodes."""
    dev = cuda_or_skip()
    nodes = 8192
    E = wl.local_edges(2 * nodes, nodes, 40, 9, 1, device=dev)      # group = src, key = dst
    F = wl.random_relation(4 * nodes, 64, nodes, 9, 2, device=dev)   # group = feature, key = node
    Cg, ws = ops.join_agg_bsr(E.group, E.key, E.val, F.key, F.group, F.val, nodes, nodes, 64)
    assert ops.sync_status(ws)[0] == 0
    Ec, Fc = wl.Relation(*[t.cpu() for t in E]), wl.Relation(*[t.cpu() for t in F])
    assert check_rows(orc, Ec, Fc, nodes, nodes, 64, Cg.cpu().numpy()) <= TOL


@pytest.mark.parametrize("n,k,form", [(4096, 64, "dense"), (4096, 4096, "block_sparse")])
def test_auto_choice_matches_both_forms(orc, n, k, form):
    """join_agg_auto takes the form the cost model picks (dense for few
    distinct keys, block-sparse for many) and returns the Q1 pair counts
    exactly: equal to the other form's, and to the oracle on sampled rows."""
    dev = cuda_or_skip()
    ida = wl.id_column(n, k, 73, 1, device=dev)
    idb = wl.id_column(n, k, 73, 2, device=dev)
    _, ka, kb = ops.dict_encode(ida, idb)
    K = int(max(ka.max(), kb.max())) + 1
    t = torch.arange(n, dtype=torch.int32, device=dev)
    args = (t, ka, None, kb, t, None, n, K, n)
    Cg, picked = ops.join_agg_auto(*args, unique=True)
    assert picked == form
    Cd, _, _ = ops.join_agg_fwd(*args, unique=True)
    Cb, _ = ops.join_agg_bsr(*args, unique=True)
    assert torch.equal(Cg, Cd) and torch.equal(Cg, Cb)
    rows = np.arange(0, n, 97, dtype=np.int32)
    RA = orc.Rel(t.cpu().numpy(), ka.cpu().numpy(), None)
    RB = orc.Rel(t.cpu().numpy(), kb.cpu().numpy(), None)
    Co, _, _ = orc.join_agg(RA, RB, n, K, n, rows=rows)
    assert np.array_equal(Cg.cpu().numpy()[rows], Co)
