"""GPU parity of the hand-written adjoint (step a4) and its autograd wrapper.

For L = sum(W * C) the value gradients are
  dL/da_i.v = (W Y^T)[g_i, k_i],   dL/db_j.w = (X^T W)[k_j, h_j],
compared with the oracle's closed form (record by record), with central
finite differences of the GPU forward, and with torch.autograd.gradcheck.
"""
import numpy as np
import pytest
import torch

from paper_2112_07552_amd import ops
from paper_2112_07552_amd import workloads as wl

from .gpu_util import TOL, abs_rel, cuda_or_skip, err_cw, to_orc

pytestmark = pytest.mark.gpu


def grad_errors(orc, A, B, W, M, K, N, dA, dB, idxA=None, idxB=None):
    RA, RB = to_orc(orc, A), to_orc(orc, B)
    Wn = W.cpu().numpy()
    ga = orc.grad(RA, RB, M, K, N, Wn, "A", idx=idxA)
    gb = orc.grad(RA, RB, M, K, N, Wn, "B", idx=idxB)
    sa = orc.grad(abs_rel(orc, RA), abs_rel(orc, RB), M, K, N, np.abs(Wn), "A", idx=idxA)
    sb = orc.grad(abs_rel(orc, RA), abs_rel(orc, RB), M, K, N, np.abs(Wn), "B", idx=idxB)
    dA = dA.cpu().numpy() if idxA is None else dA.cpu().numpy()[idxA]
    dB = dB.cpu().numpy() if idxB is None else dB.cpu().numpy()[idxB]
    return err_cw(dA, ga, sa), err_cw(dB, gb, sb)


@pytest.mark.parametrize("seed,nA,nB,M,K,N,bad", [
    (30, 30_000, 40_000, 200, 131, 170, 0.0),
    (31, 20_000, 20_000, 129, 1, 257, 0.0),
    (32, 40_000, 30_000, 150, 190, 140, 0.03),
])
def test_bwd_random_relations_full_oracle(orc, seed, nA, nB, M, K, N, bad):
    dev = cuda_or_skip()
    A = wl.random_relation(nA, M, K, seed, 1, device=dev, bad_fraction=bad)
    B = wl.random_relation(nB, N, K, seed, 2, device=dev, bad_fraction=bad)
    W = wl.draw_values("uniform", M * N, seed, 99, device=dev).reshape(M, N)
    dA, dB, ws = ops.join_agg_bwd(A.group, A.key, A.val, B.key, B.group, B.val, M, K, N, W)
    st, info = ops.sync_status(ws)
    ea, eb = grad_errors(orc, A, B, W, M, K, N, dA, dB)
    assert ea <= TOL and eb <= TOL, (ea, eb)
    if bad:
        assert st == ops._lib.TCU_ERR_KEY_RANGE
        badA = ((A.group < 0) | (A.group >= M) | (A.key < 0) | (A.key >= K)).cpu().numpy()
        assert np.all(dA.cpu().numpy()[badA] == 0.0)


def test_bwd_one_side_only(orc):
    """Asking for one gradient gives the same bits as asking for both
    (dense tables: unique cells, so the encodings are deterministic)."""
    dev = cuda_or_skip()
    M, K, N = 100, 80, 90
    A, B = wl.mm_query(M, K, N, seed=33, device=dev)
    W = wl.draw_values("uniform", M * N, 33, 99, device=dev).reshape(M, N)
    dA, dB, _ = ops.join_agg_bwd(A.group, A.key, A.val, B.key, B.group, B.val, M, K, N, W,
                                 need_a=True, need_b=False)
    assert dB is None
    dA2, dB2, _ = ops.join_agg_bwd(A.group, A.key, A.val, B.key, B.group, B.val, M, K, N, W,
                                   need_a=False, need_b=True)
    assert dA2 is None
    dA3, dB3, _ = ops.join_agg_bwd(A.group, A.key, A.val, B.key, B.group, B.val, M, K, N, W)
    assert torch.equal(dA, dA3) and torch.equal(dB2, dB3)


@pytest.mark.parametrize("unique", [False, True])
def test_bwd_saved_encodings_match_checkpointing(unique):
    """Reusing the forward's X and Y gives the same bits as re-encoding."""
    dev = cuda_or_skip()
    M, K, N = 300, 257, 200
    A, B = wl.mm_query(M, K, N, seed=34, device=dev)
    W = wl.draw_values("uniform", M * N, 34, 99, device=dev).reshape(M, N)
    _, _, ws = ops.join_agg_fwd(A.group, A.key, A.val, B.key, B.group, B.val, M, K, N,
                                unique=unique, for_backward=True)
    dA1, dB1, _ = ops.join_agg_bwd(A.group, A.key, A.val, B.key, B.group, B.val, M, K, N, W,
                                   ws=ws, unique=unique, saved_encodings=True)
    dA2, dB2, _ = ops.join_agg_bwd(A.group, A.key, A.val, B.key, B.group, B.val, M, K, N, W,
                                   unique=unique)
    assert torch.equal(dA1, dA2) and torch.equal(dB1, dB2)


@pytest.mark.parametrize("saved", [False, True])
def test_bwd_stream_ordered_on_a_side_stream(saved):
    """With both gradients the adjoint runs its dA gather (and, when
    re-encoding, the encoding of X) on an internal stream and joins it back
    to the caller's stream: work queued afterwards on the caller's stream
    sees finished gradients, with no device-wide synchronisation between.
    The gathers move values exactly, so the result matches a run on the
    default stream bit for bit."""
    dev = cuda_or_skip()
    M, K, N = 640, 512, 768
    A, B = wl.mm_query(M, K, N, seed=36, device=dev)
    W = wl.draw_values("uniform", M * N, 36, 99, device=dev).reshape(M, N)
    ref_a, ref_b, _ = ops.join_agg_bwd(A.group, A.key, A.val, B.key, B.group, B.val, M, K, N, W,
                                       unique=True)
    torch.cuda.synchronize(dev)
    s = torch.cuda.Stream(device=dev)
    s.wait_stream(torch.cuda.current_stream(dev))
    with torch.cuda.stream(s):
        ws = None
        if saved:
            _, _, ws = ops.join_agg_fwd(A.group, A.key, A.val, B.key, B.group, B.val, M, K, N,
                                        unique=True, for_backward=True)
        dA, dB, _ = ops.join_agg_bwd(A.group, A.key, A.val, B.key, B.group, B.val, M, K, N, W,
                                     ws=ws, unique=True, saved_encodings=saved)
        # consumers on the same stream, right behind the call
        cA, cB = dA.clone(), dB.clone()
    s.synchronize()
    assert torch.equal(cA, ref_a) and torch.equal(cB, ref_b)


def test_bwd_cut_dy_product_matches_uncut(orc):
    """dY = X^T W large enough for more than one round of GEMM workgroups
    (K x N = 2200 x 4000 is 18 x 32 tiles of 128 x 128): with both gradients
    the FP64 product is cut into two row blocks whose dB gathers run on two
    streams.  Each entry of dY is the same dot product either way, so dB
    equals the one-gradient call (one launch, one gather) bit for bit;
    records outside the matrices get 0; sampled records match the oracle."""
    dev = cuda_or_skip()
    M, K, N = 64, 2200, 4000
    A = wl.random_relation(100_000, M, K, 37, 1, device=dev, bad_fraction=0.01)
    B = wl.random_relation(2_000_000, N, K, 37, 2, device=dev, bad_fraction=0.01)
    W = wl.draw_values("uniform", M * N, 37, 99, device=dev).reshape(M, N)
    _, _, ws = ops.join_agg_fwd(A.group, A.key, A.val, B.key, B.group, B.val, M, K, N,
                                for_backward=True)
    args = (A.group, A.key, A.val, B.key, B.group, B.val, M, K, N, W)
    dA, dB, _ = ops.join_agg_bwd(*args, ws=ws, saved_encodings=True)
    _, dB1, _ = ops.join_agg_bwd(*args, ws=ws, saved_encodings=True, need_a=False)
    dA1, _, _ = ops.join_agg_bwd(*args, ws=ws, saved_encodings=True, need_b=False)
    torch.cuda.synchronize(dev)
    assert torch.equal(dB, dB1) and torch.equal(dA, dA1)
    badB = ((B.group < 0) | (B.group >= N) | (B.key < 0) | (B.key >= K)).cpu().numpy()
    assert badB.any() and np.all(dB.cpu().numpy()[badB] == 0.0)
    rng = np.random.default_rng(37)
    ia = rng.choice(A.n, 2000, replace=False).astype(np.int64)
    ib = rng.choice(B.n, 4000, replace=False).astype(np.int64)
    ea, eb = grad_errors(orc, A, B, W, M, K, N, dA, dB, ia, ib)
    assert ea <= TOL and eb <= TOL, (ea, eb)


def test_bwd_cut_dy_product_checkpointed_matches_uncut(orc):
    """The cut dY product with the encodings rebuilt inside the call (X on
    the internal stream, waited for before dY): dense tables with unique
    cells encode deterministically, so both gradients match the
    one-gradient calls bit for bit."""
    dev = cuda_or_skip()
    M, K, N = 96, 2200, 4000
    A, B = wl.mm_query(M, K, N, seed=38, device=dev)
    W = wl.draw_values("uniform", M * N, 38, 99, device=dev).reshape(M, N)
    args = (A.group, A.key, A.val, B.key, B.group, B.val, M, K, N, W)
    dA, dB, ws = ops.join_agg_bwd(*args, unique=True)
    assert ops.sync_status(ws)[0] == 0
    _, dB1, _ = ops.join_agg_bwd(*args, unique=True, need_a=False)
    dA1, _, _ = ops.join_agg_bwd(*args, unique=True, need_b=False)
    torch.cuda.synchronize(dev)
    assert torch.equal(dB, dB1) and torch.equal(dA, dA1)
    rng = np.random.default_rng(38)
    ia = rng.choice(A.n, 2000, replace=False).astype(np.int64)
    ib = rng.choice(B.n, 4000, replace=False).astype(np.int64)
    ea, eb = grad_errors(orc, A, B, W, M, K, N, dA, dB, ia, ib)
    assert ea <= TOL and eb <= TOL, (ea, eb)


@pytest.mark.parametrize("checkpoint", [True, False])
def test_autograd_checkpoint_modes_agree(checkpoint):
    dev = cuda_or_skip()
    M, K, N = 130, 100, 120
    A, B = wl.mm_query(M, K, N, seed=35, device=dev)
    W = wl.draw_values("uniform", M * N, 35, 99, device=dev).reshape(M, N)
    av = A.val.clone().requires_grad_(True)
    bv = B.val.clone().requires_grad_(True)
    Cm = ops.join_agg(A.group, A.key, av, B.key, B.group, bv, M, K, N, unique=True,
                      checkpoint=checkpoint)
    (Cm * W).sum().backward()
    dA, dB, _ = ops.join_agg_bwd(A.group, A.key, A.val, B.key, B.group, B.val, M, K, N, W)
    assert torch.equal(av.grad, dA) and torch.equal(bv.grad, dB)


def test_fwd_bwd_2pow24_records(orc):
    """2^24 records per table (N = 4096), seed 2, W = U[-1,1) (seed 1002):
    512 whole rows of C, 4096 sampled cells and Freivalds' check; oracle
    gradient on 4096 + 4096 sampled records; central differences (h = 1e-6)
    on 32 + 32 records."""
    from .test_gpu_parity import sampled_checks
    dev = cuda_or_skip()
    N = 4096
    A, B = wl.mm_query(N, N, N, seed=2, device=dev)
    # the launch configuration the benchmark times: unique cells, saved encodings
    Cg, _, ws = ops.join_agg_fwd(A.group, A.key, A.val, B.key, B.group, B.val, N, N, N,
                                 unique=True, for_backward=True)
    assert ops.sync_status(ws)[0] == 0
    assert sampled_checks(orc, A, B, Cg, N, N, N, seed=2, ncells=4096, nrows=512) <= TOL
    W = wl.draw_values("uniform", N * N, 1002, 0, device=dev).reshape(N, N)
    dA, dB, ws = ops.join_agg_bwd(A.group, A.key, A.val, B.key, B.group, B.val, N, N, N, W,
                                  ws=ws, unique=True, saved_encodings=True)
    assert ops.sync_status(ws)[0] == 0
    rng = np.random.default_rng(1002)
    ia = rng.choice(A.n, 4096, replace=False).astype(np.int64)
    ib = rng.choice(B.n, 4096, replace=False).astype(np.int64)
    ea, eb = grad_errors(orc, A, B, W, N, N, N, dA, dB, ia, ib)
    assert ea <= TOL and eb <= TOL, (ea, eb)

    # central differences of L = sum(W * C); C changes only in one row (A
    # record) or one column (B record), so dL is summed over that line only
    h = 1e-6
    worst = 0.0
    for which, idx in (("A", ia[:32]), ("B", ib[:32])):
        R = A if which == "A" else B
        grad = dA if which == "A" else dB
        for i in idx.tolist():
            vals = []
            for sgn in (1.0, -1.0):
                v = R.val.clone()
                v[i] += sgn * h
                if which == "A":
                    Cp, _, _ = ops.join_agg_fwd(A.group, A.key, v, B.key, B.group, B.val, N, N, N)
                    g = int(A.group[i])
                    vals.append((Cp[g], W[g]))
                else:
                    Cp, _, _ = ops.join_agg_fwd(A.group, A.key, A.val, B.key, B.group, v, N, N, N)
                    hh = int(B.group[i])
                    vals.append((Cp[:, hh], W[:, hh]))
            (cp, w), (cm, _) = vals
            # the two perturbed values differ from v by +-h after rounding
            vp = float(R.val[i]) + h
            vm = float(R.val[i]) - h
            fd = float(torch.sum(w * (cp - cm))) / (vp - vm)
            g_ = float(grad[i])
            worst = max(worst, abs(fd - g_) / max(1.0, abs(g_)))
    assert worst <= 1e-5, worst


def test_autograd_gradcheck():
    dev = cuda_or_skip()
    M, K, N = 5, 4, 6
    A = wl.random_relation(30, M, K, 40, 1, device=dev)
    B = wl.random_relation(25, N, K, 40, 2, device=dev)
    av = A.val.clone().requires_grad_(True)
    bv = B.val.clone().requires_grad_(True)
    f = lambda a, b: ops.join_agg(A.group, A.key, a, B.key, B.group, b, M, K, N)
    assert torch.autograd.gradcheck(f, (av, bv), eps=1e-6, atol=1e-8, rtol=1e-6)


def test_autograd_matches_direct_adjoint():
    """Autograd through JoinAgg gives the direct adjoint's bits (dense tables:
    unique cells, deterministic encodings); FP32 value columns get FP32 grads."""
    dev = cuda_or_skip()
    M, K, N = 140, 70, 130
    A = wl.dense_relation(K, M, 41, 1, device=dev)
    B = wl.dense_relation(N, K, 41, 2, device=dev, dtype=torch.float32, row_is_group=True)
    W = wl.draw_values("uniform", M * N, 41, 99, device=dev).reshape(M, N)
    av = A.val.clone().requires_grad_(True)
    bv = B.val.clone().requires_grad_(True)
    Cm = ops.join_agg(A.group, A.key, av, B.key, B.group, bv, M, K, N)
    (Cm * W).sum().backward()
    dA, dB, _ = ops.join_agg_bwd(A.group, A.key, A.val, B.key, B.group, B.val, M, K, N, W)
    assert torch.equal(av.grad, dA)
    assert bv.grad.dtype == torch.float32 and torch.equal(bv.grad, dB.to(torch.float32))
