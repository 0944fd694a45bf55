"""The largest workload on one GPU: 2^30 records per table (N = 32768, the
paper's largest matrix multiplication query, Section 5.4.1), FP32 values from
N(0,1) with 5% of the values multiplied by 1e3 (seed 4).  Both mixed int8
forms (digit slices and residues) run forward plus adjoint with activation
checkpointing (the adjoint rebuilds X and Y from the records); the FP64 form
is the comparator.

The oracle checks, all from the records:
  * a 64 x 64 block of C (relations filtered to the block's groups, which is
    selection, not arithmetic of the operator) against both forms;
  * Freivalds' check C r = X (Y r) for two random +-1 vectors;
  * the value gradient of records in a 64 x 64 block of keys.
"""
import numpy as np
import pytest
import torch

from paper_2112_07552_amd import ops
from paper_2112_07552_amd import workloads as wl

from .gpu_util import cuda_or_skip

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

N = 32768
TOL = 1e-12


def log(msg):
    print(f"[large] {msg}", flush=True)


def remap(values, chosen, size):
    lut = np.full(size, -1, dtype=np.int64)
    lut[chosen] = np.arange(len(chosen))
    return lut[values]


def test_mixed_forms_2pow30_records_forward_adjoint_checkpointed(orc):
    dev = cuda_or_skip()
    free, total = torch.cuda.mem_get_info(dev)
    if free < 160 * 2**30:
        pytest.skip(f"needs about 160 GiB of free device memory, {free / 2**30:.0f} GiB free")
    log("generating 2 x 2^30 records")
    A, B = wl.mm_query(N, N, N, seed=4, values="mixture", dtype=torch.float32, device=dev)
    W = wl.draw_values("uniform", N * N, 1004, 0, device=dev).reshape(N, N)
    torch.cuda.synchronize()

    log("fp64 forward")
    C64, _, ws = ops.join_agg_fwd(A.group, A.key, A.val, B.key, B.group, B.val, N, N, N,
                                  unique=True)
    assert ops.sync_status(ws)[0] == 0
    del ws
    torch.cuda.empty_cache()

    log("copying to the host")
    ag, ak = A.group.cpu().numpy(), A.key.cpu().numpy()
    av = A.val.cpu().numpy().astype(np.float64)
    bk, bh = B.key.cpu().numpy(), B.group.cpu().numpy()
    bw = B.val.cpu().numpy().astype(np.float64)
    RA, RB = orc.Rel(ag, ak, av), orc.Rel(bh, bk, bw)
    rng = np.random.default_rng(4)
    rows = np.sort(rng.choice(N, 64, replace=False)).astype(np.int64)
    cols = np.sort(rng.choice(N, 64, replace=False)).astype(np.int64)
    keys = np.sort(rng.choice(N, 64, replace=False)).astype(np.int64)
    trows, tcols = torch.as_tensor(rows, device=dev), torch.as_tensor(cols, device=dev)

    # -- oracle: C on a 64 x 64 block -----------------------------------------
    log("oracle block of C")
    ga = remap(ag, rows, N)
    ma = ga >= 0
    hb = remap(bh, cols, N)
    mb = hb >= 0
    Af = orc.Rel(ga[ma].astype(np.int32), ak[ma], av[ma])
    Bf = orc.Rel(hb[mb].astype(np.int32), bk[mb], bw[mb])
    Co, _, _ = orc.join_agg(Af, Bf, 64, N, 64)
    So, _, _ = orc.join_agg(orc.Rel(Af.group, Af.key, np.abs(Af.val)),
                            orc.Rel(Bf.group, Bf.key, np.abs(Bf.val)), 64, N, 64)

    # -- oracle: Freivalds right-hand sides ---------------------------------
    log("oracle Freivalds")
    scale = orc.freivalds(orc.Rel(ag, ak, np.abs(av)), orc.Rel(bh, bk, np.abs(bw)), N, N, N,
                          np.ones(N))
    probes = []
    for trial in range(2):
        r = np.where(rng.random(N) < 0.5, -1.0, 1.0)
        probes.append((r, orc.freivalds(RA, RB, N, N, N, r)))

    def freivalds_err(Cm):
        worst = 0.0
        for r, rhs in probes:
            rt = torch.as_tensor(r, device=dev)
            # C r with r = +-1: exact products, pairwise summation on the host
            lhs = np.empty(N)
            for r0 in range(0, N, 2048):
                chunk = (Cm[r0:r0 + 2048] * rt).cpu().numpy()
                lhs[r0:r0 + 2048] = chunk.sum(axis=1)
            worst = max(worst, float(np.max(np.abs(lhs - rhs) / scale)))
        return worst

    blk_64 = C64[trows][:, tcols].cpu().numpy()
    err64 = float(np.max(np.abs(blk_64 - Co) / So))
    fe64 = freivalds_err(C64)
    log(f"fp64: block err_cw {err64:.2e}, Freivalds {fe64:.2e}")
    assert err64 <= 1e-12 and fe64 <= 1e-12
    del C64
    torch.cuda.empty_cache()

    # -- oracle: gradients on a block of keys --------------------------------
    log("oracle gradients")
    Wn_rows = W[trows].cpu().numpy()          # 64 x N
    Wn_cols = W[:, tcols].cpu().numpy()       # N x 64
    kk_a = remap(ak, keys, N)
    kk_b = remap(bk, keys, N)
    # dA for A records with group in rows and key in keys
    ia = np.nonzero(ma & (kk_a >= 0))[0]
    mbk = kk_b >= 0
    A_sub = orc.Rel(ga[ia].astype(np.int32), kk_a[ia].astype(np.int32), av[ia])
    B_key = orc.Rel(bh[mbk], kk_b[mbk].astype(np.int32), bw[mbk])
    gA = orc.grad(A_sub, B_key, 64, 64, N, Wn_rows, "A")
    sA = orc.grad(orc.Rel(A_sub.group, A_sub.key, np.abs(A_sub.val)),
                  orc.Rel(B_key.group, B_key.key, np.abs(B_key.val)), 64, 64, N,
                  np.abs(Wn_rows), "A")
    # dB for B records with key in keys and group in cols
    ib = np.nonzero(mb & mbk)[0]
    mak = kk_a >= 0
    A_key = orc.Rel(ag[mak], kk_a[mak].astype(np.int32), av[mak])
    B_sub = orc.Rel(hb[ib].astype(np.int32), kk_b[ib].astype(np.int32), bw[ib])
    gB = orc.grad(A_key, B_sub, N, 64, 64, Wn_cols, "B")
    sB = orc.grad(orc.Rel(A_key.group, A_key.key, np.abs(A_key.val)),
                  orc.Rel(B_sub.group, B_sub.key, np.abs(B_sub.val)), N, 64, 64,
                  np.abs(Wn_cols), "B")
    tia, tib = torch.as_tensor(ia, device=dev), torch.as_tensor(ib, device=dev)

    # -- each mixed form -------------------------------------------------------
    for precision in ("crt_i8", "split_i8"):
        log(f"{precision} forward")
        Cs, _, ws = ops.join_agg_fwd(A.group, A.key, A.val, B.key, B.group, B.val, N, N, N,
                                     precision=precision, tol=TOL, unique=True)
        st, info = ops.sync_status(ws)
        log(f"{precision} plan: {info}")
        assert st == 0
        if precision == "crt_i8":
            # the residue form certifies this workload; the digit forms' bound
            # carries a term (S - 1) K 2^-7S per cell that 8 digits cannot
            # bring under 1e-12 (|X||Y|) at K = 32768, so they may run in FP64
            assert info["flags"] & ops._lib.TCU_FLAG_FALLBACK == 0
        del ws
        log(f"{precision} adjoint, checkpointed")
        dAs, dBs, ws = ops.join_agg_bwd(A.group, A.key, A.val, B.key, B.group, B.val, N, N, N,
                                        W, precision=precision, tol=TOL, unique=True)
        assert ops.sync_status(ws)[0] == 0
        del ws
        torch.cuda.empty_cache()
        blk_s = Cs[trows][:, tcols].cpu().numpy()
        errs = float(np.max(np.abs(blk_s - Co) / So))
        fes = freivalds_err(Cs)
        log(f"{precision}: block err_cw {errs:.2e}, Freivalds {fes:.2e}")
        assert errs <= 1e-12 and fes <= 1e-12
        got_a = dAs[tia].cpu().numpy()
        assert float(np.max(np.abs(got_a - gA) / sA)) <= TOL
        got_b = dBs[tib].cpu().numpy()
        assert float(np.max(np.abs(got_b - gB) / sB)) <= TOL
        log(f"{precision} gradient checks: {len(ia)} A records, {len(ib)} B records")
        del Cs, dAs, dBs
        torch.cuda.empty_cache()
