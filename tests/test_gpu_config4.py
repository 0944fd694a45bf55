"""The mixed forms at 2^24 records per table with values log-uniform in
magnitude on [1e-4, 1e4] and random sign (seed 3): the dense matrix
multiplication query of Section 5.4.1 with N = 4096, the workload on which
the narrow forms must match the FP64 form's accuracy.

Every form (residues, int8 digits, BF16 digits) runs the forward and the
adjoint, with the forward's encodings kept (saved) and rebuilt from the
records (checkpointed).  Against the FP64 oracle, on 512 whole rows of C,
4096 random cells, Freivalds' check over all of C and the gradients of 4096
random records of each table, every sampled value must meet the certified
guarantee err_cw <= 1e-12 (the error relative to |X||Y|, |W||Y^T| or
|X^T||W| of that cell).  The checkpointed adjoint must equal the saved one
bit for bit (the encodings of unique cells are rebuilt exactly).
"""
import numpy as np
import pytest
import torch

from oracle import sample
from paper_2112_07552_amd import ops
from paper_2112_07552_amd import workloads as wl

from .gpu_util import cuda_or_skip, to_orc

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

N = 4096
TOL = 1e-12


def log(msg):
    print(f"[config4] {msg}", flush=True)


@pytest.fixture(scope="module")
def case(orc):
    dev = cuda_or_skip()
    log("inputs and the oracle's sample")
    A, B = wl.mm_query(N, N, N, seed=3, values="loguniform", device=dev)
    W = wl.draw_values("uniform", N * N, 1003, 0, device=dev).reshape(N, N)
    ref = sample.reference(to_orc(orc, A), to_orc(orc, B), N, N, N, W.cpu().numpy(), seed=3)
    log("oracle sample ready")
    return A, B, W, ref


@pytest.mark.parametrize("precision", ["crt_i8", "split_i8", "split_bf16"])
def test_config4_mixed_forward_adjoint(case, precision):
    A, B, W, ref = case
    args = (A.group, A.key, A.val, B.key, B.group, B.val, N, N, N)
    log(f"{precision}: forward")
    Cm, _, ws = ops.join_agg_fwd(*args, precision=precision, tol=TOL, unique=True,
                                 for_backward=True)
    st, info = ops.sync_status(ws)
    assert st == 0, info
    assert info["flags"] & ops._lib.TCU_FLAG_FALLBACK == 0, info
    log(f"{precision}: plan {info}")
    C = Cm.cpu().numpy()
    log(f"{precision}: adjoint (saved encodings)")
    dA, dB, _ = ops.join_agg_bwd(*args, W, precision=precision, tol=TOL, ws=ws, unique=True,
                                 saved_encodings=True)
    st, info_b = ops.sync_status(ws)
    assert st == 0 and info_b["flags"] & ops._lib.TCU_FLAG_FALLBACK == 0, info_b
    dA, dB = dA.cpu().numpy(), dB.cpu().numpy()
    errs = sample.errors(ref, C, dA, dB)
    log(f"{precision}: err_cw {errs}")
    assert errs["max"] <= TOL, errs
    log(f"{precision}: adjoint (checkpointed)")
    dA2, dB2, ws2 = ops.join_agg_bwd(*args, W, precision=precision, tol=TOL, unique=True)
    assert ops.sync_status(ws2)[0] == 0
    assert np.array_equal(dA2.cpu().numpy(), dA) and np.array_equal(dB2.cpu().numpy(), dB)


def test_config4_fp64_reference_error(case):
    """The FP64 form on the same sample: the accuracy the narrow forms must
    match."""
    A, B, W, ref = case
    args = (A.group, A.key, A.val, B.key, B.group, B.val, N, N, N)
    Cm, _, ws = ops.join_agg_fwd(*args, unique=True, for_backward=True)
    dA, dB, _ = ops.join_agg_bwd(*args, W, ws=ws, unique=True, saved_encodings=True)
    assert ops.sync_status(ws)[0] == 0
    errs = sample.errors(ref, Cm.cpu().numpy(), dA.cpu().numpy(), dB.cpu().numpy())
    log(f"fp64: err_cw {errs}")
    assert errs["max"] <= TOL, errs
