"""The FP64 forward captured in a HIP graph (through torch.cuda.graph) and
replayed: every replay, with other work and synchronisations between them,
gives the eager result bit for bit, and the eager result matches the oracle.
The forward enqueues kernels only (the status block is cleared and the
matrices zeroed by kernels, the contraction splits into a second kernel at
1024^3), so it can be captured; the mixed forms read their plan back once
per product and cannot."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2112_07552_amd import _lib, ops
from paper_2112_07552_amd import workloads as wl

from .gpu_util import TOL, abs_rel, cuda_or_skip, err_cw, to_orc

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("N", [128, 1024])
def test_fp64_forward_replays_in_a_hip_graph(orc, N):
    dev = cuda_or_skip()
    A, B = wl.mm_query(N, N, N, seed=50 + N, device=dev)
    rA = ops.make_relation(A.group, A.key, A.val, unique=True)
    rB = ops.make_relation(B.group, B.key, B.val, unique=True)
    L = _lib.load()
    ws = ops.alloc_workspace(ops.workspace_bytes(rA, rB, N, N, N), dev)
    Cm = torch.empty((N, N), dtype=torch.float64, device=dev)
    s = torch.cuda.Stream(device=dev)

    def fwd():
        _lib.check(L.tcu_join_agg_fwd(C.byref(rA), C.byref(rB), N, N, N, 0, 0.0,
                                      C.c_void_p(Cm.data_ptr()), None,
                                      C.c_void_p(ws.data_ptr()), ws.numel(),
                                      C.c_void_p(s.cuda_stream)), "fwd")

    with torch.cuda.stream(s):
        fwd()
    torch.cuda.synchronize()
    eager = Cm.clone()
    assert ops.sync_status(ws)[0] == 0
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        fwd()
    for rep in range(3):
        Cm.fill_(float("nan"))  # eager work between the replays
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            g.replay()
        torch.cuda.synchronize()
        assert torch.equal(Cm, eager), rep
        assert ops.sync_status(ws)[0] == 0
    RA, RB = to_orc(orc, A), to_orc(orc, B)
    Co, _, _ = orc.join_agg(RA, RB, N, N, N)
    So, _, _ = orc.join_agg(abs_rel(orc, RA), abs_rel(orc, RB), N, N, N)
    assert err_cw(eager.cpu().numpy(), Co, So) <= TOL
    del g
