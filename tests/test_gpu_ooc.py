"""The FP64 product over host-resident operands, streamed through a small
device buffer in blocks (Section 4.2.3), against the oracle.

The oracle evaluates the join-aggregate of the dense tables of A and B (one
record per cell), i.e. the product by its definition, with Dot2.  Small
blocks force many k-blocks, ragged edges and reuse of both device buffers."""
import numpy as np
import pytest
import torch

from paper_2112_07552_amd import ops

from .gpu_util import TOL, abs_rel, cuda_or_skip, dense_relation_from_matrix, err_cw, to_orc

pytestmark = pytest.mark.gpu


def pinned_uniform(rows, cols, seed):
    g = torch.Generator().manual_seed(seed)
    t = torch.empty((rows, cols), dtype=torch.float64, pin_memory=True)
    t.copy_(torch.rand((rows, cols), generator=g, dtype=torch.float64) * 2 - 1)
    return t


@pytest.mark.parametrize("m,n,k,block", [(700, 500, 900, 128), (257, 129, 1000, 128),
                                         (1000, 300, 1, 256), (130, 140, 150, 0),
                                         # edge blocks 188 x 244 wide with k blocks of
                                         # 256 and 132: tiles moved back inside, adding
                                         # into C
                                         (700, 500, 900, 256), (700, 500, 900, 384)])
def test_host_gemm_matches_oracle(orc, m, n, k, block):
    cuda_or_skip()
    A, B = pinned_uniform(m, k, m + k), pinned_uniform(k, n, n + k + 1)
    dev_bytes = 48 * block * block if block else 64 << 20
    Cg = ops.gemm_f64_host(A, B, dev_bytes=dev_bytes, block=block).numpy()
    RA = to_orc(orc, dense_relation_from_matrix(A, False))
    RB = to_orc(orc, dense_relation_from_matrix(B, True))
    Co, _, _ = orc.join_agg(RA, RB, m, k, n)
    So, _, _ = orc.join_agg(abs_rel(orc, RA), abs_rel(orc, RB), m, k, n)
    assert err_cw(Cg, Co, So) <= TOL


def test_host_gemm_k_zero_and_large_blocks(orc):
    cuda_or_skip()
    A = torch.empty((300, 0), dtype=torch.float64, pin_memory=True)
    B = torch.empty((0, 200), dtype=torch.float64, pin_memory=True)
    out = torch.full((300, 200), 7.0, dtype=torch.float64, pin_memory=True)
    ops.gemm_f64_host(A, B, out=out, dev_bytes=48 * 128 * 128, block=128)
    assert torch.all(out == 0)
    # 4096^3 in 1024-blocks against the device-resident product on sampled cells
    N = 4096
    A, B = pinned_uniform(N, N, 11), pinned_uniform(N, N, 12)
    Ch = ops.gemm_f64_host(A, B, dev_bytes=48 * 1024 * 1024 * 8, block=1024).numpy()
    rng = np.random.default_rng(3)
    cg = rng.integers(0, N, 512).astype(np.int32)
    ch = rng.integers(0, N, 512).astype(np.int32)
    RA = to_orc(orc, dense_relation_from_matrix(A, False))
    RB = to_orc(orc, dense_relation_from_matrix(B, True))
    vo, _ = orc.join_agg_cells(RA, RB, N, N, N, cg, ch)
    so, _ = orc.join_agg_cells(abs_rel(orc, RA), abs_rel(orc, RB), N, N, N, cg, ch)
    assert np.max(np.abs(Ch[cg, ch] - vo) / so) <= TOL
