"""The matrix-core peak probe: rates within the published dense peaks of
MI355X (FP64 78.6 TFLOP/s, int8 5.0 POPS) and deterministic checksums.
Not a step of the method; it is the yardstick the bench reads its roofline
fractions against beside the published peaks."""
import ctypes as C

import pytest
import torch

from paper_2112_07552_amd import _lib

from .gpu_util import cuda_or_skip

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind,peak", [(0, 78.6), (1, 5000.0), (2, 5000.0)])
def test_probe_rate_and_checksum(kind, peak):
    cuda_or_skip()
    L = _lib.load()
    iters = 256
    out = torch.empty(L.tcu_mfma_peak_out_bytes(), dtype=torch.uint8, device="cuda:0")
    sp = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    _lib.check(L.tcu_mfma_peak(kind, iters, C.c_void_p(out.data_ptr()), sp), "peak")
    torch.cuda.synchronize()
    first = out.clone()
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    _lib.check(L.tcu_mfma_peak(kind, iters, C.c_void_p(out.data_ptr()), sp), "peak")
    end.record()
    torch.cuda.synchronize()
    rate = L.tcu_mfma_peak_ops(kind, iters) / (start.elapsed_time(end) * 1e-3) / 1e12
    assert 0.2 * peak < rate <= 1.02 * peak
    assert torch.equal(first, out)
    if kind == 0:
        assert torch.isfinite(out.view(torch.float64)).all()
