"""Helpers shared by the GPU parity tests: device selection, relation
conversion, and the error metrics used against the oracle.

Error metric (componentwise, the form of the standard dot-product error
bound |fl(x^T y) - x^T y| <= gamma_K |x|^T |y|):
    err_cw = max over cells of |C_gpu - C_oracle| / (|X| |Y|)[g,h]
where (|X||Y|)[g,h] = sum over joined pairs of |a.v| |b.w| is itself
evaluated by the oracle on the absolute values.  Cells with no joined pair
must be exactly zero.
"""
import numpy as np
import pytest
import torch

from paper_2112_07552_amd import workloads as wl

TOL = 1e-12  # FP64 tolerance relative to |X||Y| (K * 2^-53 < 1e-12 for K <= 9007)


def cuda_or_skip():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def to_orc(orc, R: wl.Relation):
    return orc.Rel(R.group.cpu().numpy(), R.key.cpu().numpy(),
                   None if R.val is None else R.val.cpu().to(torch.float64).numpy())


def abs_rel(orc, r):
    return orc.Rel(r.group, r.key, None if r.val is None else np.abs(r.val))


def dense_relation_from_matrix(X: torch.Tensor, transpose: bool) -> wl.Relation:
    """Records (row, col, X[row, col]) for every cell.  transpose=False: the
    matrix is X (rows = groups g, cols = keys k); True: Y (rows = keys k,
    cols = groups h)."""
    R, Cc = X.shape
    r = torch.arange(R, dtype=torch.int32, device=X.device).repeat_interleave(Cc)
    c = torch.arange(Cc, dtype=torch.int32, device=X.device).repeat(R)
    v = X.reshape(-1).contiguous()
    if transpose:
        return wl.Relation(c, r, v)  # group = col (h), key = row (k)
    return wl.Relation(r, c, v)      # group = row (g), key = col (k)


def err_cw(got: np.ndarray, ref: np.ndarray, scale: np.ndarray) -> float:
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.asarray(scale, dtype=np.float64)
    zero = scale == 0
    if np.any(got[zero] != 0):
        return float("inf")
    diff = np.abs(got - ref)
    if not np.any(~zero):
        return 0.0
    return float(np.max(diff[~zero] / scale[~zero]))


def describe_worst(got, ref, scale):
    diff = np.abs(np.asarray(got) - np.asarray(ref)) / np.maximum(np.asarray(scale), 1e-300)
    idx = np.unravel_index(int(np.argmax(diff)), diff.shape)
    return f"worst at {idx}: got {np.asarray(got)[idx]!r} ref {np.asarray(ref)[idx]!r}"
