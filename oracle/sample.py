"""The oracle on a sample of a large output (test infrastructure).

For outputs too large to evaluate whole on the CPU, the FP64 oracle
(oracle.py) is evaluated on:
  * whole rows of C,
  * random cells of C,
  * Freivalds' check (R. Freivalds, 1977): C r against X (Y r) for random
    +-1 vectors r, which covers every cell of C at O(n) cost,
  * the value gradients of random records of A and B,
each with its componentwise scale, the same quantity for the absolute
values (|X||Y| for C, (|W||Y^T|) and (|X^T||W|) for the gradients, |X||Y| 1
for Freivalds).  err_cw of a part is max |got - ref| / scale.

Only the tests, the smoke check and the benchmark's checks use this module.
"""
from __future__ import annotations

import numpy as np

from . import oracle as orc


def _abs(R: orc.Rel) -> orc.Rel:
    return orc.Rel(R.group, R.key, None if R.val is None else np.abs(R.val))


def reference(RA: orc.Rel, RB: orc.Rel, M: int, K: int, N: int, W=None, rows: int = 512,
              cells: int = 4096, records: int = 4096, probes: int = 2, seed: int = 0) -> dict:
    """Oracle values on a seeded sample (W: the M x N adjoint seed dC as a
    numpy array, or None for the forward only)."""
    rng = np.random.default_rng(seed)
    RAa, RBa = _abs(RA), _abs(RB)
    ref = {"M": M, "K": K, "N": N}
    ridx = np.sort(rng.choice(M, min(rows, M), replace=False)).astype(np.int32)
    ref["rows"] = ridx
    ref["C_rows"] = orc.join_agg(RA, RB, M, K, N, rows=ridx)[0]
    ref["S_rows"] = orc.join_agg(RAa, RBa, M, K, N, rows=ridx)[0]
    cg = rng.integers(0, M, cells).astype(np.int32)
    ch = rng.integers(0, N, cells).astype(np.int32)
    ref["cells"] = (cg, ch)
    ref["C_cells"] = orc.join_agg_cells(RA, RB, M, K, N, cg, ch)[0]
    ref["S_cells"] = orc.join_agg_cells(RAa, RBa, M, K, N, cg, ch)[0]
    ref["probes"] = []
    for _ in range(probes):
        r = np.where(rng.random(N) < 0.5, -1.0, 1.0)
        ref["probes"].append((r, orc.freivalds(RA, RB, M, K, N, r)))
    ref["S_freivalds"] = orc.freivalds(RAa, RBa, M, K, N, np.ones(N))
    if W is not None:
        Wa = np.abs(W)
        for name, R in (("A", RA), ("B", RB)):
            idx = np.sort(rng.choice(R.n, min(records, R.n), replace=False)).astype(np.int64)
            ref[f"idx_{name}"] = idx
            ref[f"g_{name}"] = orc.grad(RA, RB, M, K, N, W, name, idx=idx)
            ref[f"s_{name}"] = orc.grad(RAa, RBa, M, K, N, Wa, name, idx=idx)
    return ref


def _err(got, want, scale) -> float:
    got = np.asarray(got, dtype=np.float64)
    diff = np.abs(got - want)
    zero = scale == 0
    if np.any(diff[zero] != 0):
        return float("inf")
    return float(np.max(diff[~zero] / scale[~zero])) if np.any(~zero) else 0.0


def errors(ref: dict, C: np.ndarray, dA=None, dB=None) -> dict:
    """err_cw of each sampled part for a result C (M x N numpy array) and
    optional gradients (numpy arrays over all records)."""
    out = {}
    out["rows"] = _err(C[ref["rows"]], ref["C_rows"], ref["S_rows"])
    cg, ch = ref["cells"]
    out["cells"] = _err(C[cg, ch], ref["C_cells"], ref["S_cells"])
    worst = 0.0
    for r, rhs in ref["probes"]:
        # C r with r = +-1: exact products, numpy's pairwise summation
        lhs = np.empty(C.shape[0])
        for r0 in range(0, C.shape[0], 1024):
            lhs[r0:r0 + 1024] = (C[r0:r0 + 1024] * r).sum(axis=1)
        worst = max(worst, _err(lhs, rhs, ref["S_freivalds"]))
    out["freivalds"] = worst
    for name, g in (("A", dA), ("B", dB)):
        if g is not None and f"idx_{name}" in ref:
            out[f"grad_{name}"] = _err(np.asarray(g)[ref[f"idx_{name}"]], ref[f"g_{name}"],
                                       ref[f"s_{name}"])
    out["max"] = max(out.values())
    return out
