"""Seeded synthetic relations shaped like the paper's workloads.

This module only draws inputs; it holds none of the operator's arithmetic, and
both the HIP path and the oracle read the same stored arrays it returns.

The measured workload is the matrix multiplication query of Section 2.3
(case study of Section 5.4.1): two tables of (row_num, col_num, val) records,
one record per cell of a dense matrix, joined on A.row_num = B.col_num and
grouped by (A.col_num, B.row_num).  The paper's data there was synthetic too.
In operator terms: A has records (group g = A.col_num, key k = A.row_num) and
B has records (key k = B.col_num, group h = B.row_num).

Random numbers come from a counter-based generator: SplitMix64's output
function (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014) applied to seed-dependent counters.  Record order is
a seeded bijection of the cells: a 4-round Feistel network over an even number
of bits with cycle walking.  Everything is torch int64 arithmetic (wrapping
multiplication), so the same arrays come out on the CPU and on a GPU.
"""
from __future__ import annotations

from typing import NamedTuple, Optional

import torch

_MASK64 = (1 << 64) - 1


def _s64(c: int) -> int:
    """An unsigned 64-bit constant as the signed int64 with the same bits."""
    c &= _MASK64
    return c - (1 << 64) if c >= (1 << 63) else c


_GOLDEN = _s64(0x9E3779B97F4A7C15)
_M1 = _s64(0xBF58476D1CE4E5B9)
_M2 = _s64(0x94D049BB133111EB)


def _srl(z: torch.Tensor, s: int) -> torch.Tensor:
    """Logical right shift of int64 bit patterns."""
    return (z >> s) & ((1 << (64 - s)) - 1)


def mix64(z: torch.Tensor) -> torch.Tensor:
    """SplitMix64 output function on int64 bit patterns (wrapping)."""
    z = (z ^ _srl(z, 30)) * _M1
    z = (z ^ _srl(z, 27)) * _M2
    return z ^ _srl(z, 31)


def mix64_int(x: int) -> int:
    """Same as mix64 on one Python integer (unsigned 64-bit semantics)."""
    z = x & _MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
    return z ^ (z >> 31)


def stream_key(seed: int, tag: int) -> int:
    """A 64-bit key per (seed, stream tag)."""
    return _s64(mix64_int((seed * 0x100000001B3 + tag * 0xD1B54A32D192ED03) & _MASK64))


def hash_counter(key: int, idx: torch.Tensor) -> torch.Tensor:
    """64 random bits for each counter value idx (int64 tensor)."""
    return mix64(idx * _GOLDEN + key)


def uniform01(key: int, idx: torch.Tensor) -> torch.Tensor:
    """Doubles in [0,1) with 53 random bits: (bits >> 11) * 2^-53 (exact)."""
    return _srl(hash_counter(key, idx), 11).to(torch.float64) * (2.0 ** -53)


def feistel_permute(idx: torch.Tensor, n: int, seed: int, tag: int) -> torch.Tensor:
    """A seeded bijection of [0, n) evaluated at idx (4 Feistel rounds over
    2b bits with 4^b >= n, cycle walking back into [0, n))."""
    if n <= 1:
        return idx.clone()
    b = 1
    while (1 << (2 * b)) < n:
        b += 1
    mask = (1 << b) - 1
    keys = [stream_key(seed, tag * 16 + r) for r in range(4)]

    def rounds(x):
        left, right = x >> b, x & mask
        for k in keys:
            left, right = right, left ^ (mix64(right + k) & mask)
        return (left << b) | right

    y = rounds(idx)
    bad = y >= n
    while bool(bad.any()):
        y[bad] = rounds(y[bad])
        bad = y >= n
    return y


class Relation(NamedTuple):
    """Struct of arrays: group (int32), key (int32), val (float64/float32 or None)."""
    group: torch.Tensor
    key: torch.Tensor
    val: Optional[torch.Tensor]

    @property
    def n(self) -> int:
        return int(self.group.shape[0])

    def to(self, device) -> "Relation":
        return Relation(self.group.to(device), self.key.to(device),
                        None if self.val is None else self.val.to(device))


def draw_values(kind: str, n: int, seed: int, tag: int, device="cpu",
                lo: int = 0, hi: int = 2, dtype=torch.float64) -> torch.Tensor:
    """n values of one distribution, stored as `dtype`.

    kind: 'uniform'     U[-1, 1)
          'loguniform'  |x| = 10^(-4 + 8u), random sign (log-uniform on [1e-4, 1e4])
          'int'         integers uniform in [lo, hi)
          'mixture'     N(0,1) (Box-Muller), each value x1e3 with probability 0.05
    """
    idx = torch.arange(n, dtype=torch.int64, device=device)
    key = stream_key(seed, 1000 + tag)
    if kind == "uniform":
        v = 2.0 * uniform01(key, idx) - 1.0
    elif kind == "loguniform":
        u = uniform01(key, idx)
        s = uniform01(stream_key(seed, 2000 + tag), idx)
        mag = torch.pow(torch.tensor(10.0, dtype=torch.float64, device=device), -4.0 + 8.0 * u)
        v = torch.where(s < 0.5, -mag, mag)
    elif kind == "int":
        u = uniform01(key, idx)
        v = torch.floor(u * float(hi - lo)) + float(lo)
    elif kind == "mixture":
        u1 = uniform01(key, idx)
        u2 = uniform01(stream_key(seed, 2000 + tag), idx)
        u3 = uniform01(stream_key(seed, 3000 + tag), idx)
        z = torch.sqrt(-2.0 * torch.log1p(-u1)) * torch.cos(2.0 * torch.pi * u2)
        v = torch.where(u3 < 0.05, z * 1e3, z)
    else:
        raise ValueError(f"unknown value distribution {kind!r}")
    return v.to(dtype)


def dense_relation(rows: int, cols: int, seed: int, tag: int, values: str = "uniform",
                   order: str = "random", device="cpu", dtype=torch.float64,
                   lo: int = 0, hi: int = 2, row_is_group: bool = False) -> Relation:
    """One record per cell of a rows x cols matrix (the MM query's tables).

    Cell c = r * cols + q holds (row_num = r, col_num = q).  For table A of the
    MM query use row_is_group=False: key = row_num, group = col_num.  For
    table B use row_is_group=True: group = row_num, key = col_num.
    order: 'random' (seeded bijection of the cells) or 'sorted' (row-major).
    """
    n = rows * cols
    idx = torch.arange(n, dtype=torch.int64, device=device)
    cell = feistel_permute(idx, n, seed, tag) if order == "random" else idx
    r = torch.div(cell, cols, rounding_mode="floor")
    q = cell - r * cols
    val = draw_values(values, n, seed, tag, device=device, lo=lo, hi=hi, dtype=dtype)
    if row_is_group:
        return Relation(r.to(torch.int32), q.to(torch.int32), val)
    return Relation(q.to(torch.int32), r.to(torch.int32), val)


def mm_query(M: int, K: int, N: int, seed: int, values: str = "uniform", order: str = "random",
             device="cpu", dtype=torch.float64, lo: int = 0, hi: int = 2):
    """Dense tables of the MM query: A is K x M (row_num = k, col_num = g),
    B is N x K (row_num = h, col_num = k).  Returns (A, B) as Relations."""
    A = dense_relation(K, M, seed, 1, values, order, device, dtype, lo, hi, row_is_group=False)
    B = dense_relation(N, K, seed, 2, values, order, device, dtype, lo, hi, row_is_group=True)
    return A, B


def random_relation(n: int, groups: int, keys: int, seed: int, tag: int,
                    values: str = "uniform", device="cpu", dtype=torch.float64,
                    lo: int = 0, hi: int = 2, bad_fraction: float = 0.0) -> Relation:
    """n records with group and key drawn uniformly (duplicates allowed).

    With bad_fraction > 0 that share of records gets an out-of-range key or
    group (negative or too large), for the operator's skip-and-report path."""
    idx = torch.arange(n, dtype=torch.int64, device=device)
    g = torch.floor(uniform01(stream_key(seed, 4000 + tag), idx) * groups).to(torch.int64)
    k = torch.floor(uniform01(stream_key(seed, 5000 + tag), idx) * keys).to(torch.int64)
    if bad_fraction > 0:
        u = uniform01(stream_key(seed, 6000 + tag), idx)
        which = uniform01(stream_key(seed, 7000 + tag), idx)
        bad = u < bad_fraction
        g = torch.where(bad & (which < 0.25), torch.full_like(g, -1), g)
        g = torch.where(bad & (which >= 0.25) & (which < 0.5), torch.full_like(g, groups), g)
        k = torch.where(bad & (which >= 0.5) & (which < 0.75), torch.full_like(k, -7), k)
        k = torch.where(bad & (which >= 0.75), torch.full_like(k, keys + 3), k)
    val = draw_values(values, n, seed, 8000 + tag, device=device, lo=lo, hi=hi, dtype=dtype)
    return Relation(g.to(torch.int32), k.to(torch.int32), val)


def id_column(n: int, distinct: int, seed: int, tag: int, device="cpu") -> torch.Tensor:
    """n int64 IDs drawn uniformly from a pool of `distinct` random 64-bit
    values.  The pool depends on the seed only, so two columns with the same
    seed and different tags share one domain (a join attribute, Section 3.1);
    the choice of pool member per record depends on the tag."""
    pool = hash_counter(stream_key(seed, 0), torch.arange(max(distinct, 1), dtype=torch.int64,
                                                          device=device))
    u = uniform01(stream_key(seed, 100 + tag), torch.arange(n, dtype=torch.int64, device=device))
    return pool[torch.floor(u * distinct).to(torch.int64)]


def local_edges(n: int, nodes: int, width: int, seed: int, tag: int, device="cpu",
                values: str = "uniform", dtype=torch.float64) -> Relation:
    """n edges (src, dst) of a graph with spatial locality, as in a road
    network: src uniform over the nodes, dst = src + d mod nodes with d
    uniform in [-width, width].  Returned as a Relation with group = src,
    key = dst."""
    idx = torch.arange(n, dtype=torch.int64, device=device)
    src = torch.floor(uniform01(stream_key(seed, 9000 + tag), idx) * nodes).to(torch.int64)
    d = torch.floor(uniform01(stream_key(seed, 9100 + tag), idx) * (2 * width + 1)).to(torch.int64)
    dst = torch.remainder(src + d - width, nodes)
    val = draw_values(values, n, seed, 9200 + tag, device=device, dtype=dtype)
    return Relation(src.to(torch.int32), dst.to(torch.int32), val)

