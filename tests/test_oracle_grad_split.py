"""Pins of the oracle's gradient and fixed-point slicing.

Gradient of L = sum(W * C): checked against exact rational brute force over
record pairs, against a library matrix product on dense tables, and against
central differences of the oracle's own forward (L is linear in each value, so
the difference quotient has no truncation error).

Slicing (the mixed-precision form's number format): checked against an exact
integer re-derivation in Python and against the reconstruction identity.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
import torch

from paper_2112_07552_amd import workloads as wl

from .test_oracle_pins import small_case, to_rel

U = 2.0 ** -53


def brute_grad(A, B, W, M, K, N):
    dA = [Fraction(0)] * A.n
    dB = [Fraction(0)] * B.n
    for i in range(A.n):
        g, k = int(A.group[i]), int(A.key[i])
        if not (0 <= g < M and 0 <= k < K):
            continue
        for j in range(B.n):
            kb, h = int(B.key[j]), int(B.group[j])
            if kb != k or not (0 <= h < N):
                continue
            dA[i] += Fraction(float(W[g, h])) * Fraction(float(B.val[j]))
            dB[j] += Fraction(float(W[g, h])) * Fraction(float(A.val[i]))
    return dA, dB


@pytest.mark.parametrize("seed,bad", [(61, 0.0), (62, 0.15)])
def test_grad_brute_force(orc, seed, bad):
    M, K, N = 5, 6, 7
    A, B = small_case(seed, 60, 64, M, K, N, bad=bad)
    W = np.random.default_rng(seed).uniform(-1, 1, (M, N))
    rA, rB = to_rel(orc, A), to_rel(orc, B)
    dA = orc.grad(rA, rB, M, K, N, W, "A")
    dB = orc.grad(rA, rB, M, K, N, W, "B")
    eA, eB = brute_grad(A, B, W, M, K, N)
    for i in range(A.n):
        assert abs(Fraction(float(dA[i])) - eA[i]) <= Fraction(U) * abs(eA[i]) + Fraction(1, 2**90)
    for j in range(B.n):
        assert abs(Fraction(float(dB[j])) - eB[j]) <= Fraction(U) * abs(eB[j]) + Fraction(1, 2**90)
    # sampled indices give the same numbers
    idx = np.array([3, 0, 59, 3], dtype=np.int64)
    assert np.array_equal(orc.grad(rA, rB, M, K, N, W, "A", idx=idx), dA[idx])


def test_grad_dense_matches_library(orc):
    """Dense tables: dX = W Y^T and dY = X^T W gathered at each record."""
    M, K, N = 48, 40, 56
    A, B = wl.mm_query(M, K, N, seed=63)
    W = np.random.default_rng(2).uniform(-1, 1, (M, N))
    X = np.zeros((M, K)); X[A.group.numpy(), A.key.numpy()] = A.val.numpy()
    Y = np.zeros((K, N)); Y[B.key.numpy(), B.group.numpy()] = B.val.numpy()
    rA, rB = to_rel(orc, A), to_rel(orc, B)
    dA = orc.grad(rA, rB, M, K, N, W, "A")
    dB = orc.grad(rA, rB, M, K, N, W, "B")
    dX, dY = W @ Y.T, X.T @ W
    sX, sY = np.abs(W) @ np.abs(Y.T), np.abs(X.T) @ np.abs(W)
    ga, ka = A.group.numpy(), A.key.numpy()
    kb, hb = B.key.numpy(), B.group.numpy()
    assert np.all(np.abs(dA - dX[ga, ka]) <= 2 * N * U * sX[ga, ka])
    assert np.all(np.abs(dB - dY[kb, hb]) <= 2 * M * U * sY[kb, hb])


def test_grad_central_difference(orc):
    """L = sum(W*C) is linear in each value: (L(v+h) - L(v-h)) / 2h equals the
    derivative up to the rounding of L alone."""
    M, K, N = 12, 10, 14
    A, B = small_case(64, 300, 300, M, K, N)
    W = np.random.default_rng(3).uniform(-1, 1, (M, N))
    rA, rB = to_rel(orc, A), to_rel(orc, B)
    dA = orc.grad(rA, rB, M, K, N, W, "A")
    h = 2.0 ** -10

    def L(Arel):
        C, _, _ = orc.join_agg(Arel, rB, M, K, N)
        return float(np.sum(np.asarray([Fraction(x) * Fraction(w) for x, w in zip(C.ravel(), W.ravel())], dtype=object)))

    for i in [0, 17, 123, 299]:
        vp = A.val.numpy().copy(); vp[i] += h
        vm = A.val.numpy().copy(); vm[i] -= h
        fd = (L(orc.Rel(rA.group, rA.key, vp)) - L(orc.Rel(rA.group, rA.key, vm))) / (2 * h)
        assert abs(fd - dA[i]) <= 1e-9 * (1 + abs(dA[i]))


def exact_slices(xs, nslices, bits):
    """Independent re-derivation with Python integers: scale the line so that
    its largest magnitude lies in [1/2, 1), then read off base-2^bits digits
    of |x| by integer division, each carrying the sign of x."""
    fr = [Fraction(float(x)) for x in xs]
    mx = max((abs(f) for f in fr), default=Fraction(0))
    e = 0
    if mx > 0:
        while mx >= Fraction(2) ** e:
            e += 1
        while mx < Fraction(2) ** (e - 1):
            e -= 1
    digits = []
    for f in fr:
        r = abs(f) / Fraction(2) ** e
        ds = []
        for _ in range(nslices):
            r *= 2 ** bits
            d = r.numerator // r.denominator
            ds.append(d if f >= 0 else -d)
            r -= d
        digits.append(ds)
    return e, digits


@pytest.mark.parametrize("kind", ["uniform", "loguniform", "int"])
def test_split_matches_integer_derivation(orc, kind):
    R, L = 9, 13
    X = wl.draw_values(kind, R * L, 71, 0, lo=-2**15, hi=2**15).numpy().reshape(R, L)
    X[3, :] = 0.0               # an all-zero line
    X[5, 2] = 2.0 ** -1070      # a subnormal
    for axis in (0, 1):
        exps, sl = orc.split(X, axis, 7, 8)
        lines = range(R) if axis == 0 else range(L)
        for line in lines:
            xs = X[line, :] if axis == 0 else X[:, line]
            e, digits = exact_slices(xs, 7, 8)
            assert exps[line] == e
            for t, ds in enumerate(digits):
                got = sl[:, line, t] if axis == 0 else sl[:, t, line]
                assert [int(d) for d in got] == ds
                assert all(abs(d) < 256 for d in ds)


def test_split_reconstruction_bound(orc):
    """x - 2^e sum_p d_p 2^(-8p) has magnitude below 2^(e - 8s), and is zero
    once s slices cover the 53 bits below the line's top bit."""
    X = wl.draw_values("uniform", 40 * 30, 72, 0).numpy().reshape(40, 30)
    for s in (2, 5, 7):
        exps, sl = orc.split(X, 0, s, 8)
        for g in range(40):
            for k in range(30):
                rec = sum(Fraction(int(sl[p, g, k])) * Fraction(2) ** (int(exps[g]) - 8 * (p + 1)) for p in range(s))
                err = abs(Fraction(float(X[g, k])) - rec)
                assert err < Fraction(2) ** (int(exps[g]) - 8 * s)
                if s == 7:
                    assert err == 0


def test_split_rejects_non_finite(orc):
    X = np.ones((3, 4))
    X[1, 2] = np.inf
    with pytest.raises(FloatingPointError):
        orc.split(X, 0, 3, 8)


def _trunc_product_exact(X, Y, bits):
    """The same definition in Python integers (independent arithmetic)."""
    M, K = X.shape
    N = Y.shape[1]
    ex = [math.frexp(max(abs(v) for v in X[g]))[1] if any(X[g]) else 0 for g in range(M)]
    ey = [math.frexp(max(abs(Y[k, h]) for k in range(K)))[1] if any(Y[:, h]) else 0
          for h in range(N)]
    xi = [[int(math.ldexp(X[g, k], bits - ex[g])) for k in range(K)] for g in range(M)]
    yi = [[int(math.ldexp(Y[k, h], bits - ey[h])) for h in range(N)] for k in range(K)]
    out = np.empty((M, N))
    for g in range(M):
        for h in range(N):
            p = sum(xi[g][k] * yi[k][h] for k in range(K))
            out[g, h] = math.ldexp(float(p), ex[g] + ey[h] - 2 * bits)
    return out


@pytest.mark.parametrize("bits", [7, 30, 42, 53])
def test_trunc_product_matches_python_integers(orc, bits):
    rng = np.random.default_rng(bits)
    X = rng.standard_normal((6, 9)) * np.exp(rng.uniform(-8, 8, (6, 9)))
    Y = rng.standard_normal((9, 5)) * np.exp(rng.uniform(-8, 8, (9, 5)))
    X[2] = 0.0           # an all-zero line
    Y[:, 1] *= 1e-300    # a line of subnormal-range magnitudes
    got = orc.trunc_product(X, Y, bits)
    assert np.array_equal(got, _trunc_product_exact(X, Y, bits))


def test_trunc_product_error_bound_and_integers(orc):
    """|X'Y' scaled - XY| <= K max|X_g| max|Y_h| (2^(2-b) + 2^(2-2b)) against the
    exact rational product; integer inputs below 2^bits come back exact."""
    rng = np.random.default_rng(7)
    X = rng.uniform(-1, 1, (8, 12)) * 10.0 ** rng.uniform(-4, 4, (8, 12))
    Y = rng.uniform(-1, 1, (12, 6)) * 10.0 ** rng.uniform(-4, 4, (12, 6))
    for bits in (10, 20, 42):
        got = orc.trunc_product(X, Y, bits)
        for g in range(8):
            for h in range(6):
                exact = sum(Fraction(X[g, k]) * Fraction(Y[k, h]) for k in range(12))
                bound = 12 * np.abs(X[g]).max() * np.abs(Y[:, h]).max() * (
                    2.0 ** (2 - bits) + 2.0 ** (2 - 2 * bits))
                assert abs(Fraction(got[g, h]) - exact) <= Fraction(bound)
    Xi = rng.integers(-1000, 1000, (7, 11)).astype(np.float64)
    Yi = rng.integers(-1000, 1000, (11, 4)).astype(np.float64)
    assert np.array_equal(orc.trunc_product(Xi, Yi, 42), Xi @ Yi)
