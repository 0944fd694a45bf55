"""Pins of the oracle's certificate (orc_certificate), the plan of the mixed
forms, against exact rational arithmetic on small inputs.

What the certificate promises, checked with Python's Fractions:
  * D_lo = 2^(e_g + f_h - 14) T <= (|X||Y|)[g,h] in every cell, with T the
    brute-force sum of the magnitude codes;
  * with b = need_bits, the exact product of the per-line truncations to
    b-bit integers differs from the exact product by at most
    2^(e_g + f_h - b) (s_g + s_h), and by at most tcrt (|X||Y|)[g,h];
  * with S = need_slices, the exact sum of the digit pairs on the first S
    anti-diagonals differs by at most 2^(e_g + f_h - 7S) (s_g + s_h +
    (S - 1) K), and by at most tdig[S] (|X||Y|)[g,h].
Inputs of 1 - 2^-53 (the largest double below 1) make every truncation lose almost a whole unit in the
same direction, so the bounds are nearly attained there: a certificate that
dropped a term of the bound would pick a width one too small and fail the
"at most tol |X||Y|" check on those inputs.
"""
from fractions import Fraction

import numpy as np
import pytest

TOL = 1e-12


def _tols(K, tol=TOL):
    tcrt = tol
    tdig = [0.0] + [tol] * 8
    return tcrt, tdig


def _exp(line):
    mx = max(abs(v) for v in line)
    return 0 if mx == 0 else int(np.frexp(mx)[1])


def _trunc(v, shift):
    """trunc(v 2^shift) exactly, as an int."""
    f = Fraction(v) * Fraction(2) ** shift
    return int(f) if f >= 0 else -int(-f)


def _digits(v, e, S):
    """S base-128 digits of v 2^-e (truncation, each step exact)."""
    r = Fraction(v) / Fraction(2) ** e
    out = []
    for _ in range(S):
        t = r * 128
        d = int(t) if t >= 0 else -int(-t)
        out.append(d)
        r = t - d
    return out


def _cases():
    rng = np.random.default_rng(7)
    near_one = 1.0 - 2.0 ** -53
    yield "uniform", rng.uniform(-1, 1, (7, 9)), rng.uniform(-1, 1, (9, 6))
    yield "loguniform", (10.0 ** rng.uniform(-4, 4, (6, 11))) * rng.choice([-1, 1], (6, 11)), \
        (10.0 ** rng.uniform(-4, 4, (11, 5))) * rng.choice([-1, 1], (11, 5))
    yield "near_one", np.full((4, 10), near_one), np.full((10, 3), near_one)
    yield "near_one_scaled", np.full((3, 8), near_one) * 2.0 ** 40, \
        np.full((8, 4), near_one) * 2.0 ** -30


@pytest.mark.parametrize("name,X,Y", list(_cases()), ids=lambda v: v if isinstance(v, str) else "")
def test_certificate_bounds_hold_exactly(orc, name, X, Y):
    M, K = X.shape
    N = Y.shape[1]
    tcrt, tdig = _tols(K)
    nb, ns, umax, T, sums = orc.certificate(X, Y, tcrt, tdig, with_detail=True)
    ex = [_exp(X[g]) for g in range(M)]
    ey = [_exp(Y[:, h]) for h in range(N)]
    sx = [sum(Fraction(abs(v)) for v in X[g]) / Fraction(2) ** ex[g] for g in range(M)]
    sy = [sum(Fraction(abs(v)) for v in Y[:, h]) / Fraction(2) ** ey[h] for h in range(N)]
    # the normalised sums: one rounding of the exact value
    for i, s in enumerate(sx + sy):
        assert abs(Fraction(sums[i]) - s) <= s * Fraction(2) ** -52
    assert umax[0] == max(float(s) for s in sx) or abs(umax[0] - float(max(sx))) <= 1e-15 * umax[0]
    qx = [[int(Fraction(abs(v)) * Fraction(2) ** (7 - ex[g])) for v in X[g]] for g in range(M)]
    qy = [[int(Fraction(abs(Y[k, h])) * Fraction(2) ** (7 - ey[h])) for k in range(K)]
          for h in range(N)]
    xd = [[_digits(X[g, k], ex[g], ns) for k in range(K)] for g in range(M)] if ns <= 8 else None
    yd = [[_digits(Y[k, h], ey[h], ns) for k in range(K)] for h in range(N)] if ns <= 8 else None
    assert ns <= 8 or ns == 255
    for g in range(M):
        for h in range(N):
            t = sum(qx[g][k] * qy[h][k] for k in range(K))
            assert T[g, h] == t
            D = sum(Fraction(abs(X[g, k])) * Fraction(abs(Y[k, h])) for k in range(K))
            exact = sum(Fraction(X[g, k]) * Fraction(Y[k, h]) for k in range(K))
            scale = Fraction(2) ** (ex[g] + ey[h])
            assert scale * t / 16384 <= D
            # residue form at the certified width
            b = nb
            p = sum(_trunc(X[g, k], b - ex[g]) * _trunc(Y[k, h], b - ey[h]) for k in range(K))
            err = abs(p * scale / Fraction(2) ** (2 * b) - exact)
            assert err <= scale * Fraction(2) ** -b * (sx[g] + sy[h])
            assert err <= Fraction(tcrt) * D, (name, g, h, float(err / D))
            # digit forms at the certified digit count
            if xd is not None:
                S = ns
                kept = sum(Fraction(xd[g][k][p1] * yd[h][k][q1], 128 ** (p1 + q1 + 2))
                           for k in range(K) for p1 in range(S) for q1 in range(S)
                           if p1 + q1 + 2 <= S + 1)
                errd = abs(kept * scale - exact)
                assert errd <= scale * Fraction(2) ** (-7 * S) * (sx[g] + sy[h] + (S - 1) * K)
                assert errd <= Fraction(tdig[S]) * D, (name, g, h, float(errd / D))


def test_certificate_near_one_is_tight(orc):
    """On the near-1 inputs the truncation error reaches most of its bound:
    one bit fewer than the certified width would break the guarantee."""
    near_one = 1.0 - 2.0 ** -53
    X = np.full((2, 16), near_one)
    Y = np.full((16, 2), near_one)
    tcrt, tdig = _tols(16)
    nb, _, _ = orc.certificate(X, Y, tcrt, tdig)
    K = 16
    exact = K * Fraction(near_one) ** 2
    b = nb - 1
    p = K * _trunc(near_one, b) ** 2
    err = abs(Fraction(p, 2 ** (2 * b)) - exact)
    assert err > Fraction(tcrt) * exact


def test_certificate_special_cells(orc):
    tcrt, tdig = _tols(4)
    Z = np.zeros((3, 4))
    assert orc.certificate(Z, np.ones((4, 2)), tcrt, tdig)[:2] == (0, 0)
    # row 0 of X: one huge and one tiny value; column 0 of Y is nonzero only
    # where X's row holds the tiny value, whose magnitude code is 0: T = 0 with
    # a nonzero bound, which no width certifies
    X = np.array([[1e6, 1e-6, 0.0, 0.0]])
    Y = np.array([[0.0], [1.0], [0.0], [0.0]])
    nb, ns, _ = orc.certificate(X, Y, tcrt, tdig)
    assert (nb, ns) == (255, 255)
    # the same row against a column that meets the huge value: certified
    Y2 = np.array([[1.0], [1.0], [0.0], [0.0]])
    nb2, ns2, _ = orc.certificate(X, Y2, tcrt, tdig)
    assert 1 <= nb2 <= 60 and (1 <= ns2 <= 8 or ns2 == 255)
