"""Exact rational solution of the LM step by brute force.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Solves Eq. 1 of the paper, (J^T J + lam D^2) p = J^T b, in exact rational
arithmetic (fractions.Fraction) by Gaussian elimination.  Every float64 value
is exactly a rational number, so for small inputs this is the exact minimiser
of Eq. 2 for the stored values.  Pure-Python loops: small inputs only.
"""
from __future__ import annotations

from fractions import Fraction
from typing import Sequence

import numpy as np


def to_fraction(x) -> Fraction:
    if isinstance(x, Fraction):
        return x
    if isinstance(x, (int, np.integer)):
        return Fraction(int(x))
    return Fraction(float(x))  # exact for any binary64 value


def solve_normal_equations(J, b, d2, lam) -> list[Fraction]:
    """Exact p with (J^T J + lam diag(d2)) p = J^T b.

    J: M x N (nested sequences or array), b: M, d2: N (the squared diagonal of D),
    lam: scalar.  All values are converted exactly to Fractions.
    """
    Jf = [[to_fraction(v) for v in row] for row in np.asarray(J, dtype=object)]
    bf = [to_fraction(v) for v in b]
    d2f = [to_fraction(v) for v in d2]
    lamf = to_fraction(lam)
    M = len(Jf)
    N = len(d2f)
    # normal matrix and right-hand side
    Mat = [[sum((Jf[r][i] * Jf[r][j] for r in range(M)), Fraction(0)) for j in range(N)]
           for i in range(N)]
    for i in range(N):
        Mat[i][i] += lamf * d2f[i]
    rhs = [sum((Jf[r][i] * bf[r] for r in range(M)), Fraction(0)) for i in range(N)]
    # Gaussian elimination with exact pivots (first nonzero pivot)
    for col in range(N):
        piv = next((r for r in range(col, N) if Mat[r][col] != 0), None)
        if piv is None:
            raise ZeroDivisionError("singular normal matrix")
        if piv != col:
            Mat[col], Mat[piv] = Mat[piv], Mat[col]
            rhs[col], rhs[piv] = rhs[piv], rhs[col]
        pv = Mat[col][col]
        for r in range(col + 1, N):
            f = Mat[r][col] / pv
            if f != 0:
                row_r, row_c = Mat[r], Mat[col]
                for c in range(col, N):
                    row_r[c] -= f * row_c[c]
                rhs[r] -= f * rhs[col]
    p = [Fraction(0)] * N
    for i in range(N - 1, -1, -1):
        s = rhs[i] - sum((Mat[i][j] * p[j] for j in range(i + 1, N)), Fraction(0))
        p[i] = s / Mat[i][i]
    return p
