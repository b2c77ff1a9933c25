"""Exact rational solution of small linear systems (test infrastructure only).

The exact solution x = A^{-1} b of a nonsingular system with rational
(here: integer or binary-fraction) entries is unique; Section 2.1 of the
paper defines the direct method as reaching it by Gaussian elimination,
PA = LU, Ly = Pb, Ux = y.  Carried out in exact rational arithmetic
(``fractions.Fraction``) no rounding occurs and the result *is* A^{-1} b, so
the FP64 oracle and the GPU path can be compared with the true answer.
Pure Python: meant for n up to a few dozen.
"""
from __future__ import annotations

from fractions import Fraction
from typing import Sequence


def solve(A: Sequence[Sequence], b: Sequence) -> list[Fraction]:
    """Exact x with A x = b; raises ZeroDivisionError if A is singular."""
    n = len(A)
    M = [[Fraction(v) for v in row] for row in A]
    y = [Fraction(v) for v in b]
    for k in range(n):
        p = next((i for i in range(k, n) if M[i][k] != 0), None)
        if p is None:
            raise ZeroDivisionError("singular matrix")
        if p != k:
            M[k], M[p] = M[p], M[k]
            y[k], y[p] = y[p], y[k]
        for i in range(k + 1, n):
            if M[i][k] != 0:
                l = M[i][k] / M[k][k]
                for j in range(k, n):
                    M[i][j] -= l * M[k][j]
                y[i] -= l * y[k]
    x = [Fraction(0)] * n
    for i in range(n - 1, -1, -1):
        s = y[i] - sum(M[i][j] * x[j] for j in range(i + 1, n))
        x[i] = s / M[i][i]
    return x


def residual(A, x, b) -> list[Fraction]:
    """b - A x exactly."""
    n = len(A)
    return [Fraction(b[i]) - sum(Fraction(A[i][j]) * Fraction(x[j]) for j in range(n))
            for i in range(n)]
