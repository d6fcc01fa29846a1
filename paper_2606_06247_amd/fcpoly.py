"""Continuation maps of the paper's own Fourier continuation for the library
(FC algorithm section: least-squares polynomial fit near each wall, eqs.
vandermonde and qr; extrapolation, eqs. f_right_gap and f_left_gap; blend with
sigma(t) = 10 t^3 - 15 t^4 + 6 t^5, eqs. fc_blend and sigma; Neumann row, eq.
FCNeumann).

The result has the layout of the FC(Gram) maps the library consumes: a C x d
row-major FP64 matrix per wall type, row r - 1 giving the continuation value
r lattice steps beyond a wall from the d values nearest it (ordered inward to
wall).  The blend weight of the high wall at continuation point k is
1 - sigma((k - 1) / (C - 1)); the low wall's point k lies C + 1 - k steps
before its periodic image and, since sigma(1 - t) = 1 - sigma(t), takes the
same row formula, so one map per wall type serves both walls.  Coordinates
are lattice units with the wall at 0; the Neumann derivative row is appended
unweighted.  The least-squares problem is solved as the paper states, by a
QR factorisation of the (augmented) Vandermonde matrix, in 60-digit
arithmetic (mpmath), and each entry is rounded to FP64 once.
"""
from __future__ import annotations

import functools

import mpmath
import numpy as np


def _blend(t):
    return 10 * t ** 3 - 15 * t ** 4 + 6 * t ** 5


def _map(d: int, p: int, C: int, neumann: bool) -> np.ndarray:
    with mpmath.workdps(60):
        nrow = d + (1 if neumann else 0)
        V = mpmath.matrix(nrow, p + 1)
        for i in range(d):
            x = mpmath.mpf(i - (d - 1))
            for m in range(p + 1):
                V[i, m] = x ** m
        if neumann:
            V[d, 1] = 1
        Q, R = mpmath.qr(V, mode="skinny")
        # coefficients for data e_j: R c = Q^T e_j  (the Neumann row's data is 0)
        coef = []
        for j in range(d):
            rhs = mpmath.matrix([Q[j, m] for m in range(p + 1)])
            c = mpmath.lu_solve(R, rhs)
            coef.append([c[m] for m in range(p + 1)])
        out = np.zeros((C, d))
        for r in range(1, C + 1):
            w = 1 - _blend(mpmath.mpf(r - 1) / (C - 1))
            for j in range(d):
                out[r - 1, j] = float(w * mpmath.fsum(coef[j][m] * mpmath.mpf(r) ** m for m in range(p + 1)))
    return out


@functools.lru_cache(maxsize=32)
def build(d: int = 10, p: int = 5, C: int = 16):
    """(Dirichlet map, Neumann map), each C x d FP64, for d fit points,
    degree p and C continuation points."""
    if not (p + 1 <= d and C >= 2):
        raise ValueError("need p + 1 <= d and C >= 2")
    return _map(d, p, C, False), _map(d, p, C, True)
