"""The paper's own Fourier continuation as continuation maps (oracle side).

TEST INFRASTRUCTURE (see ``oracle/__init__.py``).

Sec. "Fourier Continuation (FC) Algorithm", steps 1-3: a degree-p polynomial
is fitted by least squares to the values at the d lattice points nearest each
wall (eqs. vandermonde, least_squares; the paper solves it by QR, eq. qr),
extrapolated into the extension (eqs. f_right_gap, f_left_gap), and the two
extrapolations are blended with sigma(t) = 10 t^3 - 15 t^4 + 6 t^5 (eqs.
fc_blend, sigma).  Neumann walls append the derivative row (eq. FCNeumann).
(The paper calls the fit points C and the extension length d; here, as in the
FC(Gram) tables, d counts matching points and C continuation points.)

Readings (where the section is garbled or silent):
* indexing as for FC(Gram): the wall is a lattice point, the C continuation
  points are distinct and the period is (n + C) lattice steps, so
  continuation point k (k = 1..C) lies k steps beyond the high wall and
  C + 1 - k steps before the low wall's periodic image (the paper's literal
  indices put the last extension point on the low wall itself);
* blend parameter t_k = (k - 1) / (C - 1) as printed;
* wall-local coordinates in lattice units (xi = 0 at the wall, xi = -1, -2, ..
  inward), which keeps the maps independent of the spacing; the Neumann row
  [0 .. 0 1 0] (the coefficient of xi, right-hand side 0) is appended
  unweighted in these units, as printed.
Because sigma(1 - t) = 1 - sigma(t), the low wall's blended extrapolation at
distance r is the high wall's formula at distance r applied to the mirrored
data, so one C x d map per wall type serves both walls (``oracle.fc``):

    M[r-1][j] = (1 - sigma(t_r)) * sum_m r^m P[m][j],

P the least-squares solution operator (coefficients from the d data values).

Construction: the least-squares solution is the unique solution of the normal
equations V^T V c = V^T f; they are solved here in exact rational arithmetic
(``fractions.Fraction``) and each map entry is rounded to FP64 once.

Parity: pinned in ``tests/test_oracle_fcpoly.py`` by exact reproduction of
constants and of polynomials of degree <= p (one-sided extrapolation times
the blend weight), the blend weights' end values and mirror symmetry, the
Neumann fit of even data, and convergence of the spectral derivative of the
paper's example function.
"""
from __future__ import annotations

from dataclasses import dataclass
from fractions import Fraction

import numpy as np


def _solve(A, b):
    """Exact Gaussian elimination (A square, nonsingular, Fractions)."""
    n = len(A)
    M = [list(A[i]) + [b[i]] for i in range(n)]
    for c in range(n):
        piv = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[piv] = M[piv], M[c]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c] / M[c][c]
                M[r] = [x - f * y for x, y in zip(M[r], M[c])]
    return [M[i][n] / M[i][i] for i in range(n)]


def sigma(t: Fraction) -> Fraction:
    """Blending polynomial of eq. sigma."""
    return 10 * t ** 3 - 15 * t ** 4 + 6 * t ** 5


def solution_operator(d: int, p: int, neumann: bool):
    """(p+1) x d matrix P with c = P f the least-squares monomial coefficients
    (c[m] multiplies xi^m) of the fit to the values f at xi = -(d-1) .. 0."""
    xs = [Fraction(j - (d - 1)) for j in range(d)]
    rows = [[x ** m for m in range(p + 1)] for x in xs]
    if neumann:
        rows.append([Fraction(1) if m == 1 else Fraction(0) for m in range(p + 1)])
    nr = len(rows)
    VtV = [[sum(rows[i][a] * rows[i][b] for i in range(nr)) for b in range(p + 1)] for a in range(p + 1)]
    P = [[Fraction(0)] * d for _ in range(p + 1)]
    for j in range(d):                       # column j: data e_j (the Neumann row's RHS is 0)
        rhs = [rows[j][a] for a in range(p + 1)]
        c = _solve(VtV, rhs)
        for m in range(p + 1):
            P[m][j] = c[m]
    return P


def continuation_map(d: int, p: int, C: int, neumann: bool) -> np.ndarray:
    P = solution_operator(d, p, neumann)
    M = np.zeros((C, d))
    for r in range(1, C + 1):
        w = 1 - sigma(Fraction(r - 1, C - 1))
        for j in range(d):
            M[r - 1, j] = float(w * sum(Fraction(r) ** m * P[m][j] for m in range(p + 1)))
    return M


@dataclass
class PolyBlendTables:
    params: dict
    M_D: np.ndarray          # C x d
    M_N: np.ndarray          # C x d

    def M(self, bc: str) -> np.ndarray:
        return {"D": self.M_D, "N": self.M_N}[bc]


def build(d: int = 10, p: int = 5, C: int = 16) -> PolyBlendTables:
    """Maps for d fit points, degree p, C continuation points (C >= 2)."""
    if not (p + 1 <= d and C >= 2):
        raise ValueError("need p + 1 <= d and C >= 2")
    return PolyBlendTables(dict(d=d, p=p, C=C), continuation_map(d, p, C, False),
                           continuation_map(d, p, C, True))
